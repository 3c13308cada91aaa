// Global step of projective dynamics as one dense GEMM per mesh class:
//   C[:, n] = Ainv * B[:, n]   for all 3 * cells columns n,
// with the constant, symmetric inverse of the class system matrix shared by
// every cell (prefactored once in FP64). Columns are stored contiguously
// ([ncols][Npad], rows >= N are zero), so the operand tiles are plain strided
// loads; Ainv is symmetric, so its row k serves as column k.
//
// FP32 and FP64 use the 16x16x4 MFMA instructions; BF16/FP16 use 16x16x32
// with FP32 accumulation and store the operator in the split form
//   Ainv = (h^2/m)(I + beta * Bt),  |Bt| <= 1,
// so that only the small correction Bt * r passes through the 8/11-bit
// mantissa and the identity part stays exact in FP32 (epilogue).
//
// Tiling: 256 threads = 4 waves in a 2x2 grid, each wave owns a
// (BM/2) x (BN/2) block of 16x16 accumulators; K advances BK rows at a time
// through double-buffered LDS tiles with register prefetch.
#include <algorithm>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "npfem_internal.h"

namespace npfem {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

template <typename T>
struct Mfma4;
template <>
struct Mfma4<float> {
  typedef floatx4 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // result register r of lane l holds row 4*(l/16) + r of column l%16
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct Mfma4<double> {
  typedef doublex4 acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // result register r of lane l holds row l/16 + 4*r of column l%16
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Row pads chosen so that the 4 k-rows read by one MFMA operand fetch land
// 16 banks apart.
__host__ __device__ constexpr int lds_pad(int w) { return ((16 - w) % 64 + 64) % 64; }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). Remap the linear id so that every XCD receives a contiguous range of
// tiles, row tiles fastest: the row tiles of one column strip then share an
// L2 and read the strip from HBM once.
__device__ __forceinline__ void xcd_tile(int& mt, int& nt) {
  const int nbx = gridDim.x, total = gridDim.x * gridDim.y;
  const int id = blockIdx.x + blockIdx.y * nbx;
  const int xcd = id & 7, slot = id >> 3;
  const int per = total >> 3, rem = total & 7;
  const int logical = xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  mt = logical % nbx;
  nt = logical / nbx;
}

// Accumulating (correction) products of FP32/FP64 columns may come with
// per-column maxima of the input (GemmArgs::colscale): a zero marks a column
// that needs no correction, which is then neither computed into nor stored.
__device__ __forceinline__ bool col_dead(const GemmArgs& g, int n) {
  return g.mode == EPI_ADD && g.colscale && g.colscale[n] == 0.0f;
}

// ---------------------------------------------------------------- FP32/FP64
template <typename T, int BM, int BN>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 ? 3 : 1)) gemm_kernel(GemmArgs g) {
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int VE = 16 / sizeof(T);  // elements per 16-byte vector
  constexpr int APAD = lds_pad(BM), BPAD = lds_pad(BN);
  constexpr int AV = BK * BM / VE, BV = BN * BK / VE;  // 16-byte vectors per tile
  constexpr int NA = (AV + 255) / 256, NB = (BV + 255) / 256;  // per thread
  static_assert(BM % 32 == 0 && BN % 32 == 0, "2x2 waves of 16x16 blocks");
  typedef typename Mfma4<T>::acc_t acc_t;
  struct alignas(16) Vec { T v[VE]; };

  __shared__ T As[2][BK][BM + APAD];
  __shared__ T Bs[2][BK][BN + BPAD];

  const T* __restrict__ A = static_cast<const T*>(g.A);
  const T* __restrict__ B = static_cast<const T*>(g.B);
  T* __restrict__ C = static_cast<T*>(g.C);
  const int Npad = g.Npad, ncols = g.ncols;
  int mt, nt;
  xcd_tile(mt, nt);
  const int m0 = mt * BM, n0 = nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  if (g.mode == EPI_ADD && g.colscale) {  // a tile with no live column returns
    bool live = false;
    for (int j = tid; j < BN; j += 256) live = live || (n0 + j < ncols && !col_dead(g, n0 + j));
    if (!__syncthreads_or(live)) return;
  }

  Vec ra[NA], rb[NB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + i * 256;
      const int kk = idx / (BM / VE), mv = idx % (BM / VE);
      const int m = m0 + mv * VE;
      if (idx < AV && m < Npad) {
        ra[i] = *reinterpret_cast<const Vec*>(A + (size_t)(k0 + kk) * Npad + m);
      } else {
#pragma unroll
        for (int e = 0; e < VE; ++e) ra[i].v[e] = T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + i * 256;
      const int kv = idx % (BK / VE), nn = idx / (BK / VE);
      const int n = n0 + nn;
      if (idx < BV && n < ncols) {
        rb[i] = *reinterpret_cast<const Vec*>(B + (size_t)n * Npad + k0 + kv * VE);
      } else {
#pragma unroll
        for (int e = 0; e < VE; ++e) rb[i].v[e] = T(0);
      }
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + i * 256;
      const int kk = idx / (BM / VE), mv = idx % (BM / VE);
      if (idx < AV) *reinterpret_cast<Vec*>(&As[buf][kk][mv * VE]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + i * 256;
      const int kv = idx % (BK / VE), nn = idx / (BK / VE);
      if (idx < BV) {
#pragma unroll
        for (int e = 0; e < VE; ++e) Bs[buf][kv * VE + e][nn] = rb[i].v[e];
      }
    }
  };

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = T(0);

  const int nk = Npad / BK;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      T af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = As[cur][kr][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = Bs[cur][kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mfma4<T>::run(af[i], bf[j], acc[i][j]);
    }
    if (kt + 1 < nk) {
      store_tiles(cur ^ 1);
      __syncthreads();
    }
  }

  // epilogue: each 16x16 block lies inside [0, Npad) or wholly outside it;
  // C = D + product (D = C when accumulating, none if null)
  const T* Dadd = g.mode == EPI_ADD ? C : static_cast<const T*>(g.D);
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int mb = m0 + wm * WM + i * 16;
    if (mb >= Npad) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + wn * WN + j * 16 + (lane & 15);
      if (n >= ncols || col_dead(g, n)) continue;
      T* c = C + (size_t)n * Npad + mb;
      if (Dadd) {
        const T* d = Dadd + (size_t)n * Npad + mb;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          c[Mfma4<T>::row(lane, r)] = d[Mfma4<T>::row(lane, r)] + acc[i][j][r];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) c[Mfma4<T>::row(lane, r)] = acc[i][j][r];
      }
    }
  }
}

// ---------------------------------------------------------------- BF16/FP16
template <typename L>
struct Mfma32;
template <>
struct Mfma32<__bf16> {
  typedef bf16x8 vec_t;
  static __device__ __forceinline__ floatx4 run(vec_t a, vec_t b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma32<_Float16> {
  typedef halfx8 vec_t;
  static __device__ __forceinline__ floatx4 run(vec_t a, vec_t b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Power-of-two scale of column n from its max |.| (1 without maxima). In the
// accumulating mode a zero maximum marks a column that needs no correction
// (the residual step found its error below the state's rounding): scale 0,
// and the column is neither read nor written.
__device__ __forceinline__ float lp_col_scale(const GemmArgs& g, int n) {
  if (!g.colscale || n >= g.ncols) return 1.0f;
  const float mx = g.colscale[n];
  if (mx > 0.0f && isfinite(mx)) return exp2f(-ceilf(log2f(mx)));
  return (g.mode == EPI_SPLIT_ADD && mx == 0.0f) ? 0.0f : 1.0f;
}

// C = hm * (B + beta * Bt * B)   (SPLIT_SET) or C += that (SPLIT_ADD).
// B columns are FP32 in memory; each column is multiplied by a power of two
// (from its max |.|) before rounding to the 16-bit type, and divided back in
// the epilogue.
template <typename L, int BM, int BN>
__global__ void __launch_bounds__(256) gemm_lp_kernel(GemmArgs g) {
  constexpr int BK = 32;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int KP = BK + 8;  // LDS row stride (elements): 80 bytes
  constexpr int AV = BM * BK / 8, BV = BN * BK / 8;  // 8-element vectors per tile
  constexpr int NA = (AV + 255) / 256, NB = (BV + 255) / 256;
  static_assert(BM % 32 == 0 && BN % 32 == 0, "2x2 waves of 16x16 blocks");
  typedef typename Mfma32<L>::vec_t vec_t;

  __shared__ L As[2][BM][KP];
  __shared__ L Bs[2][BN][KP];
  __shared__ float sc_in[BN];

  const L* __restrict__ A = static_cast<const L*>(g.A);
  const float* __restrict__ B = static_cast<const float*>(g.B);
  float* __restrict__ C = static_cast<float*>(g.C);
  const int Npad = g.Npad, ncols = g.ncols;
  int mt, nt;
  xcd_tile(mt, nt);
  const int m0 = mt * BM, n0 = nt * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  bool live = false;
  for (int j = tid; j < BN; j += 256) {
    const float s = lp_col_scale(g, n0 + j);
    sc_in[j] = s;
    live = live || (s != 0.0f && n0 + j < ncols);
  }
  if (!__syncthreads_or(live)) return;  // no column of the tile needs work

  vec_t ra[NA], rb[NB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + i * 256;
      const int mm = idx / (BK / 8), kv = idx % (BK / 8);
      const int m = m0 + mm, k = k0 + kv * 8;
      if (idx < AV && m < Npad && k < Npad) {
        ra[i] = *reinterpret_cast<const vec_t*>(A + (size_t)m * Npad + k);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[i][e] = L(0.0f);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + i * 256;
      const int nn = idx / (BK / 8), kv = idx % (BK / 8);
      const int n = n0 + nn, k = k0 + kv * 8;
      if (idx < BV && n < ncols && k < Npad) {
        const float4 lo = *reinterpret_cast<const float4*>(B + (size_t)n * Npad + k);
        const float4 hi = *reinterpret_cast<const float4*>(B + (size_t)n * Npad + k + 4);
        const float s = sc_in[nn];
        rb[i][0] = L(lo.x * s);
        rb[i][1] = L(lo.y * s);
        rb[i][2] = L(lo.z * s);
        rb[i][3] = L(lo.w * s);
        rb[i][4] = L(hi.x * s);
        rb[i][5] = L(hi.y * s);
        rb[i][6] = L(hi.z * s);
        rb[i][7] = L(hi.w * s);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) rb[i][e] = L(0.0f);
      }
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = tid + i * 256;
      const int mm = idx / (BK / 8), kv = idx % (BK / 8);
      if (idx < AV) *reinterpret_cast<vec_t*>(&As[buf][mm][kv * 8]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + i * 256;
      const int nn = idx / (BK / 8), kv = idx % (BK / 8);
      if (idx < BV) *reinterpret_cast<vec_t*>(&Bs[buf][nn][kv * 8]) = rb[i];
    }
  };

  floatx4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nk = (Npad + BK - 1) / BK;
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * BK);
    const int kq = (lane >> 4) * 8;
    vec_t af[TM], bf[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
      af[i] = *reinterpret_cast<const vec_t*>(&As[cur][wm * WM + i * 16 + (lane & 15)][kq]);
#pragma unroll
    for (int j = 0; j < TN; ++j)
      bf[j] = *reinterpret_cast<const vec_t*>(&Bs[cur][wn * WN + j * 16 + (lane & 15)][kq]);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = Mfma32<L>::run(af[i], bf[j], acc[i][j]);
    if (kt + 1 < nk) {
      store_tiles(cur ^ 1);
      __syncthreads();
    }
  }

  const float hm = (float)g.hm, beta = (float)g.beta;
  const float* Dadd = g.mode == EPI_SPLIT_ADD ? C : static_cast<const float*>(g.D);
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int m = m0 + wm * WM + i * 16 + (lane >> 4) * 4;
    if (m >= Npad) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int nn = wn * WN + j * 16 + (lane & 15);
      const int n = n0 + nn;
      if (n >= ncols || sc_in[nn] == 0.0f) continue;
      const float unscale = beta / sc_in[nn];
      const float* bcol = B + (size_t)n * Npad + m;
      float* c = C + (size_t)n * Npad + m;
      if (Dadd) {
        const float* d = Dadd + (size_t)n * Npad + m;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = d[r] + hm * (bcol[r] + unscale * acc[i][j][r]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = hm * (bcol[r] + unscale * acc[i][j][r]);
      }
    }
  }
}

// ------------------------------------------------------- column-stationary
// The global step is a tall-skinny product: one Npad x Npad operator against
// thousands of columns. Here one workgroup owns RS_NG * 16 consecutive
// columns (16 cells' three coordinates for RS_NG = 3) for the whole product
// and keeps them in LDS; the operator, which every workgroup needs whole,
// streams from L2 (1.7 MB in FP32, 0.9 MB in 16 bits: every XCD's L2 holds
// it) in 16-row blocks straight into MFMA operand registers, ahead of its use.
// 12288 columns make 256 workgroups, one per CU, so there is no tile
// quantisation; the four waves split the row blocks, and the row blocks left
// over after an even split are split by column group. With fewer column
// blocks than CUs (FP32, small batches) the row blocks are further split over
// up to four workgroups per column block (gridDim.y), each staging the whole
// column block, so that the product still spreads over the chip (while every
// part keeps at least one row pair per wave).
//
// LDS layout: k-chunks of 4 (FP32) or 8 (16-bit) values of each column are
// contiguous 16-byte records, chunk-major: record (q, n) at q * RS_BN + n.
// The 16 lanes of an MFMA operand fetch read 16 consecutive records (256
// contiguous bytes), so a wave's fetch touches every bank once per 256 bytes.
constexpr int RS_NG = 3;
constexpr int RS_BN = RS_NG * 16;
constexpr int kNumTilesTiled = 14;  // tile ids below are tiled shapes, this one column-stationary

__host__ __device__ inline int rs_k32(int npad) { return (npad + 31) / 32 * 32; }

// Rows [16 rb, 16 (rb + NR)) of column groups [g0, g0 + NGU) (FP32). Lane l
// feeds the MFMA k-index l/16 with k = k0 + 4 (l/16) + j at sub-step j, for A
// and B alike, so one 16-byte load covers four sub-steps; every B fragment
// read from LDS serves NR row blocks. With a single row block and column
// group the four sub-steps accumulate separately (independent MFMA chains)
// and are summed at the end. NIT >= 0: the main loop's trip count,
// Npad / 16 / 8, fixed at compile time, so that it unrolls completely (with
// a loop, the accumulators were rotated through extra registers at every
// back edge); -1: read from Npad.
template <int NR, int NGU, int NIT = -1>
__device__ __forceinline__ void rs_rows_f32(const float* __restrict__ A, const float* Bs, int Npad,
                                            int rb, int g0, float* __restrict__ C, int n0,
                                            int ncols, const float* Dadd, const GemmArgs& g,
                                            int lane) {
  constexpr int NJ = (NR * NGU == 1) ? 4 : 1;
  constexpr int D = 4;  // prefetch distance in 16-k groups
  floatx4 acc[NR][NGU][NJ];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int u = 0; u < NGU; ++u)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[r][u][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // operator in fragment order: the 4 values of lane l for row block rb and
  // 16-k group kg at ((rb * nkg + kg) * 64 + l) * 4 (1 KB per wave load)
  const int nkg = Npad / 16;
  const float* arow[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) arow[r] = A + ((size_t)(rb + r) * nkg * 64 + lane) * 4;
  // record (4 kg + lane/16, g * 16 + lane%16) for k-group kg
  const float* bcol[NGU];
#pragma unroll
  for (int u = 0; u < NGU; ++u) bcol[u] = Bs + 4 * ((lane >> 4) * RS_BN + (g0 + u) * 16 + (lane & 15));
  // Straight-line prefetch: out-of-range prefetches re-read the last group
  // (clamped address, value unused), so the loop body has no branches and the
  // compiler can wait for exactly the load it needs.
  auto load_a = [&](int r, int kg) {
    return *reinterpret_cast<const float4*>(arow[r] + 256 * min(kg, nkg - 1));
  };
  auto step = [&](int kg, const float4 (&a)[NR]) {
    float4 b[NGU];
#pragma unroll
    for (int u = 0; u < NGU; ++u) b[u] = *reinterpret_cast<const float4*>(bcol[u] + 16 * RS_BN * kg);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int u = 0; u < NGU; ++u)
        acc[r][u][0 % NJ] = Mfma4<float>::run(a[r].x, b[u].x, acc[r][u][0 % NJ]);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int u = 0; u < NGU; ++u)
        acc[r][u][1 % NJ] = Mfma4<float>::run(a[r].y, b[u].y, acc[r][u][1 % NJ]);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int u = 0; u < NGU; ++u)
        acc[r][u][2 % NJ] = Mfma4<float>::run(a[r].z, b[u].z, acc[r][u][2 % NJ]);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int u = 0; u < NGU; ++u)
        acc[r][u][3 % NJ] = Mfma4<float>::run(a[r].w, b[u].w, acc[r][u][3 % NJ]);
  };
  // two register sets that alternate: the loads for the next D groups go
  // into one (issued, and kept ahead of the scheduler, before) while the
  // other's D groups are multiplied; nothing is copied between them
  float4 a0[D][NR], a1[D][NR];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int r = 0; r < NR; ++r) a0[i][r] = load_a(r, i);
  // the addend of the rows this lane stores, requested after the first
  // operator groups (so that their wait does not include it) and long before
  // the epilogue (clamped column index: columns past the last are never stored)
  float4 dv[NR][NGU];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int u = 0; u < NGU; ++u) {
      const int n = min(n0 + (g0 + u) * 16 + (lane & 15), ncols - 1);
      dv[r][u] = Dadd ? *reinterpret_cast<const float4*>(Dadd + (size_t)n * Npad + (rb + r) * 16 +
                                                         4 * (lane >> 4))
                      : float4{0.f, 0.f, 0.f, 0.f};
    }
  auto load_set = [&](float4(&dst)[D][NR], int kg0) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int r = 0; r < NR; ++r) dst[i][r] = load_a(r, kg0 + i);
  };
  int kg = 0;
  auto two_sets = [&](int k0) {
    load_set(a1, k0 + D);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < D; ++i) step(k0 + i, a0[i]);
    load_set(a0, k0 + 2 * D);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < D; ++i) step(k0 + D + i, a1[i]);
  };
  if constexpr (NIT >= 0) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) two_sets(2 * D * it);
    kg = 2 * D * NIT;
  } else {
    for (; kg + 2 * D <= nkg; kg += 2 * D) two_sets(kg);
  }
  // fewer than 2D groups left, the first D of them (clamped) in a0
  if (kg + D < nkg) {
    load_set(a1, kg + D);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < D; ++i) step(kg + i, a0[i]);
#pragma unroll
    for (int i = 0; i < D; ++i)
      if (kg + D + i < nkg) step(kg + D + i, a1[i]);
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i)
      if (kg + i < nkg) step(kg + i, a0[i]);
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int u = 0; u < NGU; ++u) {
#pragma unroll
      for (int j = 1; j < NJ; ++j) acc[r][u][0] += acc[r][u][j];
      const int n = n0 + (g0 + u) * 16 + (lane & 15);
      if (n >= ncols || col_dead(g, n)) continue;
      float4* c =
          reinterpret_cast<float4*>(C + (size_t)n * Npad + (rb + r) * 16 + 4 * (lane >> 4));
      const float4 v{acc[r][u][0][0], acc[r][u][0][1], acc[r][u][0][2], acc[r][u][0][3]};
      if (Dadd) {
        float4 o = dv[r][u];
        o.x += v.x;
        o.y += v.y;
        o.z += v.z;
        o.w += v.w;
        *c = o;
      } else {
        *c = v;
      }
    }
  }
}

__global__ void __launch_bounds__(256) gemm_rs_f32_kernel(GemmArgs g) {
  extern __shared__ float rs_lds[];
  const float* __restrict__ A = static_cast<const float*>(g.A_frag);
  const float* __restrict__ B = static_cast<const float*>(g.B);
  float* __restrict__ C = static_cast<float*>(g.C);
  const int Npad = g.Npad, ncols = g.ncols;
  const int n0 = blockIdx.x * RS_BN;
  const int tid = threadIdx.x;
  if (g.mode == EPI_ADD && g.colscale) {  // no live column: nothing to do
    bool live = false;
    for (int j = tid; j < RS_BN; j += 256) live = live || (n0 + j < ncols && !col_dead(g, n0 + j));
    if (!__syncthreads_or(live)) return;
  }
  // staging, column index fastest (consecutive threads write consecutive
  // records); 8 loads per thread in flight at a time (clamped addresses,
  // values outside the matrix replaced by zeros, no branches)
  const int total = RS_BN * (Npad / 4);
  for (int i0 = tid; i0 < total; i0 += 256 * 8) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = min(i0 + 256 * u, total - 1);
      const int q = i / RS_BN, n = i - q * RS_BN;
      v[u] = *reinterpret_cast<const float4*>(B + (size_t)min(n0 + n, ncols - 1) * Npad + 4 * q);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + 256 * u;
      if (i < total) {
        const int n = i % RS_BN;
        if (n0 + n >= ncols) v[u] = float4{0.f, 0.f, 0.f, 0.f};
        *reinterpret_cast<float4*>(rs_lds + 4 * i) = v[u];
      }
    }
  }
  __syncthreads();
  // row blocks in pairs, the pairs split evenly over the four waves; the
  // remaining row blocks one column group at a time. Every workgroup needs
  // the whole operator: workgroups on one XCD (consecutive ones sit on
  // different XCDs) start at different row pairs, so that their concurrent
  // requests spread over the L2 channels instead of queueing on the same
  // lines.
  const int wave = tid >> 6, lane = tid & 63;
  const int nrb = Npad / 16, full = nrb & ~7;
  const int rot = full > 0 ? 2 * ((blockIdx.x / 8) % (full / 2)) : 0;
  // C = D + product (D = C when accumulating, none if null)
  const float* Dadd = g.mode == EPI_ADD ? C : static_cast<const float*>(g.D);
  // rows split over gridDim.y workgroups per column block (few columns):
  // part s takes the row pairs and leftover units s, s + parts, ...
  const int s = blockIdx.y, parts = gridDim.y;
  auto pairs = [&](auto nit) {
    for (int p = s + parts * wave; 2 * p < full; p += 4 * parts) {
      const int i = 2 * p;
      const int rb = i + rot < full ? i + rot : i + rot - full;
      rs_rows_f32<2, RS_NG, decltype(nit)::value>(A, rs_lds, Npad, rb, 0, C, n0, ncols, Dadd, g,
                                                  lane);
    }
  };
  switch (nrb / 8) {  // main-loop trip count of rs_rows_f32
    case 1: pairs(std::integral_constant<int, 1>{}); break;
    case 2: pairs(std::integral_constant<int, 2>{}); break;
    case 3: pairs(std::integral_constant<int, 3>{}); break;
    case 4: pairs(std::integral_constant<int, 4>{}); break;
    case 5: pairs(std::integral_constant<int, 5>{}); break;
    case 6: pairs(std::integral_constant<int, 6>{}); break;
    default: pairs(std::integral_constant<int, -1>{}); break;
  }
  for (int u = s + parts * wave; u < (nrb - full) * RS_NG; u += 4 * parts)
    rs_rows_f32<1, 1>(A, rs_lds, Npad, full + u / RS_NG, u % RS_NG, C, n0, ncols, Dadd, g,
                      lane);
}

// 16-bit version: the split operator Bt (16-bit, [Npad][Npad]) against the
// columns converted once into LDS (each scaled by a power of two as in the
// tiled kernel), k-steps of 32 (16x16x32 MFMA). The number of k-steps NKS is
// a template parameter (Npad rounded up to 32, then to a multiple of
// RS_KS_STEP k-steps), so that a row block's multiply is one straight-line
// block: the accumulators stay in place and the LDS reads run ahead of the
// MFMAs. k at or beyond Npad: the LDS records hold zeros, and the operator
// values there (read from a clamped, in-row address) multiply those zeros.
// A wave holds a whole 16-row block of the operator in registers and
// fetches the next one into a second register image while it multiplies
// (the two images alternate, nothing is copied). The epilogue applies
// C = D + hm (B + beta / s_n Bt B) (D = C when accumulating) with B re-read
// in FP32; those loads, and the loads of D, are issued before
// the next row block's operator loads so that the epilogue waits for them
// alone.
constexpr int RS_KS_STEP = 3;
constexpr int RS_KS_MAX = 24;  // Npad <= 768

__host__ __device__ inline int rs_nks(int npad) {
  const int k = rs_k32(npad) / 32;
  return (k + RS_KS_STEP - 1) / RS_KS_STEP * RS_KS_STEP;
}

size_t rs_lds_bytes(int kind, int npad) {
  if (kind == 0) return sizeof(float) * RS_BN * (size_t)npad;
  if (kind >= 2) {
    if (rs_nks(npad) > RS_KS_MAX) return 0;
    return 2 * RS_BN * 32 * (size_t)rs_nks(npad) + sizeof(float) * RS_BN;
  }
  return 0;
}

template <typename L, int NKS, int NGU>
struct RsLpRows {
  typedef typename Mfma32<L>::vec_t vec_t;
  // epilogue inputs of one row block and NGU column groups
  struct Epi {
    float4 b[NGU];
    float4 c[NGU];
  };
  // register image of one row block: k-step ks of lane l covers
  // k = 32 ks + 8 (l/16) .. + 7 of row 16 rb + l%16, read from the fragment
  // copy (one wave's k-step is 1 KB of consecutive memory)
  static __device__ __forceinline__ void load(const L* __restrict__ Af, int Npad, int rb, int lane,
                                              vec_t (&dst)[NKS]) {
    const L* __restrict__ src = Af + ((size_t)rb * NKS * 64 + lane) * 8;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) dst[ks] = *reinterpret_cast<const vec_t*>(src + 512 * ks);
  }
  // lane l holds rows 16 rb + 4 (l/16) .. + 3 of column group g0 + u, column
  // l%16 (clamped column index: columns past the last are never stored)
  static __device__ __forceinline__ void load_epi(const float* __restrict__ B,
                                                  const float* __restrict__ D, int Npad, int rb,
                                                  int g0, int n0, int ncols, bool add, int lane,
                                                  Epi& e) {
    const int m_ep = rb * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int u = 0; u < NGU; ++u) {
      const int n = min(n0 + (g0 + u) * 16 + (lane & 15), ncols - 1);
      e.b[u] = *reinterpret_cast<const float4*>(B + (size_t)n * Npad + m_ep);
      e.c[u] = add ? *reinterpret_cast<const float4*>(D + (size_t)n * Npad + m_ep)
                   : float4{0.f, 0.f, 0.f, 0.f};
    }
  }
  static __device__ __forceinline__ void run(const vec_t (&a)[NKS], const L* Bs, int Npad, int rb,
                                             int g0, float* __restrict__ C, const float* sc,
                                             int n0, int ncols, float hm, float beta, bool add,
                                             int lane, const Epi& e) {
    // independent accumulation chains when a single column group is done
    constexpr int NJ = NGU == 1 ? RS_KS_STEP : 1;
    floatx4 acc[NGU][NJ];
#pragma unroll
    for (int u = 0; u < NGU; ++u)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[u][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const L* bcol = Bs + 8 * ((lane >> 4) * RS_BN + g0 * 16 + (lane & 15));
    // LDS fragments PF k-steps ahead of their MFMAs (scheduling barriers keep
    // the compiler from folding the reads back next to their use)
    constexpr int PF = 2;
    vec_t bq[PF + 1][NGU];
    auto read_b = [&](int ks) {
#pragma unroll
      for (int u = 0; u < NGU; ++u)
        bq[ks % (PF + 1)][u] = *reinterpret_cast<const vec_t*>(bcol + 8 * (4 * RS_BN * ks + 16 * u));
    };
#pragma unroll
    for (int ks = 0; ks < PF && ks < NKS; ++ks) read_b(ks);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      if (ks + PF < NKS) read_b(ks + PF);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < NGU; ++u)
        acc[u][ks % NJ] = Mfma32<L>::run(a[ks], bq[ks % (PF + 1)][u], acc[u][ks % NJ]);
      __builtin_amdgcn_sched_barrier(0);
    }
    const int m_ep = rb * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int u = 0; u < NGU; ++u) {
#pragma unroll
      for (int j = 1; j < NJ; ++j) acc[u][0] += acc[u][j];
      const int nl = (g0 + u) * 16 + (lane & 15);
      const int n = n0 + nl;
      if (n >= ncols || sc[nl] == 0.0f) continue;
      const float unscale = beta / sc[nl];
      float4 v;
      v.x = hm * (e.b[u].x + unscale * acc[u][0][0]);
      v.y = hm * (e.b[u].y + unscale * acc[u][0][1]);
      v.z = hm * (e.b[u].z + unscale * acc[u][0][2]);
      v.w = hm * (e.b[u].w + unscale * acc[u][0][3]);
      if (add) {
        v.x += e.c[u].x;
        v.y += e.c[u].y;
        v.z += e.c[u].z;
        v.w += e.c[u].w;
      }
      *reinterpret_cast<float4*>(C + (size_t)n * Npad + m_ep) = v;
    }
  }
};

template <typename L, int NKS>
__global__ void __launch_bounds__(256) gemm_rs_lp_kernel(GemmArgs g) {
  typedef RsLpRows<L, NKS, RS_NG> Rows;
  typedef RsLpRows<L, NKS, 1> Rows1;
  typedef typename Mfma32<L>::vec_t vec_t;
  extern __shared__ float rs_lds_lp[];
  const L* __restrict__ A = static_cast<const L*>(g.A_frag);
  const float* __restrict__ B = static_cast<const float*>(g.B);
  float* __restrict__ C = static_cast<float*>(g.C);
  const int Npad = g.Npad, ncols = g.ncols;
  const int n0 = blockIdx.x * RS_BN;
  const int tid = threadIdx.x;
  float* sc = rs_lds_lp;                               // [RS_BN] column scales
  L* Bs = reinterpret_cast<L*>(rs_lds_lp + RS_BN);     // records (q, n), 8 values each
  bool live = false;
  for (int j = tid; j < RS_BN; j += 256) {
    const float s = lp_col_scale(g, n0 + j);
    sc[j] = s;
    live = live || (s != 0.0f && n0 + j < ncols);
  }
  if (!__syncthreads_or(live)) return;  // no column of the workgroup needs work
  // staging, column index fastest; 8 vector pairs per thread in flight at a
  // time (clamped addresses, values outside the matrix replaced by zeros)
  const int total = RS_BN * (4 * NKS);
  for (int i0 = tid; i0 < total; i0 += 256 * 8) {
    float4 lo[8], hi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = min(i0 + 256 * u, total - 1);
      const int q = i / RS_BN, n = i - q * RS_BN;
      const float* src = B + (size_t)min(n0 + n, ncols - 1) * Npad + min(8 * q, Npad - 8);
      lo[u] = *reinterpret_cast<const float4*>(src);
      hi[u] = *reinterpret_cast<const float4*>(src + 4);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + 256 * u;
      if (i < total) {
        const int q = i / RS_BN, n = i - q * RS_BN;
        const bool in = n0 + n < ncols && 8 * q < Npad;
        const float s = in ? sc[n] : 0.0f;
        vec_t v;
        v[0] = L(lo[u].x * s);
        v[1] = L(lo[u].y * s);
        v[2] = L(lo[u].z * s);
        v[3] = L(lo[u].w * s);
        v[4] = L(hi[u].x * s);
        v[5] = L(hi[u].y * s);
        v[6] = L(hi[u].z * s);
        v[7] = L(hi[u].w * s);
        *reinterpret_cast<vec_t*>(Bs + 8 * i) = v;
      }
    }
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int nrb = Npad / 16, full = nrb & ~3;
  const float hm = (float)g.hm, beta = (float)g.beta;
  // C = D + product (D = C when accumulating, none if null)
  const float* Dadd = g.mode == EPI_SPLIT_ADD ? C : static_cast<const float*>(g.D);
  const bool add = Dadd != nullptr;
  // full row blocks, four per round (one per wave); the starting row block
  // rotates with the workgroup as in the FP32 kernel
  {
    const int rot = full > 0 ? (blockIdx.x / 8) % full : 0;
    auto phys = [&](int i) { return i + rot < full ? i + rot : i + rot - full; };
    vec_t a0[NKS], a1[NKS];
    // the epilogue inputs (HBM) of a row block are requested one row block
    // earlier than its operator image, two row blocks before their use
    typename Rows::Epi e0, e1;
    if (wave < full) {
      Rows::load_epi(B, Dadd, Npad, phys(wave), 0, n0, ncols, add, lane, e0);
      Rows::load(A, Npad, phys(wave), lane, a0);
    }
    if (wave + 4 < full) Rows::load_epi(B, Dadd, Npad, phys(wave + 4), 0, n0, ncols, add, lane, e1);
    for (int i = wave; i < full; i += 8) {
      if (i + 4 < full) Rows::load(A, Npad, phys(i + 4), lane, a1);
      __builtin_amdgcn_sched_barrier(0);
      Rows::run(a0, Bs, Npad, phys(i), 0, C, sc, n0, ncols, hm, beta, add, lane, e0);
      if (i + 4 >= full) break;
      if (i + 8 < full) Rows::load_epi(B, Dadd, Npad, phys(i + 8), 0, n0, ncols, add, lane, e0);
      if (i + 8 < full) Rows::load(A, Npad, phys(i + 8), lane, a0);
      __builtin_amdgcn_sched_barrier(0);
      Rows::run(a1, Bs, Npad, phys(i + 4), 0, C, sc, n0, ncols, hm, beta, add, lane, e1);
      if (i + 12 < full) Rows::load_epi(B, Dadd, Npad, phys(i + 12), 0, n0, ncols, add, lane, e1);
    }
  }
  // the remaining row blocks one column group at a time
  for (int u = wave; u < (nrb - full) * RS_NG; u += 4) {
    const int rb = full + u / RS_NG, g0 = u % RS_NG;
    vec_t a[NKS];
    typename Rows1::Epi e;
    Rows1::load_epi(B, Dadd, Npad, rb, g0, n0, ncols, add, lane, e);
    Rows1::load(A, Npad, rb, lane, a);
    Rows1::run(a, Bs, Npad, rb, g0, C, sc, n0, ncols, hm, beta, add, lane, e);
  }
}

template <typename L>
static const void* rs_lp_kernel(int nks) {
  switch (nks) {
    case 3: return (const void*)gemm_rs_lp_kernel<L, 3>;
    case 6: return (const void*)gemm_rs_lp_kernel<L, 6>;
    case 9: return (const void*)gemm_rs_lp_kernel<L, 9>;
    case 12: return (const void*)gemm_rs_lp_kernel<L, 12>;
    case 15: return (const void*)gemm_rs_lp_kernel<L, 15>;
    case 18: return (const void*)gemm_rs_lp_kernel<L, 18>;
    case 21: return (const void*)gemm_rs_lp_kernel<L, 21>;
    case 24: return (const void*)gemm_rs_lp_kernel<L, 24>;
    default: return nullptr;
  }
}

static const void* rs_kernel(int kind, int npad) {
  return kind == 0 ? (const void*)gemm_rs_f32_kernel
       : kind == 2 ? rs_lp_kernel<__bf16>(rs_nks(npad))
       : kind == 3 ? rs_lp_kernel<_Float16>(rs_nks(npad))
                   : nullptr;
}

// Raises the dynamic-LDS limit of the column-stationary kernel to what a
// class of Npad rows needs (not a stream operation: call before capture).
hipError_t gemm_prepare(int kind, int tile, int npad) {
  if (tile != kNumTilesTiled) return hipSuccess;
  const size_t smem = rs_lds_bytes(kind, npad);
  const void* fn = rs_kernel(kind, npad);
  if (!fn || smem == 0 || smem > 160 * 1024) return hipErrorInvalidValue;
  if (smem <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
}

// Compute units of the current device (queried once per device).
static int device_cu_count() {
  static int cached[16] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

static hipError_t run_gemm_rs(int kind, const GemmArgs& g, hipStream_t st) {
  const size_t smem = rs_lds_bytes(kind, g.Npad);
  const void* fn = rs_kernel(kind, g.Npad);
  if (!fn || smem == 0 || smem > 160 * 1024) return hipErrorInvalidValue;
  if (kind != 1 && !g.A_frag) return hipErrorInvalidValue;
  GemmArgs a = g;
  void* args[] = {&a};
  const int blocks = (g.ncols + RS_NG * 16 - 1) / (RS_NG * 16);
  // FP32 with fewer column blocks than CUs: the rows are split over up to
  // four workgroups per column block (each stages the whole column block),
  // as long as every part keeps a row pair per wave
  int parts = 1;
  if (kind == 0) {
    const int cus = device_cu_count();
    const int pairs = (g.Npad / 16 & ~7) / 2;
    parts = std::max(1, std::min({4, cus / std::max(blocks, 1), pairs / 4}));
  }
  return hipLaunchKernel(fn, dim3(blocks, parts), dim3(256), args, smem, st);
}

// ---------------------------------------------------------------- dispatch
struct TileShape {
  int bm, bn;
};
// Tiled shapes, then (last entry, bm = 0) the column-stationary kernel with
// RS_NG * 16 columns per workgroup (FP32 and 16-bit only).
static const TileShape kTiles[] = {{64, 64},  {64, 128}, {128, 64}, {128, 128}, {96, 64},
                                   {96, 128}, {224, 32}, {224, 64}, {96, 96},   {224, 96},
                                   {224, 128}, {64, 96}, {128, 96}, {64, 32},  {0, RS_NG * 16}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

int gemm_num_tiles(int) { return kNumTiles; }

void gemm_tile_shape(int tile, int* bm, int* bn) {
  const bool ok = tile >= 0 && tile < kNumTiles;
  *bm = ok ? kTiles[tile].bm : 0;
  *bn = ok ? kTiles[tile].bn : 0;
}

template <typename T, int BM, int BN>
static hipError_t run_gemm(const GemmArgs& g, hipStream_t st) {
  dim3 grid((g.Npad + BM - 1) / BM, (g.ncols + BN - 1) / BN);
  hipLaunchKernelGGL((gemm_kernel<T, BM, BN>), grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

template <typename L, int BM, int BN>
static hipError_t run_gemm_lp(const GemmArgs& g, hipStream_t st) {
  dim3 grid((g.Npad + BM - 1) / BM, (g.ncols + BN - 1) / BN);
  hipLaunchKernelGGL((gemm_lp_kernel<L, BM, BN>), grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

template <int BM, int BN>
static hipError_t run_kind(int kind, const GemmArgs& g, hipStream_t st) {
  switch (kind) {
    case 0: return run_gemm<float, BM, BN>(g, st);
    case 1: return run_gemm<double, BM, BN>(g, st);
    case 2: return run_gemm_lp<__bf16, BM, BN>(g, st);
    case 3: return run_gemm_lp<_Float16, BM, BN>(g, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm(int kind, int tile, const GemmArgs& g, hipStream_t st) {
  if (g.ncols == 0) return hipSuccess;
  switch (tile) {
    case 0: return run_kind<64, 64>(kind, g, st);
    case 1: return run_kind<64, 128>(kind, g, st);
    case 2: return run_kind<128, 64>(kind, g, st);
    case 3: return run_kind<128, 128>(kind, g, st);
    case 4: return run_kind<96, 64>(kind, g, st);
    case 5: return run_kind<96, 128>(kind, g, st);
    case 6: return run_kind<224, 32>(kind, g, st);
    case 7: return run_kind<224, 64>(kind, g, st);
    case 8: return run_kind<96, 96>(kind, g, st);
    case 9: return run_kind<224, 96>(kind, g, st);
    case 10: return run_kind<224, 128>(kind, g, st);
    case 11: return run_kind<64, 96>(kind, g, st);
    case 12: return run_kind<128, 96>(kind, g, st);
    case 13: return run_kind<64, 32>(kind, g, st);
    case kNumTilesTiled: return run_gemm_rs(kind, g, st);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------- 16-bit fragment order
int gemm_rs_nks(int Npad) { return rs_nks(Npad) <= RS_KS_MAX ? rs_nks(Npad) : 0; }

__global__ void __launch_bounds__(256) fragment_f32_kernel(const float* __restrict__ op, int Npad,
                                                           float* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // one 4-value vector
  const int nkg = Npad / 16;
  const size_t total = (size_t)(Npad / 16) * nkg * 64;
  if (idx >= total) return;
  const int lane = (int)(idx % 64);
  const int kg = (int)((idx / 64) % nkg);
  const int rb = (int)(idx / (64 * (size_t)nkg));
  const float* src = op + (size_t)(rb * 16 + (lane & 15)) * Npad + 16 * kg + 4 * (lane >> 4);
  *reinterpret_cast<float4*>(out + 4 * idx) = *reinterpret_cast<const float4*>(src);
}

template <typename L>
__global__ void __launch_bounds__(256) fragment_kernel(const L* __restrict__ op, int Npad, int nks,
                                                       L* __restrict__ out) {
  typedef typename Mfma32<L>::vec_t vec_t;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // one 8-value vector
  const size_t total = (size_t)(Npad / 16) * nks * 64;
  if (idx >= total) return;
  const int lane = (int)(idx % 64);
  const int ks = (int)((idx / 64) % nks);
  const int rb = (int)(idx / (64 * (size_t)nks));
  const int row = rb * 16 + (lane & 15), k0 = 32 * ks + 8 * (lane >> 4);
  vec_t v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = k0 + j < Npad ? op[(size_t)row * Npad + k0 + j] : L(0.0f);
  *reinterpret_cast<vec_t*>(out + 8 * idx) = v;
}

hipError_t launch_convert_fragments(int kind, const void* op, int Npad, void* out,
                                    hipStream_t st) {
  if (kind == 0) {  // FP32: 16-k groups of 4 values per lane
    if (Npad % 16 != 0) return hipErrorInvalidValue;
    const size_t total = (size_t)(Npad / 16) * (Npad / 16) * 64;
    hipLaunchKernelGGL(fragment_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       st, static_cast<const float*>(op), Npad, static_cast<float*>(out));
    return hipGetLastError();
  }
  const int nks = gemm_rs_nks(Npad);
  if (Npad % 16 != 0 || nks == 0) return hipErrorInvalidValue;
  const size_t total = (size_t)(Npad / 16) * nks * 64;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (kind == 2)
    hipLaunchKernelGGL(fragment_kernel<__bf16>, grid, dim3(256), 0, st,
                       static_cast<const __bf16*>(op), Npad, nks, static_cast<__bf16*>(out));
  else if (kind == 3)
    hipLaunchKernelGGL(fragment_kernel<_Float16>, grid, dim3(256), 0, st,
                       static_cast<const _Float16*>(op), Npad, nks, static_cast<_Float16*>(out));
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace npfem
