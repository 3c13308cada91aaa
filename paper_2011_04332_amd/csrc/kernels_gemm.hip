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

// ---------------------------------------------------------------- FP32/FP64
template <typename T, int BM, int BN>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
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

  // epilogue: each 16x16 block lies inside [0, Npad) or wholly outside it
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int mb = m0 + wm * WM + i * 16;
    if (mb >= Npad) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + wn * WN + j * 16 + (lane & 15);
      if (n >= ncols) continue;
      T* c = C + (size_t)n * Npad + mb;
      if (g.mode == EPI_ADD) {
#pragma unroll
        for (int r = 0; r < 4; ++r) c[Mfma4<T>::row(lane, r)] += acc[i][j][r];
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

  for (int j = tid; j < BN; j += 256) {
    float s = 1.0f;
    const int n = n0 + j;
    if (g.colscale && n < ncols) {
      const float mx = g.colscale[n];
      if (mx > 0.0f && isfinite(mx)) s = exp2f(-ceilf(log2f(mx)));
    }
    sc_in[j] = s;
  }
  __syncthreads();

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
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int m = m0 + wm * WM + i * 16 + (lane >> 4) * 4;
    if (m >= Npad) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int nn = wn * WN + j * 16 + (lane & 15);
      const int n = n0 + nn;
      if (n >= ncols) continue;
      const float unscale = beta / sc_in[nn];
      const float* bcol = B + (size_t)n * Npad + m;
      float* c = C + (size_t)n * Npad + m;
      if (g.mode == EPI_SPLIT_ADD) {
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] += hm * (bcol[r] + unscale * acc[i][j][r]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = hm * (bcol[r] + unscale * acc[i][j][r]);
      }
    }
  }
}

// ---------------------------------------------------------------- dispatch
struct TileShape {
  int bm, bn;
};
static const TileShape kTiles[] = {{64, 64},  {64, 128}, {128, 64}, {128, 128},
                                   {96, 64},  {96, 128}, {224, 32}, {224, 64}};
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
    default: return hipErrorInvalidValue;
  }
}

}  // namespace npfem
