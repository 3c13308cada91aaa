"""The allocation-free volume query (npfem_get_volume_noalloc) against
npfem_get_volume, through the C ABI.

Both run the same per-cell FP64 volume kernel; the first stages its results
in the library's static device array, the second in the batch's own buffer,
so the outputs must be bitwise equal. Two calls in a row, the second on a
smaller batch (the static array keeps the first call's contents beyond the
second's cells), and a batch above the array's capacity is refused.
"""
import ctypes

import numpy as np
import pytest

from npfem_workload import meshes, suspensions as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_04332_amd import _lib
    _lib.load()


def _volumes(b):
    from paper_2011_04332_amd import _lib
    lib = _lib.load()
    a = np.full(b.n_cells, np.nan)
    c = np.full(b.n_cells, np.nan)
    _lib.check(lib.npfem_get_volume(b.handle, a.ctypes.data))
    _lib.check(lib.npfem_get_volume_noalloc(b.handle, c.ctypes.data))
    return a, c


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_volume_noalloc_equals_volume(prec):
    from paper_2011_04332_amd import solver
    # first call: 40 lattice RBCs after two steps
    s = W.stiff(W.rbc_lattice(n_cells=40, n_steps=2))
    b, pos, vel, f, _ = solver.batch_from_suspension(s, precision=prec)
    for _ in range(2):
        b.step(f, s.dt, 3)
    b.sync_status()
    a, c = _volumes(b)
    b.close()
    assert np.all(np.isfinite(a)) and np.array_equal(a, c)
    # second call: a smaller batch of a different class (platelets + RBCs)
    s2 = W.precision_sweep(n_rbc=3, n_plt=5, n_steps=1)
    b2, pos2, vel2, f2, _ = solver.batch_from_suspension(s2, precision=prec)
    b2.step(f2, s2.dt, 2)
    b2.sync_status()
    a2, c2 = _volumes(b2)
    b2.close()
    assert np.all(np.isfinite(a2)) and np.array_equal(a2, c2)
    assert a2.shape == (8,)


def test_volume_noalloc_refuses_more_cells_than_the_array_holds():
    import torch
    from paper_2011_04332_amd import _lib, solver
    x, t = meshes.icosahedron()
    m = solver.Mesh(x, t)
    n = (1 << 16) + 1
    pos = torch.tensor(np.tile(x.T, (1, n)), dtype=torch.float32, device="cuda").contiguous()
    vel = torch.zeros_like(pos)
    b = solver.Batch([m], np.zeros(n, dtype=np.int32), pos, vel, precision="fp32")
    out = np.empty(n)
    rc = _lib.load().npfem_get_volume_noalloc(b.handle, out.ctypes.data)
    assert rc == _lib.ERR_INVALID_ARG
    assert b"65536" in _lib.load().npfem_last_error()
    # the allocating query still serves it
    _lib.check(_lib.load().npfem_get_volume(b.handle, out.ctypes.data))
    assert np.allclose(out, out[0]) and out[0] > 0
    b.close()
