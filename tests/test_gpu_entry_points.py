"""Entry points no driver in the package calls: cm_mesh_create (the
single-cell form of cm_batch_create), cm_qs_update (the bounded Newton
update, y += s x, s = min(1, cap / m), m the largest |component| of x over a
cell's nodes) and cm_stream_copy (the reference copy of the byte-counter
calibration)."""
import ctypes

import numpy as np
import pytest

from gpu_util import require_gpu
from synth.configs import small_sphere_case, uneven_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_mesh_create_equals_one_cell_batch():
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    c = small_sphere_case(1011)
    cb = CellBatch.single(c.x, c.tets)
    cb.set_params([c.theta[0]], [c.theta[1]], [c.theta[2]])
    f_ref, E_ref = cb.forces(cb.to_device(c.y))
    lib = nat.lib()
    x = np.ascontiguousarray(c.x, dtype=np.float64)
    tets = np.ascontiguousarray(c.tets, dtype=np.int32)
    h = ctypes.c_void_p()
    nat.check(lib.cm_mesh_create(len(x), len(tets), _ptr(x), _ptr(tets), None,
                                 _stream(None), ctypes.byref(h)))
    try:
        n = len(x)
        perm = np.empty(n, dtype=np.int64)
        nat.check(lib.cm_permutation(h, _ptr(perm)))
        mu, ka, w = (np.array([v], dtype=np.float64) for v in c.theta)
        nat.check(lib.cm_set_params(h, _ptr(mu), _ptr(ka), _ptr(w), 0, _stream(None)))
        y = torch.from_numpy(np.ascontiguousarray(
            c.y[perm].astype(np.float32).T).reshape(-1)).cuda()
        f = torch.empty(3 * n, dtype=torch.float32, device="cuda")
        E = torch.empty(1, dtype=torch.float64, device="cuda")
        nat.check(lib.cm_forces(h, _ptr(y), _ptr(f), _ptr(E), None, _stream(None)))
        torch.cuda.synchronize()
        assert torch.equal(f, f_ref) and torch.equal(E, E_ref)
    finally:
        lib.cm_destroy(h)


def test_qs_update_formula():
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    b = uneven_batch(n_cells=3, seed=83, tet_lo=300, tet_hi=2000, ladder=3)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    N = cb.n_nodes
    rng = np.random.default_rng(84)
    xh = rng.normal(size=(N, 3)).astype(np.float32)
    n0, n1 = b.node_off[2], b.node_off[3]
    xh[n0:n1] = 0.0  # cell 2 takes no step
    yh = rng.normal(size=(N, 3)).astype(np.float32)
    x, y = cb.to_device(xh), cb.to_device(yh)
    state = torch.full((cb.n_cells, 16), -7.0, dtype=torch.float64, device=cb.device)
    cap = 0.5
    nat.check(nat.lib().cm_qs_update(cb._h, _ptr(x), cap, _ptr(y), _ptr(state),
                                     _stream(None)))
    torch.cuda.synchronize()
    yn = cb.to_host(y).astype(np.float64)
    st = state.cpu().numpy()
    for c in range(cb.n_cells):
        sl = slice(b.node_off[c], b.node_off[c + 1])
        m = float(np.abs(xh[sl]).max())
        s = np.float32(min(1.0, cap / m)) if m > 0 else np.float32(1.0)
        want = yh[sl].astype(np.float64) + float(s) * xh[sl]
        assert np.abs(yn[sl] - want).max() <= 1e-6 * np.abs(want).max(), c
        if m > 0:
            assert st[c, 4] == float(s) and abs(st[c, 6] - m * float(s)) <= 1e-12 * m
        else:
            assert st[c, 4] == -7.0 and st[c, 6] == -7.0  # untouched


def test_stream_copy():
    """cm_stream_copy copies n floats exactly (sizes below, at and above one
    workgroup's 256 and past the 65,536-workgroup grid cap, so the grid
    stride loop runs), leaves the rest of dst alone, accepts n = 0 and
    rejects n < 0 and null pointers."""
    import torch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    lib = nat.lib()
    g = torch.Generator(device="cuda").manual_seed(5)
    for n in (1, 255, 256, 1000, 65536 * 256 + 77):
        src = torch.randn(n + 8, device="cuda", generator=g)
        dst = torch.full((n + 8,), -7.0, device="cuda")
        nat.check(lib.cm_stream_copy(_ptr(src), _ptr(dst), n, _stream(None)))
        torch.cuda.synchronize()
        assert torch.equal(dst[:n], src[:n]), n
        assert bool((dst[n:] == -7.0).all()), n
    dst = torch.zeros(4, device="cuda")
    nat.check(lib.cm_stream_copy(None, _ptr(dst), 0, _stream(None)))
    assert lib.cm_stream_copy(_ptr(dst), _ptr(dst), -1, _stream(None)) == nat.CM_EINVAL
    assert lib.cm_stream_copy(None, _ptr(dst), 4, _stream(None)) == nat.CM_EINVAL
