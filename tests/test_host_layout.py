"""Host logic of the device library, on the CPU: the C ABI exports what the
header declares, the preparation step (FP64 precompute, ordering, tiling,
owned/shared node tables) is exact, and its errors fire."""
import ctypes
import os
import re

import numpy as np
import pytest

from synth.configs import radial_regions, small_sphere_case, uneven_batch
from synth.mesh import sphere_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cellmech.h")


def _lib_or_skip():
    from paper_2003_03130_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.fail("libcellmech.so is not built (run __graft_entry__.build())")
    return _native


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_header_function():
    nat = _lib_or_skip()
    lib = ctypes.CDLL(nat.LIB_PATH)
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"{n} declared in cellmech.h but not exported"
        assert n in nat.SIGNATURES, f"{n} has no ctypes signature"
    assert set(nat.SIGNATURES) == set(names)
    assert nat.lib().cm_version() == 1


def test_binding_arity_matches_header():
    """Every ctypes signature takes as many arguments as the C declaration
    (a missing or extra argument would shift every pointer after it)."""
    nat = _lib_or_skip()
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    decls = re.findall(r"\b(?:int|void|const char\*)\s+(cm_[a-z_0-9]+)\s*\(([^;]*?)\);",
                       text, flags=re.S)
    assert len(decls) == len(header_functions())
    for name, params in decls:
        n = 0 if params.strip() in ("", "void") else len(params.split(","))
        assert len(nat.SIGNATURES[name][1]) == n, name


def test_layout_create_is_the_single_region_form():
    """cm_layout_create prepares exactly what cm_layout_create_regions does
    without regions (every exported table equal)."""
    from paper_2003_03130_amd import HostLayout
    from paper_2003_03130_amd.cells import _host_inputs, _options, _ptr
    nat = _lib_or_skip()
    b = uneven_batch(n_cells=3, seed=78, tet_lo=300, tet_hi=3000, ladder=3)
    L = HostLayout(b.node_off, b.tet_off, b.x, b.tets, tile_tets=256)
    node_off, tet_off, x, tets = _host_inputs(b.node_off, b.tet_off, b.x, b.tets)
    opt = _options(None, 256, None)
    h = ctypes.c_void_p()
    nat.check(nat.lib().cm_layout_create(len(node_off) - 1, _ptr(node_off), _ptr(tet_off),
                                         _ptr(x), _ptr(tets), ctypes.byref(opt),
                                         ctypes.byref(h)))
    L2 = HostLayout.__new__(HostLayout)
    L2.n_regions = 1
    L2._load(h)
    for name in ("tiles", "slot_node", "shared_node", "shared_slot_ptr", "shared_slots",
                 "cell_tile_off", "cell_shared_off", "new_to_old", "tile_mat", "B", "V0",
                 "local_idx", "empty"):
        assert np.array_equal(getattr(L, name), getattr(L2, name)), name


def _batch(n_cells=5):
    return uneven_batch(n_cells=n_cells, seed=77, tet_lo=300, tet_hi=6000,
                        ladder=4)


def _decode_tets(L, b):
    """Rebuild every tetrahedron (input numbering, cell-local, in the slot
    order the layout chose) from the tiles: rows (cell, v0..v3, chunk, lane,
    tile)."""
    out = []
    for t in range(L.n_tiles):
        cb, nt, ob, no, sb, ns, cell, nch = L.tiles[t]
        count = 0
        for c in range(cb, cb + nch):
            for lane in np.flatnonzero(~L.empty[c]):
                loc = L.local_idx[c, lane]
                assert (loc < no + ns).all()
                internal = np.where(loc < no, ob + loc,
                                    L.slot_node[sb + np.minimum(loc - no, ns - 1)])
                out.append((cell, *(L.new_to_old[internal] - b.node_off[cell]),
                            c, lane, t))
                count += 1
        assert count == nt
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("order,tile", [(0, 64), (1, 256), (2, 1024), (2, 128),
                                        (3, 768), (3, 192)])
def test_layout_is_a_relabelling_of_the_input(order, tile):
    from paper_2003_03130_amd import HostLayout
    b = _batch()
    L = HostLayout(b.node_off, b.tet_off, b.x, b.tets, order=order,
                   tile_tets=tile)
    assert L.n_nodes == b.n_nodes and L.n_cells == b.n_cells
    # permutation that keeps each cell in its own node range
    assert np.array_equal(np.sort(L.new_to_old), np.arange(b.n_nodes))
    for c in range(b.n_cells):
        seg = L.new_to_old[b.node_off[c]:b.node_off[c + 1]]
        assert seg.min() >= b.node_off[c] and seg.max() < b.node_off[c + 1]
    # every input tetrahedron exactly once (its vertices may be reordered)
    rec = _decode_tets(L, b)
    got = np.concatenate([rec[:, :1], np.sort(rec[:, 1:5], axis=1)], axis=1)
    cell_of_tet = np.repeat(np.arange(b.n_cells), np.diff(b.tet_off))
    want = np.concatenate([cell_of_tet[:, None], np.sort(b.tets, axis=1)],
                          axis=1)
    got_s = got[np.lexsort(got.T[::-1])]
    want_s = want[np.lexsort(want.T[::-1])]
    assert np.array_equal(got_s, want_s)
    # tiles stay within a cell and hold at most tile_tets tetrahedra
    assert (L.tiles[:, 1] <= tile).all() and (L.tiles[:, 1] > 0).all()
    # within a chunk, each vertex slot names distinct nodes (the kernels add
    # slot by slot without atomics)
    for c in range(L.n_chunks):
        live = ~L.empty[c]
        for slot in range(4):
            ids = L.local_idx[c, live, slot]
            assert len(np.unique(ids)) == len(ids), (c, slot)
    for c in range(b.n_cells):
        assert (L.tiles[L.cell_tile_off[c]:L.cell_tile_off[c + 1], 6] == c).all()
    # FP64-derived B and V0, stored in float32: B (x^k - x^4) = I
    xg = b.x[b.node_off[rec[:, 0]][:, None] + rec[:, 1:5]]
    Dm = np.stack([xg[:, k] - xg[:, 3] for k in range(3)], axis=2)
    Bst = L.B[rec[:, 5], rec[:, 6]].astype(np.float64)
    err = np.abs(Bst @ Dm - np.eye(3)).max(axis=(1, 2))
    cond = np.linalg.cond(Dm)
    assert (err <= 4e-7 * cond).all()
    V0 = L.V0[rec[:, 5], rec[:, 6]].astype(np.float64)
    assert np.allclose(V0, np.abs(np.linalg.det(Dm)) / 6, rtol=2e-7, atol=0)


@pytest.mark.parametrize("order", [2, 3])
def test_owned_and_shared_tables_partition_the_nodes(order):
    from paper_2003_03130_amd import HostLayout
    b = _batch(4)
    L = HostLayout(b.node_off, b.tet_off, b.x, b.tets, tile_tets=256,
                   order=order)
    owner = np.full(b.n_nodes, -1)
    for t in range(L.n_tiles):
        ob, no = L.tiles[t, 2], L.tiles[t, 3]
        assert (owner[ob:ob + no] == -1).all()
        owner[ob:ob + no] = t
    shared = np.zeros(b.n_nodes, dtype=bool)
    shared[L.shared_node] = True
    assert ((owner >= 0) ^ shared).all()
    # tiles touching each node, from the decoded tetrahedra
    rec = _decode_tets(L, b)
    touch = {}
    tile_of_chunk = np.repeat(np.arange(L.n_tiles), L.tiles[:, 7])
    internal = L.new_to_old.argsort()
    for row in rec:
        cell = row[0]
        t = tile_of_chunk[row[5]]
        for v in row[1:5]:
            touch.setdefault(int(internal[b.node_off[cell] + v]), set()).add(int(t))
    for s, g in enumerate(L.shared_node):
        slots = L.shared_slots[L.shared_slot_ptr[s]:L.shared_slot_ptr[s + 1]]
        assert (L.slot_node[slots] == g).all()
        tiles = [int(np.searchsorted(L.tiles[:, 4], sl, side="right") - 1)
                 for sl in slots]
        assert tiles == sorted(touch.get(int(g), set()))
    for g in np.flatnonzero(owner >= 0):
        assert touch[int(g)] == {int(owner[g])}


@pytest.mark.parametrize("order", [2, 3])
def test_layout_scatter_matches_direct_assembly(order):
    """Summing per-tetrahedron corner values through the tile tables (LDS
    accumulation, owned stores, slot partials, finalize) equals a direct
    scatter-add: checks the reduction plumbing independently of the physics."""
    from paper_2003_03130_amd import HostLayout
    b = _batch(3)
    L = HostLayout(b.node_off, b.tet_off, b.x, b.tets, tile_tets=192,
                   order=order)
    rng = np.random.default_rng(0)
    rec = _decode_tets(L, b)
    vals = rng.normal(size=(len(rec), 4))
    direct = np.zeros(b.n_nodes)
    for r, v in zip(rec, vals):
        np.add.at(direct, b.node_off[r[0]] + r[1:5], v)
    # through the layout
    out = np.full(b.n_nodes, np.nan)
    part = np.zeros(L.n_slots)
    tile_of_chunk = np.repeat(np.arange(L.n_tiles), L.tiles[:, 7])
    by_tile = {}
    for r, v in zip(rec, vals):
        by_tile.setdefault(tile_of_chunk[r[5]], []).append((r, v))
    for t in range(L.n_tiles):
        cb, nt, ob, no, sb, ns, cell, _ = L.tiles[t]
        acc = np.zeros(no + ns)
        for r, v in by_tile[t]:
            np.add.at(acc, L.local_idx[r[5], r[6]], v)
        out[ob:ob + no] = acc[:no]
        part[sb:sb + ns] = acc[no:]
    for s, g in enumerate(L.shared_node):
        out[g] = part[L.shared_slots[L.shared_slot_ptr[s]:
                                     L.shared_slot_ptr[s + 1]]].sum()
    got = np.empty_like(out)
    got[L.new_to_old] = out
    assert np.allclose(got, direct, rtol=0, atol=1e-12)


def test_template_layout_replicates_one_cell():
    """cm_layout_create_template: one chunk array, and per cell the tables of
    the single-cell layout shifted by that cell's node and slot offsets, tile
    k of cell c at k n_cells + c; decoding it gives every cell's tetrahedra
    and the reduction plumbing still equals a direct scatter-add."""
    from paper_2003_03130_amd import HostLayout
    cell = small_sphere_case(1001)
    x, tets = cell.x, cell.tets
    n, C = len(x), 3
    L1 = HostLayout([0, n], [0, len(tets)], x, tets, tile_tets=256)
    LT = HostLayout.template(C, x, tets, tile_tets=256)
    assert LT.n_chunks == L1.n_chunks and LT.n_cells == C
    assert LT.n_tiles == C * L1.n_tiles and LT.n_nodes == C * n
    assert LT.n_slots == C * L1.n_slots and LT.n_shared == C * L1.n_shared
    assert np.array_equal(LT.local_idx, L1.local_idx)
    assert np.array_equal(LT.B, L1.B) and np.array_equal(LT.V0, L1.V0)
    S1, H1 = L1.n_slots, L1.n_shared
    for c in range(C):
        t = LT.tiles[c::C]
        want = L1.tiles.copy()
        want[:, 2] += c * n
        want[:, 4] += c * S1
        want[:, 6] = c
        assert np.array_equal(t, want)
        sl = slice(c * S1, (c + 1) * S1)
        assert np.array_equal(LT.slot_node[sl], L1.slot_node + c * n)
        assert np.array_equal(LT.shared_slots[sl], L1.shared_slots + c * S1)
        sh = slice(c * H1, (c + 1) * H1)
        assert np.array_equal(LT.shared_node[sh], L1.shared_node + c * n)
        assert np.array_equal(LT.shared_slot_ptr[c * H1:(c + 1) * H1 + 1],
                              L1.shared_slot_ptr + c * S1)
        assert np.array_equal(LT.new_to_old[c * n:(c + 1) * n],
                              L1.new_to_old + c * n)
        assert np.array_equal(LT.cell_shared_off[c:c + 2],
                              [c * H1, (c + 1) * H1])

    class _B:
        node_off = np.arange(C + 1) * n
    rec = _decode_tets(LT, _B)
    for c in range(C):
        got = np.sort(rec[rec[:, 0] == c, 1:5], axis=1)
        want = np.sort(tets, axis=1)
        assert np.array_equal(got[np.lexsort(got.T[::-1])],
                              want[np.lexsort(want.T[::-1])])
    # plumbing with shared chunks: per (tile, lane) values through the tables
    rng = np.random.default_rng(5)
    vals = rng.normal(size=(len(rec), 4))
    direct = np.zeros(C * n)
    for r, v in zip(rec, vals):
        np.add.at(direct, r[0] * n + r[1:5], v)
    out = np.full(C * n, np.nan)
    part = np.zeros(LT.n_slots)
    acc = {}
    for r, v in zip(rec, vals):
        cb, nt, ob, no, sb, ns, _, _ = LT.tiles[r[7]]
        a = acc.setdefault(int(r[7]), np.zeros(no + ns))
        np.add.at(a, LT.local_idx[r[5], r[6]], v)
    for t, a in acc.items():
        cb, nt, ob, no, sb, ns, _, _ = LT.tiles[t]
        out[ob:ob + no] = a[:no]
        part[sb:sb + ns] = a[no:]
    for s_, g in enumerate(LT.shared_node):
        out[g] = part[LT.shared_slots[LT.shared_slot_ptr[s_]:
                                      LT.shared_slot_ptr[s_ + 1]]].sum()
    got = np.empty_like(out)
    got[LT.new_to_old] = out
    assert np.allclose(got, direct, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", [2, 3])
def test_region_layout_tiles_one_region_each(order):
    """cm_layout_create_regions: still a relabelling of every cell's
    tetrahedra; every tile holds tetrahedra of one region only, the one its
    material slot names; the tiles of each slot are its first/count range; a
    region without tetrahedra in a cell gets no tiles."""
    from paper_2003_03130_amd import HostLayout
    b = _batch(4)
    R = 4  # region 3 is never used
    reg = np.concatenate([radial_regions(b.x[b.node_off[c]:b.node_off[c + 1]],
                                         b.tets[b.tet_off[c]:b.tet_off[c + 1]])
                          for c in range(b.n_cells)])
    L = HostLayout(b.node_off, b.tet_off, b.x, b.tets, tile_tets=256,
                   regions=reg, n_regions=R, order=order)
    rec = _decode_tets(L, b)
    # region of every decoded tetrahedron, by matching its sorted vertices
    key = {}
    for c in range(b.n_cells):
        for t in range(b.tet_off[c], b.tet_off[c + 1]):
            key[(c, *np.sort(b.tets[t]))] = int(reg[t])
    seen = set()
    for row in rec:
        k = (int(row[0]), *np.sort(row[1:5]))
        assert k not in seen
        seen.add(k)
        mt = L.tile_mat[row[7]]
        assert mt // R == row[0] and mt % R == key[k]
    assert len(seen) == b.n_tets
    for c in range(b.n_cells):
        tiles_c = []
        for r in range(R):
            m = c * R + r
            first, cnt = L.mat_tile_first[m], L.mat_tile_count[m]
            t = np.arange(first, first + cnt)
            assert (L.tile_mat[t] == m).all()
            tiles_c.extend(t.tolist())
            n_r = int((reg[b.tet_off[c]:b.tet_off[c + 1]] == r).sum())
            assert L.tiles[t, 1].sum() == n_r
            assert (cnt == 0) == (n_r == 0)
        assert sorted(tiles_c) == list(range(L.cell_tile_off[c],
                                             L.cell_tile_off[c + 1]))
    # one region: same tiles as the plain layout
    L1 = HostLayout(b.node_off, b.tet_off, b.x, b.tets, tile_tets=256,
                    regions=np.zeros(b.n_tets, np.uint8), n_regions=1)
    L0 = HostLayout(b.node_off, b.tet_off, b.x, b.tets, tile_tets=256)
    assert np.array_equal(L1.tiles, L0.tiles)
    assert np.array_equal(L1.local_idx, L0.local_idx)
    assert np.array_equal(L1.tile_mat, L0.tiles[:, 6])


@pytest.mark.parametrize("case", ["id_range", "zero", "too_many"])
def test_region_preparation_errors(case):
    from paper_2003_03130_amd import HostLayout, CellmechError
    from paper_2003_03130_amd import _native as nat
    x, tets = sphere_mesh(150, 3)
    reg = np.zeros(len(tets), np.uint8)
    nr = 2
    if case == "id_range":
        reg[4] = 2
    elif case == "zero":
        nr = 0
    else:
        nr = 65
    with pytest.raises(CellmechError) as ei:
        HostLayout([0, len(x)], [0, len(tets)], x, tets, regions=reg,
                   n_regions=nr)
    assert ei.value.status == nat.CM_EINVAL


@pytest.mark.parametrize("case", ["cells", "sizes", "index_range"])
def test_template_preparation_errors(case):
    from paper_2003_03130_amd import HostLayout, CellmechError
    from paper_2003_03130_amd import _native as nat
    x, tets = sphere_mesh(150, 3)
    tets = tets.copy()
    n_cells = 2
    if case == "cells":
        n_cells = 0
    elif case == "sizes":
        x = np.zeros((0, 3))
    elif case == "index_range":
        tets[5, 2] = len(x)
    with pytest.raises(CellmechError) as ei:
        HostLayout.template(n_cells, x, tets)
    assert ei.value.status == nat.CM_EINVAL


def test_unreferenced_node_is_shared_with_no_slots():
    from paper_2003_03130_amd import HostLayout
    c = small_sphere_case(1000)
    x = np.concatenate([c.x, [[5.0, 5.0, 5.0]]])
    L = HostLayout([0, len(x)], [0, len(c.tets)], x, c.tets, tile_tets=512)
    g = int(np.flatnonzero(L.new_to_old == len(x) - 1)[0])
    s = int(np.flatnonzero(L.shared_node == g)[0])
    assert L.shared_slot_ptr[s] == L.shared_slot_ptr[s + 1]


@pytest.mark.parametrize("case", ["index_range", "repeat", "degenerate",
                                  "tile", "empty_cell", "order", "offsets"])
def test_preparation_errors(case):
    from paper_2003_03130_amd import HostLayout, CellmechError
    from paper_2003_03130_amd import _native as nat
    x, tets = sphere_mesh(150, 3)
    node_off, tet_off, kw = [0, len(x)], [0, len(tets)], {}
    tets = tets.copy()
    x = x.copy()
    status = nat.CM_EINVAL
    if case == "index_range":
        tets[5, 2] = len(x)
    elif case == "repeat":
        tets[7, 3] = tets[7, 0]
    elif case == "degenerate":
        a, bb, cc, d = tets[9]
        x[d] = (x[a] + x[bb] + x[cc]) / 3.0  # flatten one tetrahedron
        status = nat.CM_EDEGENERATE
    elif case == "tile":
        kw["tile_tets"] = 100
    elif case == "empty_cell":
        node_off, tet_off = [0, len(x), len(x)], [0, len(tets), len(tets)]
    elif case == "order":
        kw["order"] = 7
    elif case == "offsets":
        node_off = [1, len(x)]
    with pytest.raises(CellmechError) as ei:
        HostLayout(node_off, tet_off, x, tets, **kw)
    assert ei.value.status == status
    if case == "degenerate":
        assert "tetrahedron" in str(ei.value)


def test_tuned_creation_rejects_bad_candidates():
    """Candidate tile sizes are validated before any device work."""
    from paper_2003_03130_amd.cells import _host_inputs, _options, _ptr
    nat = _lib_or_skip()
    b = uneven_batch(n_cells=2, seed=79, tet_lo=300, tet_hi=800, ladder=2)
    node_off, tet_off, x, tets = _host_inputs(b.node_off, b.tet_off, b.x, b.tets)
    opt = _options(None, None, None)
    for cand in ([100], [64, 8192], [0]):
        c = np.array(cand, dtype=np.int32)
        h = ctypes.c_void_p()
        rc = nat.lib().cm_batch_create_tuned(
            2, _ptr(node_off), _ptr(tet_off), _ptr(x), _ptr(tets),
            ctypes.byref(opt), _ptr(c), len(c), None, None, None,
            ctypes.byref(h))
        assert rc == nat.CM_EINVAL and "multiples of 64" in nat.lib().cm_last_error().decode()
    h = ctypes.c_void_p()
    rc = nat.lib().cm_batch_create_tuned(
        2, _ptr(node_off), _ptr(tet_off), _ptr(x), _ptr(tets), ctypes.byref(opt),
        _ptr(np.array([256], dtype=np.int32)), 0, None, None, None, ctypes.byref(h))
    assert rc == nat.CM_EINVAL
