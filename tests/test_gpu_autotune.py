"""cm_autotune with its JSON cache: a miss measures and stores one entry per
(device, mesh) key; a hit takes the stored configuration without measuring;
other keys in the file survive."""
import json

import numpy as np
import pytest

from gpu_util import require_gpu
from synth.configs import uneven_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_autotune_cache_miss_then_hit(tmp_path):
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=12, seed=81, tet_lo=500, tet_hi=4000, ladder=3)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    path = tmp_path / "tune.json"
    path.write_text('{\n  "other-device|mesh": {"waves": 8, "blocks_per_cu": 4, "ms": 1.0}\n}\n')
    got = cb.autotune(y, str(path))
    rec = json.loads(path.read_text())
    assert "other-device|mesh" in rec and len(rec) == 2
    key = next(k for k in rec if k != "other-device|mesh")
    assert (rec[key]["waves"], rec[key]["blocks_per_cu"]) == tuple(got)
    assert rec[key]["ms"] > 0
    # a hit: the stored configuration is taken as it is
    other = (2, 0) if tuple(got) != (2, 0) else (1, 0)
    rec[key]["waves"], rec[key]["blocks_per_cu"] = other
    path.write_text("{\n" + ",\n".join(
        f'  "{k}": {json.dumps(v)}' for k, v in rec.items()) + "\n}\n")
    assert tuple(cb.autotune(y, str(path))) == other
    assert tuple(cb.get_launch()) == other
    # results do not depend on the launch configuration
    f1, E1 = cb.forces(y)
    cb.set_launch(*got)
    f2, E2 = cb.forces(y)
    assert np.array_equal(cb.to_host(f1), cb.to_host(f2))
    assert np.array_equal(E1.cpu().numpy(), E2.cpu().numpy())


def test_tuned_creation_picks_fastest_tile_and_caches(tmp_path):
    """cm_batch_create_tuned times every candidate tile size and keeps the
    fastest; its results equal those of a handle created directly with that
    tile size and launch; a cache hit prepares only the stored tile size."""
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=10, seed=82, tet_lo=800, tet_hi=6000, ladder=3)
    cand = [256, 384, 512]
    path = tmp_path / "tune.json"
    cb = CellBatch.tuned(b.node_off, b.tet_off, b.x, b.tets,
                         tile_candidates=cand, cache_path=str(path))
    ms = cb.candidate_ms
    assert np.all(np.isfinite(ms)) and np.all(ms > 0)
    tile = cb.info["tile_tets"]
    assert tile == cand[int(np.argmin(ms))]
    launch = cb.get_launch()
    rec = json.loads(path.read_text())
    (key, val), = rec.items()
    assert (val["tile"], val["waves"], val["blocks_per_cu"]) == (tile, *launch)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    ref = CellBatch(b.node_off, b.tet_off, b.x, b.tets, tile_tets=tile)
    ref.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    ref.set_launch(*launch)
    f1, E1 = cb.forces(cb.to_device(b.y))
    f2, E2 = ref.forces(ref.to_device(b.y))
    torch.cuda.synchronize()
    assert np.array_equal(cb.to_host(f1), ref.to_host(f2))
    assert torch.equal(E1, E2)
    # a hit: nothing is measured, the stored tile size and launch are taken
    cb2 = CellBatch.tuned(b.node_off, b.tet_off, b.x, b.tets,
                          tile_candidates=cand, cache_path=str(path))
    assert np.all(np.isinf(cb2.candidate_ms))
    assert cb2.info["tile_tets"] == tile and cb2.get_launch() == launch
    # parameters are the caller's to set
    from paper_2003_03130_amd._native import CellmechError
    with pytest.raises(CellmechError):
        cb2.forces(cb2.to_device(b.y))
