"""DAS launch plans (host only): the LDS window invariants that keep every
index of the kernel inside its buffers hold for every workload shape."""

import pytest

import paper_1811_01566_amd as wf
import phantom
from phantom.configs import served_mix
from wfhelp import scan_from_workload

QMAX = 511  # Q9.23: window-local delay sums stay below 512 samples
LDS_LIMIT = 163840  # gfx950: up to 160 KB of LDS for one workgroup
THREADS = 256


def _check(w):
    info = wf.tile_info(scan_from_workload(w), w.n_s, w.n_frames)
    span, nst, slot = info["span"], info["nst"], info["slot"]
    nt = info["threads"]
    # unmasked: entry (n0 & 7) + floor(tx + rx) <= 7 + 2 span < nst
    assert 7 + 2 * span < nst
    # masked: receive delay = nst, entry <= 7 + nst + span < slot
    assert 7 + nst + span < slot
    assert nst + span <= QMAX
    assert nst % 8 == 0
    assert info["lds_bytes"] <= LDS_LIMIT
    assert info["lds_bytes"] >= 2 * info["chunk"] * slot * 8 + 32 * w.n_tx
    # staged groups of one pass fit the per-lane register staging (1 group
    # per lane on 1024-thread tiles, 2 on 512-thread, 4 on 256-thread tiles)
    ng = {1024: 1, 512: 2}.get(nt, 4)
    assert info["chunk"] * (nst // 8) <= ng * nt
    assert (nt, info["px"]) in ((1024, 2), (512, 2), (512, 1), (256, 1))
    assert info["tile_z"] * info["tile_x"] == nt * info["px"]
    assert nt % info["tile_z"] == 0
    assert info["ntz"] * info["tile_z"] >= w.nz > (info["ntz"] - 1) * info["tile_z"]
    assert info["ntx"] * info["tile_x"] >= w.nx > (info["ntx"] - 1) * info["tile_x"]
    return info


@pytest.mark.parametrize("name", ["stai_small", "stai_full", "pwi", "pwi_batch8", "paper_stai",
                                  "paper_pwi"])
def test_named_workloads(name):
    info = _check(phantom.get_workload(name))
    if name == "pwi":
        assert info["px"] * info["threads"] >= 1024 and info["tile_z"] == 64


def test_tiny_and_edge_workloads():
    for w in (phantom.tiny_stai(), phantom.tiny_pwi(), phantom.tiny_pwi(nz=1, nx=1),
              phantom.tiny_stai(f_number=0.8, t0=0.3e-6)):
        _check(w)


def test_served_mix_shapes():
    n = 0
    for w in served_mix():
        _check(w)
        n += 1
    assert n == 207  # 23 (mode, N, T) combinations x 3 record lengths x 3 grids


def _split(w, frames=None):
    info = wf.tile_info(scan_from_workload(w), w.n_s, frames or w.n_frames)
    ws = wf.das_workspace_bytes(scan_from_workload(w), w.n_s, frames or w.n_frames)
    return info, ws


def _check_split(w):
    info, ws = _split(w)
    tiles = info["ntz"] * info["ntx"]
    nch = -(-w.n_ch // info["chunk"])  # channel chunks
    nsc = -(-nch // info["split_chunks"])  # chunk splits
    assert info["nsplit"] == nsc * info["split_tx_parts"]
    assert info["split_tx"] * info["split_tx_parts"] >= w.n_tx
    assert 0 < info["workgroups"] <= tiles * info["nsplit"]
    # the workspace holds one partial frame per split (none without a split)
    frame = w.nz * w.nx * 4 * w.n_frames
    assert ws == (info["nsplit"] * frame if info["nsplit"] > 1 else 0)
    # the plan never depends on the frame count (batch and frames agree)
    info8, ws8 = _split(w, frames=8)
    assert {k: v for k, v in info8.items()} == info
    assert ws8 == (info["nsplit"] * w.nz * w.nx * 4 * 8 if info["nsplit"] > 1 else 0)
    return info


@pytest.mark.parametrize("name", ["stai_small", "stai_full", "pwi", "paper_stai", "paper_pwi"])
def test_split_plans(name):
    w = phantom.get_workload(name)
    info = _check_split(w)
    tiles = info["ntz"] * info["ntx"]
    if name == "pwi":
        # uniform work, one tile per workgroup slot: no split, every tile runs
        assert info["nsplit"] == 1 and info["workgroups"] == tiles
    if name == "stai_full":
        # the 5-50 mm grid outruns the 2048-sample record and the f/1.5
        # aperture leaves chunks idle: split, and empty items left out
        assert info["nsplit"] > 1 and info["workgroups"] < tiles * info["nsplit"]


def test_split_plans_served_mix():
    for w in served_mix()[::7]:
        _check_split(w)


@pytest.mark.parametrize("name", ["stai_small", "stai_full", "pwi", "paper_stai", "paper_pwi"])
def test_adjoint_tiles(name):
    """The adjoint keeps the gather's tiles when they have 1024 threads, else
    runs a 1024-pixel tile candidate with 1024 x 1 threads where one fits
    (STAI full: the 64 x 16 tile), else the gather's tiles."""
    w = phantom.get_workload(name)
    info = wf.tile_info(scan_from_workload(w), w.n_s, 1)
    adj = (info["adjoint_threads"], info["adjoint_px"], info["adjoint_tile_z"])
    gather = (info["threads"], info["px"], info["tile_z"])
    if info["threads"] == 1024:
        assert adj == gather and info["adjoint_nsplit"] == info["nsplit"]
    else:
        assert adj == gather or adj[:2] == (1024, 1)
    if name == "stai_full":
        assert gather[:2] == (512, 1) and adj == (1024, 1, 64)
    if name == "pwi":
        assert adj == (1024, 2, 64)


# The tile shape and height that ran fastest in a same-box sweep of every
# candidate (DAS launch time on MI355X), per geometry; the planner's cost
# model must keep choosing them.
MEASURED_BEST = {
    "stai_full": (512, 1, 32),
    "paper_stai": (512, 2, 64),
    "stai_small": (512, 1, 16),
    "paper_pwi": (512, 1, 64),
    "pwi": (1024, 2, 64),
    "stai_n128_t32_s1024_1024x512": (512, 2, 64),
    "stai_n64_t64_s1024_256x128": (512, 1, 32),
    "stai_n192_t64_s1024_512x256": (512, 2, 64),
    "pwi_n128_t128_s2048_512x256": (512, 2, 64),
}


@pytest.mark.parametrize("name", sorted(MEASURED_BEST))
def test_planner_picks_the_measured_best_tiles(name):
    from phantom.configs import served_pool

    pool = {w.name: w for w in served_pool(8)}
    w = pool[name] if name in pool else phantom.get_workload(name)
    info = wf.tile_info(scan_from_workload(w), w.n_s, 1)
    assert (info["threads"], info["px"], info["tile_z"]) == MEASURED_BEST[name]


def test_adjoint_tiles_served_mix():
    """Over the served shape classes the adjoint's launch is the gather's, or
    1024 x 1 threads over a 1024-pixel tile of the same family (its tile
    height one the gather's candidates take), with a split of its own."""
    for w in served_mix()[::3]:
        info = wf.tile_info(scan_from_workload(w), w.n_s, 1)
        adj = (info["adjoint_threads"], info["adjoint_px"])
        gather = (info["threads"], info["px"])
        assert adj == gather or adj == (1024, 1), (w.name, gather, adj)
        if adj != gather:
            assert gather[0] < 1024
            assert info["adjoint_tile_z"] in (8, 16, 32, 64)
        assert 1 <= info["adjoint_nsplit"] <= 64
