"""The two forms of the x and y transforms of the FFT Poisson solve (Sec. 2.3)
on the GPU: one workgroup per z plane and row parity, the z pass joining the
two halves of the y transform (the default wherever two such half planes fit
on a CU), and separate x and y passes.  Both must give the oracle's potential,
and each other's to rounding, on even and odd half-row lengths (nx / 2), even
and odd half-column lengths (ny / 2 = 9 and 3), radix-3 lengths, non-square
planes and the 128^3 grid.
"""
import numpy as np
import pytest

from gpu_helpers import make_pair, say

pytestmark = pytest.mark.gpu


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


def _rel(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def _phi_and_step(gp, cfg, st, form):
    sim, orc = make_pair(cfg, st)
    sim.set_fft_form(form)
    phi0 = sim.get_field("phi").cpu().numpy()
    sim.step(1)
    sim.sync()
    phi1 = sim.get_field("phi").cpu().numpy()
    return sim, orc, phi0, phi1


@pytest.mark.parametrize("shape,seed", [((16, 12, 8), 3), ((18, 12, 8), 5), ((96, 24, 12), 8), ((8, 36, 6), 2),
                                        ((128, 16, 4), 7), ((12, 18, 8), 11), ((16, 6, 4), 12)])
def test_forms_match_oracle(gp, W, shape, seed):
    say("fft forms", shape)
    cfg, st = W.random_periodic(n=shape, seed=seed)
    out = {}
    for form in (gp.GP_FFT_AUTO, gp.GP_FFT_LINES):
        sim, orc, phi0, phi1 = _phi_and_step(gp, cfg, st, form)
        ref0 = orc.get_field("phi")
        assert _rel(phi0, ref0) < 1e-12, (form, _rel(phi0, ref0))
        orc.step(1)
        ref1 = orc.get_field("phi")
        assert _rel(phi1, ref1) < 1e-12, (form, _rel(phi1, ref1))
        d, do = sim.diag()[-1], orc.diag()[-1]
        assert d["e_pot"] == pytest.approx(do["e_pot"], rel=1e-11)
        out[form] = (phi0, phi1, d["e_pot"])
    a, b = out[gp.GP_FFT_AUTO], out[gp.GP_FFT_LINES]
    assert _rel(a[0], b[0]) < 1e-13 and _rel(a[1], b[1]) < 1e-13
    assert a[2] == pytest.approx(b[2], rel=1e-13)


def test_forms_agree_fp32(gp, W):
    """FP32 transforms: both forms within FP32 rounding of the FP64 oracle."""
    say("fft forms fp32")
    cfg, st = W.random_periodic(n=(32, 24, 16), seed=11)
    cfg = dict(cfg, precision="fp32")
    phis = []
    for form in (gp.GP_FFT_AUTO, gp.GP_FFT_LINES):
        sim, orc = make_pair(cfg, st)
        sim.set_fft_form(form)
        phis.append(sim.get_field("phi").cpu().numpy().astype(np.float64))
    ref = orc.get_field("phi")
    for p in phis:
        assert _rel(p, ref) < 1e-6
    assert _rel(phis[0], phis[1]) < 1e-6


def test_forms_agree_two_disk_128(gp, W):
    """The 128^3 two-disk state: the plane form (one workgroup per z plane)
    against the separate passes, potential and potential energy."""
    import torch
    say("fft forms two-disk 128^3")
    cfg, st = W.two_disk_collision(128)
    res = []
    for form in (gp.GP_FFT_AUTO, gp.GP_FFT_LINES):
        sim = gp.Sim(cfg)
        sim.set_state({k: v.to("cuda") for k, v in st.items()})
        sim.set_fft_form(form)
        phi = sim.get_field("phi").cpu().numpy()
        sim.step(1)
        sim.sync()
        res.append((phi, sim.get_field("phi").cpu().numpy(), sim.diag()[-1]["e_pot"]))
        del sim
        torch.cuda.synchronize()
    (a0, a1, ea), (b0, b1, eb) = res
    assert _rel(a0, b0) < 1e-13 and _rel(a1, b1) < 1e-13
    assert ea == pytest.approx(eb, rel=1e-13)


def test_bad_form_rejected(gp, W):
    cfg, st = W.random_periodic(n=(8, 8, 8), seed=1)
    sim = gp.Sim(cfg)
    with pytest.raises(Exception):
        sim.set_fft_form(7)
