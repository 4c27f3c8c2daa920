"""Oscillating point mass source (Sec. IV.C, Eqs. VC1, VC6-VC8) on the HIP
path: parity with the oracle in 1D and 2D, with the run split across step
calls so that the source's time carries over, and the paper's acoustic plane
wave, whose decay gives the bulk viscosity (Eq. VC4) to compare with Eq.
(C8b), and whose amplitude the linearised equations fix at RT rate / (2 c_s)
for a source that adds mass at the local temperature."""
import numpy as np
import pytest

import lelbm_inputs as li
from helpers import gpu_moments, oracle_moments, rel_linf, run_oracle

pytestmark = pytest.mark.gpu


def _case(name):
    print("\n[gpu case] %s" % name, flush=True)


@pytest.mark.parametrize("dim", [1, 2])
def test_source_parity_across_calls(dim):
    import paper_2508_06911_amd as lb
    _case("mass source parity dim %d, 7 + 13 steps" % dim)
    if dim == 1:
        cfg, prim = li.acoustic_source(n=160, RT=1.0, rate=2e-3, period=16.0, nu_b=0.3, nu=0.05)
    else:
        cfg, prim = li.smooth_periodic(5, n=40, ny=24, dim=2)
        cfg["source"] = {"x": 11, "y": 7, "rate": 5e-3, "omega": 0.6, "t0": 2.0}
    ref, _ = run_oracle(cfg, prim, 20, mom=oracle_moments(cfg, prim))
    ctx = lb.Lelbm(cfg, gpu_moments(cfg, prim))
    ctx.step(7)
    ctx.step(13)
    out = ctx.read_moments()
    ctx.close()
    err = rel_linf(out, ref)
    print("rel Linf vs oracle %.3g" % err, flush=True)
    assert err < 1e-10
    # the source did something: the total mass moved by the injected amount
    m0 = oracle_moments(cfg, prim)[0].sum()
    src = cfg["source"]
    added = sum(src["rate"] * np.sin(src["omega"] * (src.get("t0", 0.0) + k)) for k in range(20))
    assert abs(out[0].sum() - m0 - added) < 1e-10 * m0


@pytest.mark.parametrize("prec,rate,tol", [(0, 1e-6, 0.03), (1, 1e-4, 0.05)])
def test_acoustic_source_bulk_viscosity(prec, rate, tol):
    import paper_2508_06911_amd as lb
    _case("acoustic source precision %d rate %g" % (prec, rate))
    cfg, prim = li.acoustic_source(n=1200, RT=1.0, rate=rate, period=64.0, nu_b=0.8, nu=1e-3)
    ctx = lb.Lelbm(cfg, gpu_moments(cfg, prim), precision=prec)
    ctx.step_nostats(320)
    hist = []
    for _ in range(128):
        ctx.step_nostats(1)
        m = ctx.read_moments()
        rho = m[0]
        ux = m[1] / rho
        RT = ((m[2] + m[4]) / rho - ux ** 2) / (1 + cfg["K"])
        hist.append(rho * RT)
    ctx.close()
    t = np.arange(320, 448) + 1.0
    w = cfg["source"]["omega"]
    A = np.stack([np.sin(w * t), np.cos(w * t), np.ones_like(t)], 1)
    coef = np.linalg.lstsq(A, np.array(hist), rcond=None)[0]
    amp = np.hypot(coef[0], coef[1])
    cs = np.sqrt(1.4)
    xs = cfg["source"]["x"]
    d1, d2 = 40, 200
    for side in (1, -1):
        ax = -np.log(amp[xs + side * d2] / amp[xs + side * d1]) / (d2 - d1)
        nu_b = 2 * cs ** 3 / w ** 2 * ax - 0.4 * cfg["nu"]
        a0 = amp[xs + side * d1] * np.exp(ax * d1) / (rate / (2 * cs))
        print("side %+d: nu_b %.4f (target %.4f), amplitude ratio %.4f" % (side, nu_b, cfg["nu_b"], a0), flush=True)
        assert abs(nu_b / cfg["nu_b"] - 1) < tol
        assert abs(a0 - 1) < tol
