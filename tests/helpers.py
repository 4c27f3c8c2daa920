"""Shared test helpers: run the same seeded input through the oracle and through
the GPU library (via its C ABI binding) and compare."""
import numpy as np

import oracle


def oracle_moments(cfg, prim):
    return oracle.moments_from_primitives(cfg["dim"], cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])


def gpu_moments(cfg, prim):
    import paper_2508_06911_amd as lb
    return lb.moments_from_primitives(cfg["dim"], cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])


def run_oracle(cfg, prim, steps, mom=None):
    m = oracle_moments(cfg, prim) if mom is None else mom
    st, out, stats, done = oracle.step(cfg, m, steps)
    assert st == 0, "oracle failed with %d at step %d cell %d" % (st, done, stats["fail_cell"])
    return out, stats


def run_gpu(cfg, prim, steps, precision=0, guess=0, mom=None):
    import paper_2508_06911_amd as lb
    m = gpu_moments(cfg, prim) if mom is None else mom
    ctx = lb.Lelbm(cfg, m, precision=precision, guess=guess)
    stats = ctx.step(steps) if steps > 0 else None
    out = ctx.read_moments()
    ctx.close()
    return out, stats


def rel_linf(a, b):
    """max over moments of max |a - b| / max(max |b_k|, max |b_0|)."""
    scale = np.maximum(np.abs(b).max(axis=1), np.abs(b[0]).max())
    return float((np.abs(a - b).max(axis=1) / scale).max())


def primitives(mom, dim, K):
    rho = mom[0]
    if dim == 1:
        ux = mom[1] / rho
        RT = ((mom[2] + mom[4]) / rho - ux * ux) / (1 + K)
        return rho, ux, np.zeros_like(ux), RT
    ux, uy = mom[1] / rho, mom[2] / rho
    RT = ((mom[3] + mom[5] + mom[8]) / rho - ux * ux - uy * uy) / (2 + K)
    return rho, ux, uy, RT
