"""dwg_gwn_grad_static (the allocation-free variant of dwg_gwn_grad, scratch from the
library's static device array) against dwg_gwn_grad with a caller workspace: two calls in a
row on one GPU, the second smaller, each within the GWN parity bound of the first entry
point's output. Inputs are seeded synthetic clouds."""
import numpy as np
import pytest

import oracle
from paper_2405_13839_amd import synth
from tests.helpers import TOL_G, TOL_W, cuda, e_g, e_w, host, unit_rows

pytestmark = pytest.mark.gpu


def _case(n, seed, lam, with_delta):
    c = synth.torus_ellipsoids(n, seed=seed)
    N = unit_rows(np.random.default_rng(seed), c.n)
    d = oracle.anchor_delta(c.P).astype(np.float32) if with_delta else None
    return c, N, d


def test_static_scratch_matches_workspace_entry_point():
    from paper_2405_13839_amd import dwg
    for n, seed, lam, with_delta, beta in [(300_000, 71, 10.0, True, 0.0), (20_000, 72, 0.0, False, 0.0),
                                           (50_000, 73, 10.0, True, 2.3)]:
        print(f"[static scratch] n={n} lam={lam} delta={with_delta} beta={beta}", flush=True)
        c, N, d = _case(n, seed, lam, with_delta)
        P, Nt, a = cuda(c.P), cuda(N), cuda(c.area)
        dt = cuda(d) if d is not None else None
        prm = dwg.Params(lam=lam, beta=beta)
        w1, g1, m1 = dwg.gwn_static(P, Nt, a, dt, P, prm, want_wmean=True)
        w0, g0, m0 = dwg.gwn(P, Nt, a, dt, P, prm, want_wmean=True)
        w0, g0 = host(w0).astype(np.float64), host(g0).astype(np.float64)
        ew, eg = e_w(host(w1), w0), e_g(host(g1), g0)
        print(f"[static scratch] e_w {ew:.2e} e_g {eg:.2e}", flush=True)
        assert ew <= TOL_W and eg <= TOL_G
        assert abs(m1.item() - m0.item()) <= 1e-6 * max(1.0, abs(m0.item()))


def test_static_scratch_rejects_sizes_beyond_it():
    from paper_2405_13839_amd import dwg
    c, N, _ = _case(700_000, 74, 0.0, False)
    P = cuda(c.P)
    with pytest.raises(dwg.DwgError) as ei:
        dwg.gwn_static(P, cuda(N), cuda(c.area), None, P)
    assert ei.value.status == dwg.DWG_E_INVALID and "static scratch" in str(ei.value)
