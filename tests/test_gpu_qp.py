"""The paper's collapse-time study (Sec. III) on the GPU against the oracle:
the approximate quasi-periodic families of Eq. (13) (k_d in {3, 5},
mu in {1, 1.75}, 40 modes) as one batch, in the paper's time integrator (RK3)
and the classical one, evolved to collapse at the paper's threshold
min A < 0.01: collapse step and time exact, the collapsed state at 1e-11; and
the mass integral of Sec. II (the sweep's mass loss) against the oracle's."""
import numpy as np
import pytest

import oracle as O
from paper_1706_07413_amd import adscl
from paper_1706_07413_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-11
FIELDS = ("Phi", "Pi", "A", "delta", "m")


def rel(g, o):
    n = np.max(np.abs(o))
    d = np.max(np.abs(np.asarray(g) - np.asarray(o)))
    return d / 1e-13 * TOL if n < 1e-12 else d / n


@pytest.mark.parametrize("rk", [3, 4])
def test_qp_families_collapse_like_the_oracle(rk):
    N, J = 257, 40
    rows = [(kd, mu, e) for kd, mu in I.QP_FAMILIES for e in (0.3, 0.16)]
    c = np.stack([I.qp_family(kd, mu, J) for kd, mu, _ in rows])
    eps = np.array([e for _, _, e in rows])
    b = adscl.Batch([N] * len(rows), a_collapse=0.01, n_modes=J, rk_order=rk)
    b.init_modes(eps, np.ascontiguousarray(c))
    M0 = b.constraints()[:, 4].copy()
    b.step(6000, 500.0)
    s = b.status()
    st = {k: v.cpu().numpy() for k, v in b.get_state().items()}
    M1 = b.constraints()[:, 4]
    b.close()
    for i, (kd, mu, e) in enumerate(rows):
        Phi, Pi = O.init_modes(N, e, c[i])
        r0 = O.evolve(Phi, Pi, 0)
        r = O.evolve_scheme(Phi, Pi, 6000, rk=rk, a_collapse=0.01)
        what = "k_d=%d mu=%g eps=%g rk%d" % (kd, mu, e, rk)
        assert r["state"] == O.COLLAPSED, what
        assert s["state"][i] == adscl.COLLAPSED and s["steps"][i] == r["steps"], (what, s["steps"][i], r["steps"])
        assert abs(s["t_c"][i] - r["t_c"]) <= 1e-12 * r["t_c"], what
        for f in FIELDS:
            assert rel(b.split(st[f])[i], r[f]) <= TOL, (what, f)
        m0 = O.mass_paper(Phi, Pi, r0["A"])
        m1 = O.mass_paper(r["Phi"], r["Pi"], r["A"])
        assert abs(M0[i] - m0) <= 1e-12 * m0 and abs(M1[i] - m1) <= 1e-11 * m1, what
