"""Property-based pins of the oracle (hypothesis, CPU only): on arbitrary tiny inputs the oracle's
prox of lam*R (+ beta*l1) equals the brute-force minimiser of the objective, and its outputs
satisfy the optimality certificate and the invariants the paper states."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
import pins

# FP32-representable weights on a coarse grid or anywhere in a range: ties, zeros and
# near-ties are all reachable
weights = st.lists(st.one_of(st.integers(-6, 6).map(lambda k: k / 4.0),
                             st.floats(-3.0, 3.0, allow_nan=False, width=32)),
                   min_size=1, max_size=5)
lams = st.sampled_from([0.0, 0.01, 0.1, 0.5, 1.0, 3.0])


@settings(max_examples=150, deadline=None)
@given(weights, lams)
def test_prox_equals_brute_force(w, lam):
    w = np.asarray(w, np.float64)
    u, perm, start = oracle.prox_f64(w, lam)
    np.testing.assert_allclose(u, pins.brute_force_prox(w, lam), atol=1e-9 * (1 + np.abs(w).max()))
    ok, msg = pins.kkt_certificate(w, u, lam, 1e-9 * (1 + np.abs(w).max()))
    assert ok, msg
    assert abs(u.sum() - w.sum()) <= 1e-9 * (1 + np.abs(w).sum())
    assert np.all(np.diff(u[np.argsort(w, kind="stable")]) >= -1e-12)


@settings(max_examples=100, deadline=None)
@given(weights, lams, st.sampled_from([0.0, 0.05, 0.3, 1.0]))
def test_prox_l1_equals_brute_force(w, lam, beta):
    w = np.asarray(w, np.float64)
    if w.shape[0] < 2:
        exp = np.sign(w) * np.maximum(np.abs(w) - beta, 0.0)
    else:
        exp = pins.brute_force_prox_l1(w, lam, beta)
    np.testing.assert_allclose(oracle.prox_l1_f64(w, lam, beta, 0.0), exp, atol=1e-9 * (1 + np.abs(w).max()))
