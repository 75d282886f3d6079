"""The scan readings the GPU path relies on, checked in numpy against the
sequential oracle (CPU only).

* Proposition 1 (supplement): folding the filter elements with the paper's
  operator from the first step reproduces the Kalman filter, including the
  missing-measurement elements of section 3 and the first-step reading.
* The operator is associative (the premise of the parallel scan).
* The per-step fold used inside a GPU thread (a Kalman filter run for an
  unknown start state: predict A, b, C through F and Q, condition on y, and
  add the information of y about the start state to eta, J) equals the
  paper's operator applied to a raw element.
* Proposition 2: the backward smoother scan reproduces the RTS smoother.
* The reverse-mode adjoint recursion of the log-likelihood (our derivation)
  composes associatively and, contracted with the parameter derivatives in
  length-scale-normalised coordinates, gives the oracle's forward-mode
  gradient.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import elements as el
from oracle.model import MATERN12, MATERN32, MATERN52, RBF, OracleModel

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _series(comps, n=120, missing=0.3, seed=0, gap="uniform"):
    w = workloads.random_series(n, comps, 0.01, missing=missing, span=6.0, gap=gap, seed=seed)
    return w["t"], w["y"], w["mask"]


def _raw_filter_elements(m, t, y, mask):
    out = []
    for k in range(t.shape[0]):
        if k == 0:
            F, Q = np.zeros((m.d, m.d)), m.Pinf
        else:
            F, Q = oracle.discretize(m, t[k] - t[k - 1])
        out.append(el.filter_element(F, Q, m.H, m.noise_var, y[k], bool(mask[k])))
    return out


def _rand_element(rng, d):
    A = rng.normal(size=(d, d)) / np.sqrt(d)
    X = rng.normal(size=(d, d))
    C = X @ X.T / d + 0.1 * np.eye(d)
    Y = rng.normal(size=(d, 2))
    J = Y @ Y.T
    return (A, rng.normal(size=d), C, rng.normal(size=d), J)


@pytest.mark.parametrize("d", [1, 2, 3, 6])
def test_filter_operator_associative(d):
    rng = np.random.default_rng(d)
    for _ in range(10):
        a, b, c = (_rand_element(rng, d) for _ in range(3))
        l = el.filter_combine(el.filter_combine(a, b), c)
        r = el.filter_combine(a, el.filter_combine(b, c))
        for x, z in zip(l, r):
            assert np.max(np.abs(x - z)) <= 1e-10 * max(1.0, np.max(np.abs(x)))


@pytest.mark.parametrize("comps", [[(MATERN32, 0, 0.5, 1.0)], [(MATERN52, 0, 1.0, 1.0)],
                                   [(RBF, 6, 1.0, 1.0)], [(MATERN12, 0, 0.4, 1.0), (MATERN32, 0, 1.0, 0.5)]])
@pytest.mark.parametrize("first_observed", [True, False])
def test_proposition1_sequential_fold_is_kalman_filter(comps, first_observed):
    t, y, mask = _series(comps)
    mask = mask.copy()
    mask[0] = 1 if first_observed else 0
    m = OracleModel(comps, 0.01)
    r = oracle.run(m, t, y, mask, smoother=False)
    raw = _raw_filter_elements(m, t, y, mask)
    acc = raw[0]
    assert np.max(np.abs(acc[0])) == 0.0  # A_1 = 0
    for k in range(t.shape[0]):
        if k > 0:
            acc = el.filter_combine(acc, raw[k])
        assert np.max(np.abs(acc[0])) <= 1e-12  # every prefix has A* = 0
        assert np.max(np.abs(acc[1] - r["mf"][k])) <= 1e-9 * max(1.0, np.max(np.abs(r["mf"][k])))
        assert np.max(np.abs(acc[2] - r["Pf"][k])) <= 1e-9 * np.max(np.abs(r["Pf"][k]))


def _fold_raw(acc, F, Q, H, R, y, observed):
    """Per-step fold of a chunk aggregate with a raw element."""
    A, b, C, eta, J = acc
    A1, b1, C1 = F @ A, F @ b, F @ C @ F.T + Q
    if not observed:
        return (A1, b1, C1, eta, J)
    S = H @ C1 @ H + R
    K = C1 @ H / S
    r = y - H @ b1
    v = A1.T @ H
    return (A1 - np.outer(K, v), b1 + K * r, C1 - S * np.outer(K, K), eta + v * r / S, J + np.outer(v, v) / S)


@pytest.mark.parametrize("comps", [[(MATERN52, 0, 1.0, 1.0)], [(RBF, 6, 1.0, 1.0)]])
def test_chunk_fold_equals_operator(comps):
    t, y, mask = _series(comps, n=60, seed=4)
    m = OracleModel(comps, 0.01)
    raw = _raw_filter_elements(m, t, y, mask)
    for start in [0, 1, 13, 40]:
        d = m.d
        acc = (np.eye(d), np.zeros(d), np.zeros((d, d)), np.zeros(d), np.zeros((d, d)))  # identity
        ref = None
        for k in range(start, start + 20):
            F, Q = (np.zeros((d, d)), m.Pinf) if k == 0 else oracle.discretize(m, t[k] - t[k - 1])
            acc = _fold_raw(acc, F, Q, m.H, m.noise_var, y[k], bool(mask[k]))
            ref = raw[k] if ref is None else el.filter_combine(ref, raw[k])
            for x, z in zip(acc, ref):
                assert np.max(np.abs(x - z)) <= 1e-9 * max(1.0, np.max(np.abs(z)))


@pytest.mark.parametrize("comps", [[(MATERN32, 0, 0.5, 1.0)], [(RBF, 6, 1.0, 1.0)],
                                   [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]])
def test_proposition2_backward_scan_is_rts(comps):
    t, y, mask = _series(comps, seed=2)
    m = OracleModel(comps, 0.01)
    r = oracle.run(m, t, y, mask)
    n = t.shape[0]
    elems = []
    for k in range(n):
        if k == n - 1:
            elems.append(el.smoother_element(None, None, r["mf"][k], r["Pf"][k], True))
        else:
            F, Q = oracle.discretize(m, t[k + 1] - t[k])
            elems.append(el.smoother_element(F, Q, r["mf"][k], r["Pf"][k], False))
    acc = elems[-1]
    for k in range(n - 1, -1, -1):
        if k < n - 1:
            acc = el.smoother_combine(elems[k], acc)
        assert np.max(np.abs(acc[0])) <= 1e-300  # every suffix has E* = 0
        assert np.max(np.abs(acc[1] - r["ms"][k])) <= 1e-9 * max(1.0, np.max(np.abs(r["ms"][k])))
        assert np.max(np.abs(acc[2] - r["Ps"][k])) <= 1e-9 * np.max(np.abs(r["Ps"][k]))
    # associativity of the smoother operator on a few triples
    for k in range(0, n - 3, 17):
        a, b, c = elems[k], elems[k + 1], elems[k + 2]
        l = el.smoother_combine(el.smoother_combine(a, b), c)
        rr = el.smoother_combine(a, el.smoother_combine(b, c))
        for x, z in zip(l, rr):
            assert np.max(np.abs(x - z)) <= 1e-11 * max(1.0, np.max(np.abs(z)))


def _normaliser(comps):
    """x_canonical = N x_normalised, N = diag(1, 1/ell, 1/ell^2, ...) per
    component: in these coordinates G = G_1 / ell and Pinf = var * Pinf_1."""
    diag = []
    for kind, order, ell, var in comps:
        dc = {MATERN12: 1, MATERN32: 2, MATERN52: 3}.get(kind, order)
        diag += [ell ** (-j) for j in range(dc)]
    return np.array(diag)


@pytest.mark.parametrize("comps", [[(MATERN32, 0, 0.5, 1.0)], [(MATERN52, 0, 0.8, 1.3)],
                                   [(RBF, 6, 1.0, 1.0)], [(MATERN32, 0, 2.0, 0.5), (RBF, 6, 0.5, 0.5)]])
def test_adjoint_recursion_gives_oracle_gradient(comps):
    noise = 0.01
    t, y, mask = _series(comps, n=150, missing=0.2, seed=6, gap="exponential")
    m = OracleModel(comps, noise, with_derivatives=True)
    g_ref = oracle.run(m, t, y, mask, gradient=True, smoother=False)["grad"]
    Nv = _normaliser(comps)
    Ni = 1.0 / Nv
    Pn = Ni[:, None] * m.Pinf * Ni[None, :]
    Gn = Ni[:, None] * m.G * Nv[None, :]
    d, n = m.d, t.shape[0]
    H = m.H * Nv
    # block generators at ell = 1 and block masks
    blocks, o = [], 0
    for kind, order, ell, var in comps:
        dc = {MATERN12: 1, MATERN32: 2, MATERN52: 3}.get(kind, order)
        Gh = np.zeros((d, d))
        Gh[o:o + dc, o:o + dc] = Gn[o:o + dc, o:o + dc] * ell
        sel = np.zeros((d, d))
        sel[o:o + dc, o:o + dc] = 1.0
        blocks.append((Gh, sel, ell, var))
        o += dc
    # the normalised generator of each block does not depend on ell
    for Gh, sel, ell, var in blocks:
        m2 = OracleModel([(c[0], c[1], c[2] * 1.7, c[3]) for c in comps], noise)
        Nv2 = _normaliser([(c[0], c[1], c[2] * 1.7, c[3]) for c in comps])
        Gn2 = (1.0 / Nv2)[:, None] * m2.G * Nv2[None, :]
        assert np.allclose(Gh, Gn2 * sel * ell * 1.7, rtol=1e-12, atol=1e-12)
    # forward filter in normalised coordinates, keeping what the adjoint needs
    mcur, Pcur = np.zeros(d), np.zeros((d, d))
    rec = []
    for k in range(n):
        if k == 0:
            F, Q = np.zeros((d, d)), Pn
        else:
            Fc, Qc = oracle.discretize(m, t[k] - t[k - 1])
            F, Q = Ni[:, None] * Fc * Nv[None, :], Ni[:, None] * Qc * Ni[None, :]
        mu, Pi = F @ mcur, F @ Pcur @ F.T + Q
        if mask[k]:
            S = H @ Pi @ H + noise
            K = Pi @ H / S
            v = y[k] - H @ mu
            mcur, Pcur = mu + K * v, Pi - S * np.outer(K, K)
        else:
            S, K, v = 1.0, np.zeros(d), 0.0
            mcur, Pcur = mu, Pi
        rec.append((F, Q, mu, Pi, S, K, v, bool(mask[k])))
    # reverse sweep
    mb, Pb = np.zeros(d), np.zeros((d, d))
    grad = np.zeros(len(g_ref))
    for k in range(n - 1, -1, -1):
        F, Q, mu, Pi, S, K, v, obs = rec[k]
        if obs:
            A = np.eye(d) - np.outer(K, H)
            mub = A.T @ mb + H * v / S
            w = A.T @ mb
            Pib = A.T @ Pb @ A + (v / S) * 0.5 * (np.outer(w, H) + np.outer(H, w)) \
                - 0.5 * (1.0 / S - v * v / S ** 2) * np.outer(H, H)
            grad[-1] += K @ Pb @ K - (v / S) * (K @ mb) - 0.5 * (1.0 / S - v * v / S ** 2)
        else:
            mub, Pib = mb, Pb
        for c, (Gh, sel, ell, var) in enumerate(blocks):
            if k > 0:
                cfac = -(t[k] - t[k - 1]) / ell ** 2
                grad[2 * c] += cfac * (mub @ Gh @ mu + 2.0 * np.sum(Pib * (Gh @ (Pi - Pn)).T))
                grad[2 * c + 1] += np.sum(Pib * (Q * sel)) / var
            else:
                grad[2 * c + 1] += np.sum(Pib * (Pn * sel)) / var
        new_mb, new_Pb = F.T @ mub, F.T @ Pib @ F
        # the adjoint element reproduces the same map
        e = el.adjoint_element(F, K, H, S, v, obs)
        am, aP = el.adjoint_apply(e, mb, Pb)
        assert np.allclose(am, new_mb, rtol=1e-10, atol=1e-10 * max(1.0, np.max(np.abs(new_mb))))
        assert np.allclose(aP, new_Pb, rtol=1e-10, atol=1e-10 * max(1.0, np.max(np.abs(new_Pb))))
        mb, Pb = new_mb, new_Pb
    assert np.max(np.abs(grad - g_ref)) <= 1e-8 * np.max(np.abs(g_ref)), (grad, g_ref)


def test_adjoint_composition_associative_and_consistent():
    rng = np.random.default_rng(3)
    d = 4
    def rnd():
        E = rng.normal(size=(d, d)) / 2
        g = rng.normal(size=d)
        L = rng.normal(size=(d, d))
        return (E, g, 0.5 * (L + L.T))
    for _ in range(10):
        a, b, c = rnd(), rnd(), rnd()
        l = el.adjoint_combine(el.adjoint_combine(a, b), c)
        r = el.adjoint_combine(a, el.adjoint_combine(b, c))
        for x, z in zip(l, r):
            assert np.allclose(x, z, rtol=1e-12, atol=1e-12)
        mb, Pb = rng.normal(size=d), rng.normal(size=(d, d))
        Pb = 0.5 * (Pb + Pb.T)
        m1, P1 = el.adjoint_apply(b, mb, Pb)
        m2, P2 = el.adjoint_apply(a, m1, P1)
        m3, P3 = el.adjoint_apply(el.adjoint_combine(a, b), mb, Pb)
        assert np.allclose(m2, m3, rtol=1e-12, atol=1e-12)
        assert np.allclose(P2, P3, rtol=1e-12, atol=1e-12)
