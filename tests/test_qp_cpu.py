"""Host side of the large-state path (quasi-periodic models, d = 10..18),
no GPU needed: the library's model (generator, stationary covariance,
observation row, state basis) against the oracle's independently built
quasi-periodic model, workspace sizing and argument errors."""
import ctypes

import numpy as np
import pytest

from oracle.model import MATERN32, QUASIPERIODIC, OracleModel

import paper_2102_09964_amd as P

CO2 = {J: [(QUASIPERIODIC, J, 1.3, 1.7, 2.5, 4.0), (MATERN32, 0, 0.8, 0.4)] for J in (1, 2, 3)}


@pytest.mark.parametrize("J", [1, 2, 3])
def test_model_matches_oracle(J):
    comps = CO2[J]
    m = P.make_model(comps, 0.02)
    d = P.state_dim(m)
    assert d == 4 * (J + 1) + 2
    T = P.state_basis(m)
    G, Pinf, H = P.model_matrices(m)
    om = OracleModel(comps, 0.02, balance=False)
    # library coordinates z, canonical x = diag(T) z
    Gc = T[:, None] * G / T[None, :]
    Pc = T[:, None] * Pinf * T[None, :]
    Hc = H / T
    assert np.max(np.abs(Gc - om.G)) <= 1e-12 * np.max(np.abs(om.G))
    assert np.max(np.abs(Pc - om.Pinf)) <= 1e-12 * np.max(np.abs(om.Pinf))
    assert np.max(np.abs(Hc - om.H)) <= 1e-15
    # every library state has unit stationary variance
    assert np.array_equal(Pinf, np.eye(d))


def test_workspace_and_argument_errors():
    L = P.lib()
    m = P.make_model(CO2[2], 0.01)
    mp = ctypes.byref(m)
    n = 1000
    wp = P.workspace_bytes(m, n, P.F32, P.OP_PREDICT)
    wl = P.workspace_bytes(m, n, P.F32, P.OP_LOGLIK)
    assert wp > wl > 0
    assert P.workspace_bytes(m, n, P.F64, P.OP_PREDICT) > wp
    assert P.workspace_bytes(m, n, P.F32, P.OP_FILTER) == 0  # not supported for these models
    fake = ctypes.c_void_p(0x1000)
    # workspace too small, NULL outputs, bad chunk
    assert L.pssgp_predict(mp, fake, fake, None, n, P.F32, fake, fake, fake, fake, wp - 1, None, None) == -3
    assert L.pssgp_predict(mp, fake, fake, None, n, P.F32, None, fake, fake, fake, wp, None, None) == -1
    o = P.make_options(chunk=2)
    assert L.pssgp_predict(mp, fake, fake, None, n, P.F32, fake, fake, fake, fake, wp, ctypes.byref(o), None) == -1
    # calls other than predict and loglik are not available for these models
    assert L.pssgp_filter(mp, fake, fake, None, None, n, P.F32, fake, fake, fake, fake, wp, None, None) == -2
    assert b"quasi-periodic" in L.pssgp_last_error()
    assert L.pssgp_loglik(mp, fake, fake, None, fake, n, P.F32, fake, fake, wl, None, None) == -2
    # harmonics outside 1..3, a missing second component, bad hyperparameters
    assert P.lib().pssgp_state_dim(ctypes.byref(P.make_model([(QUASIPERIODIC, 4, 1.0, 1.0, 1.0, 1.0),
                                                               (MATERN32, 0, 1.0, 1.0)], 0.01))) == -2
    assert P.lib().pssgp_state_dim(ctypes.byref(P.make_model([(QUASIPERIODIC, 2, 1.0, 1.0, 1.0, 1.0)], 0.01))) == -2
    assert P.lib().pssgp_state_dim(ctypes.byref(P.make_model([(QUASIPERIODIC, 2, 1.0, 1.0, 0.0, 1.0),
                                                               (MATERN32, 0, 1.0, 1.0)], 0.01))) == -6
