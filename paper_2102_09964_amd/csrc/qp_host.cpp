// Host construction of the quasi-periodic models (the paper's CO2 composite
// kernel, section 5: a periodic kernel times a Matern-3/2, plus a second
// Matern-3/2) for the large-state path.
//
// Periodic factor: sigma^2 exp(-2 sin^2(w0 tau / 2) / ell_p^2) with
// w0 = 2 pi / period equals sigma^2 exp(-a) exp(a cos(w0 tau)),
// a = ell_p^-2. Keeping the Taylor polynomial of degree J of exp(a cos x)
// and expanding the powers of the cosine into harmonics gives the cosine
// series sum_{j<=J} q_j^2 cos(j x) with
//   q_j^2 = c_j exp(-a) sum_{m=0}^{(J-j)/2} (a/2)^(j+2m) / (m! (j+m)!),
// c_0 = 1, c_j = 2 (the truncated series of the modified Bessel functions
// 2 I_j(a)). Harmonic j is an undamped oscillator (two states, rotation
// generator of rate j w0, stationary covariance q_j^2 I); the product with
// the Matern-3/2 is the Kronecker construction. In the library's
// coordinates every state has unit stationary variance: the Matern-3/2
// states are (f, f' / lam), lam = sqrt(3) / ell, and harmonic j's states are
// divided by sigma q_j; the observation row then carries sigma q_j at the
// first state of harmonic j and sigma_a at the additive Matern's first state.
//
// The model's state (what pssgp_model_matrices and pssgp_state_basis
// describe) is harmonic j at 4 j .. 4 j + 3 (state 2 c + r) and the additive
// Matern at 4 (J + 1), 4 (J + 1) + 1. The kernels propagate the 4 (J + 1)
// coupled or observed ones only (qp_team.h): harmonic 0's c = 1 pair is
// neither observed nor coupled to the rest.
#include <cmath>
#include <cstring>

#include "../../include/pssgp.h"
#include "model.h"
#include "qp_launch.h"

bool qp_is_model(const pssgp_model *spec)
{
    return spec && spec->n_comp >= 1 && spec->comp[0].kind == PSSGP_QUASIPERIODIC;
}

static bool positive(double x) { return x > 0.0 && std::isfinite(x); }

int qp_build(const pssgp_model *spec, QPDev *out, double *tdiag)
{
    if (!spec) {
        pssgp_set_error("model is NULL");
        return PSSGP_EINVAL;
    }
    const pssgp_component &p = spec->comp[0];
    if (spec->n_comp < 1 || spec->n_comp > 2 || p.kind != PSSGP_QUASIPERIODIC) {
        pssgp_set_error("quasi-periodic model: component 0 quasi-periodic, optionally component 1 Matern-3/2");
        return PSSGP_EUNSUPPORTED;
    }
    if (p.order < 1 || p.order > QP_MAXJ) {
        pssgp_set_error("quasi-periodic model: %d harmonics beyond the constant; 1..%d are compiled in", p.order,
                        QP_MAXJ);
        return PSSGP_EUNSUPPORTED;
    }
    if (spec->n_comp != 2 || spec->comp[1].kind != PSSGP_MATERN32) {
        pssgp_set_error("quasi-periodic model: the compiled layouts add one Matern-3/2 component (component 1)");
        return PSSGP_EUNSUPPORTED;
    }
    const pssgp_component &a = spec->comp[1];
    if (!positive(p.lengthscale) || !positive(p.variance) || !positive(p.period) || !positive(p.lengthscale2) ||
        !positive(a.lengthscale) || !positive(a.variance) || !positive(spec->noise_var)) {
        pssgp_set_error("quasi-periodic model: length-scales, variances, period and noise_var must be positive and "
                        "finite");
        return PSSGP_EMODEL;
    }
    const int J = p.order;
    const int d = 4 * (J + 1) + 2;
    if (!out && !tdiag) return d;
    QPDev m;
    std::memset(&m, 0, sizeof(m));
    m.J = J;
    m.d = d;
    m.w0 = 2.0 * M_PI / p.period;
    m.lam_m = std::sqrt(3.0) / p.lengthscale2;
    m.lam_a = std::sqrt(3.0) / a.lengthscale;
    m.R = spec->noise_var;
    const double ia = 1.0 / (p.lengthscale * p.lengthscale);
    double fact[2 * QP_MAXJ + 2];
    fact[0] = 1.0;
    for (int i = 1; i < 2 * QP_MAXJ + 2; i++) fact[i] = fact[i - 1] * i;
    const double sd = std::sqrt(p.variance), sa = std::sqrt(a.variance);
    for (int j = 0; j <= J; j++) {
        double acc = 0.0;
        for (int mm = 0; j + 2 * mm <= J; mm++) acc += std::pow(0.5 * ia, j + 2 * mm) / (fact[mm] * fact[j + mm]);
        const double q2 = (j == 0 ? 1.0 : 2.0) * std::exp(-ia) * acc;
        m.hq[j] = sd * std::sqrt(q2);
        if (tdiag)
            for (int c = 0; c < 2; c++) {
                tdiag[4 * j + 2 * c] = m.hq[j];
                tdiag[4 * j + 2 * c + 1] = m.hq[j] * m.lam_m;
            }
    }
    m.ha = sa;
    if (tdiag) {
        tdiag[4 * (J + 1)] = sa;
        tdiag[4 * (J + 1) + 1] = sa * m.lam_a;
    }
    // propagated states: observed rows 0 (harmonic 0), 2 (additive), 4 j
    m.h[0] = m.hq[0];
    m.h[2] = sa;
    for (int j = 1; j <= J; j++) m.h[4 * j] = m.hq[j];
    for (int i = 0; i < 4 * (J + 1); i++) m.u[i] = (i == 0) ? 0.0 : m.h[i] / m.h[0];
    if (out) *out = m;
    return d;
}

void qp_matrices(const QPDev &m, double *G, double *Pinf, double *H)
{
    const int d = m.d, hb = 4 * (m.J + 1);
    for (int i = 0; i < d; i++) {
        if (H) H[i] = (i == hb) ? m.ha : ((i & 3) == 0 && i < hb) ? m.hq[i >> 2] : 0.0;
        for (int j = 0; j < d; j++) {
            if (Pinf) Pinf[i * d + j] = (i == j) ? 1.0 : 0.0;
            if (G) G[i * d + j] = 0.0;
        }
    }
    if (!G) return;
    // Matern-3/2 generator in (f, f' / lam): lam [[0, 1], [-1, -2]]
    auto matern = [&](int off, double lam) {
        G[off * d + off + 1] += lam;
        G[(off + 1) * d + off] += -lam;
        G[(off + 1) * d + off + 1] += -2.0 * lam;
    };
    for (int j = 0; j <= m.J; j++) {
        const int b = 4 * j;
        for (int c = 0; c < 2; c++) matern(b + 2 * c, m.lam_m);
        // rotation generator (x) I_2: [[0, -j w0], [j w0, 0]]
        for (int r = 0; r < 2; r++) {
            G[(b + r) * d + b + 2 + r] = -j * m.w0;
            G[(b + 2 + r) * d + b + r] = j * m.w0;
        }
    }
    matern(hb, m.lam_a);
}
