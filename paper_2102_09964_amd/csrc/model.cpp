// Host construction of the device model constants (FP64, O(1) in the number
// of steps: stage 1 of the paper's complexity list, section 4.4).
//
// Per component, at unit length-scale and unit variance:
//  * Matern-nu, d = nu + 1/2, lam = sqrt(2 nu): G1 is the companion matrix
//    of (s + lam)^d; the stationary covariance has the textbook closed form
//    (d = 1: [1]; d = 2: diag(1, lam^2); d = 3: [[1, 0, -k], [0, k, 0],
//    [-k, 0, lam^4]] with k = lam^2 / 3).
//  * RBF, Taylor order n (paper section 5.1: "approximated to the 6th
//    order"): G1 is the companion matrix of the monic polynomial whose
//    roots are the left-half-plane roots of T_n(-u^2 / 2), T_n the degree-n
//    Taylor polynomial of exp; the white-noise density is
//    sqrt(2 pi) 2^n n!. Roots by the Aberth-Ehrlich iteration. The
//    stationary covariance solves the Lyapunov equation of section 4.1,
//    here in the eigenbasis of G1 (the eigenvectors of a companion matrix
//    are Vandermonde columns), where it decouples entrywise.
// Then an Osborne radix-2 balancing D of G1 (section 4.2; the paper treats
// D as a constant in the gradient, which is exact here since G1 does not
// depend on the hyperparameters), normalised so that H keeps its unit
// entry, and the expansion matrices of exp(s G1) described in model.h.
#include "model.h"

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/pssgp.h"

namespace {

thread_local char g_err[512] = "no error";

using cd = std::complex<double>;

struct Comp {
    int kind, order, dim;
    double ell, var;
    double G1[PSSGP_MAXD * PSSGP_MAXD];  // balanced, unit length-scale
    double P1[PSSGP_MAXD * PSSGP_MAXD];  // balanced, unit variance
    double D[PSSGP_MAXD];                // balancing (canonical-normalised = D * balanced)
    double lam;
    int npair, nreal;
    double alpha[PSSGP_MAXRT], beta[PSSGP_MAXRT];
    std::vector<double> M;               // dim expansion matrices, dim*dim each
};

int comp_dim(int kind, int order)
{
    switch (kind) {
    case PSSGP_MATERN12: return 1;
    case PSSGP_MATERN32: return 2;
    case PSSGP_MATERN52: return 3;
    case PSSGP_RBF: return order;
    default: return -1;
    }
}

// Roots of sum_k a[k] u^k (a[deg] != 0) by the Aberth-Ehrlich
// simultaneous iteration, followed by Newton polishing.
std::vector<cd> poly_roots(const std::vector<double> &a)
{
    const int deg = (int)a.size() - 1;
    auto eval = [&](cd z, cd &dp) {
        cd p = a[deg];
        dp = 0.0;
        for (int k = deg - 1; k >= 0; k--) {
            dp = dp * z + p;
            p = p * z + a[k];
        }
        return p;
    };
    // Cauchy bound on the root moduli
    double bound = 0.0;
    for (int k = 0; k < deg; k++) bound = std::fmax(bound, std::fabs(a[k] / a[deg]));
    bound += 1.0;
    std::vector<cd> z(deg);
    for (int i = 0; i < deg; i++)
        z[i] = std::polar(0.5 * bound, 2.0 * M_PI * (i + 0.25) / deg + 0.3);
    for (int it = 0; it < 500; it++) {
        double worst = 0.0;
        for (int i = 0; i < deg; i++) {
            cd dp;
            cd p = eval(z[i], dp);
            if (std::abs(p) == 0.0) continue;
            cd ratio = p / dp;
            cd s = 0.0;
            for (int j = 0; j < deg; j++)
                if (j != i) s += 1.0 / (z[i] - z[j]);
            cd w = ratio / (1.0 - ratio * s);
            z[i] -= w;
            worst = std::fmax(worst, std::abs(w) / std::fmax(1.0, std::abs(z[i])));
        }
        if (worst < 1e-16) break;
    }
    for (int i = 0; i < deg; i++)
        for (int it = 0; it < 3; it++) {
            cd dp;
            cd p = eval(z[i], dp);
            if (std::abs(dp) > 0.0) z[i] -= p / dp;
        }
    return z;
}

// Complex Gauss-Jordan inverse with partial pivoting.
bool cinv(int n, const cd *A, cd *Ainv)
{
    cd a[PSSGP_MAXD * PSSGP_MAXD * 2];
    const int w = 2 * n;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < w; j++) a[i * w + j] = (j < n) ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (std::abs(a[r * w + c]) > std::abs(a[p * w + c])) p = r;
        if (std::abs(a[p * w + c]) == 0.0) return false;
        if (p != c)
            for (int j = 0; j < w; j++) std::swap(a[p * w + j], a[c * w + j]);
        cd piv = a[c * w + c];
        for (int j = 0; j < w; j++) a[c * w + j] /= piv;
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            cd f = a[r * w + c];
            if (f == 0.0) continue;
            for (int j = 0; j < w; j++) a[r * w + j] -= f * a[c * w + j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = a[i * w + n + j];
    return true;
}

// Osborne balancing with powers of two: scale factors D such that
// D^-1 A D has comparable off-diagonal row and column sums.
void balance_radix2(int n, const double *A_in, double *D)
{
    double A[PSSGP_MAXD * PSSGP_MAXD];
    std::memcpy(A, A_in, sizeof(double) * n * n);
    for (int i = 0; i < n; i++) D[i] = 1.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        bool moved = false;
        for (int i = 0; i < n; i++) {
            double col = 0.0, row = 0.0;
            for (int j = 0; j < n; j++)
                if (j != i) { col += std::fabs(A[j * n + i]); row += std::fabs(A[i * n + j]); }
            if (col == 0.0 || row == 0.0) continue;
            const double before = col + row;
            double f = 1.0;
            while (col * 2.0 < row) { col *= 2.0; row *= 0.5; f *= 2.0; }
            while (col > row * 2.0) { col *= 0.5; row *= 2.0; f *= 0.5; }
            if (col + row < 0.95 * before) {
                D[i] *= f;
                for (int j = 0; j < n; j++) { A[j * n + i] *= f; A[i * n + j] /= f; }
                moved = true;
            }
        }
        if (!moved) break;
    }
}

int build_component(const pssgp_component &spec, Comp &c)
{
    c.kind = spec.kind;
    c.order = spec.order;
    c.dim = comp_dim(spec.kind, spec.order);
    c.ell = spec.lengthscale;
    c.var = spec.variance;
    const int d = c.dim;
    double G[PSSGP_MAXD * PSSGP_MAXD] = {0}, P[PSSGP_MAXD * PSSGP_MAXD] = {0};
    double coef[PSSGP_MAXD];  // monic characteristic polynomial, low to high
    std::vector<cd> eig;
    if (spec.kind != PSSGP_RBF) {
        const double nu = d - 0.5;
        c.lam = std::sqrt(2.0 * nu);
        // (s + lam)^d
        double binom = 1.0;
        for (int j = 0; j <= d; j++) {
            if (j < d) coef[j] = binom * std::pow(c.lam, d - j);
            binom = binom * (d - j) / (j + 1);
        }
        const double l2 = c.lam * c.lam;
        if (d == 1) {
            P[0] = 1.0;
        } else if (d == 2) {
            P[0] = 1.0; P[3] = l2;
        } else {
            const double k = l2 / 3.0;
            P[0] = 1.0; P[2] = -k; P[4] = k; P[6] = -k; P[8] = l2 * l2;
        }
        c.npair = c.nreal = 0;
    } else {
        const int n = d;
        std::vector<double> a(2 * n + 1, 0.0);
        double fact = 1.0;
        for (int k = 0; k <= n; k++) {
            if (k > 0) fact *= k;
            a[2 * k] = std::pow(-0.5, k) / fact;
        }
        std::vector<cd> r = poly_roots(a);
        std::vector<cd> pairs, reals;
        for (auto &z : r) {
            if (z.real() >= 0.0) continue;
            if (std::fabs(z.imag()) <= 1e-9 * std::abs(z)) reals.push_back(cd(z.real(), 0.0));
            else if (z.imag() > 0.0) pairs.push_back(z);
        }
        if ((int)(2 * pairs.size() + reals.size()) != n) {
            pssgp_set_error("RBF order %d: root finder returned an unexpected spectrum", n);
            return PSSGP_EMODEL;
        }
        c.npair = (int)pairs.size();
        c.nreal = (int)reals.size();
        for (int p = 0; p < c.npair; p++) {
            c.alpha[p] = pairs[p].real();
            c.beta[p] = pairs[p].imag();
            eig.push_back(pairs[p]);
            eig.push_back(std::conj(pairs[p]));
        }
        for (int q = 0; q < c.nreal; q++) {
            c.alpha[c.npair + q] = reals[q].real();
            c.beta[c.npair + q] = 0.0;
            eig.push_back(reals[q]);
        }
        // monic polynomial prod (s - rho)
        std::vector<cd> poly(1, 1.0);
        for (auto &z : eig) {
            std::vector<cd> nxt(poly.size() + 1, 0.0);
            for (size_t i = 0; i < poly.size(); i++) {
                nxt[i + 1] += poly[i];
                nxt[i] -= z * poly[i];
            }
            poly = nxt;
        }
        for (int j = 0; j < n; j++) coef[j] = poly[j].real();
        c.lam = 0.0;
    }
    for (int i = 0; i + 1 < d; i++) G[i * d + i + 1] = 1.0;
    for (int j = 0; j < d; j++) G[(d - 1) * d + j] = -coef[j];

    // modal data of the RBF block: Vandermonde eigenvectors and their inverse
    cd V[PSSGP_MAXD * PSSGP_MAXD], Vi[PSSGP_MAXD * PSSGP_MAXD];
    if (spec.kind == PSSGP_RBF) {
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++) V[i * d + j] = std::pow(eig[j], i);
        if (!cinv(d, V, Vi)) {
            pssgp_set_error("RBF order %d: singular eigenvector matrix", d);
            return PSSGP_EMODEL;
        }
        // Lyapunov in the eigenbasis: X_ij = -q w_i conj(w_j) / (rho_i + conj(rho_j)),
        // w = V^-1 e_d, then P = V X V^H
        double fact = 1.0;
        for (int k = 2; k <= d; k++) fact *= k;
        const double q = std::sqrt(2.0 * M_PI) * std::ldexp(1.0, d) * fact;
        cd X[PSSGP_MAXD * PSSGP_MAXD];
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++)
                X[i * d + j] = -q * Vi[i * d + d - 1] * std::conj(Vi[j * d + d - 1]) /
                               (eig[i] + std::conj(eig[j]));
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++) {
                cd s = 0.0;
                for (int a2 = 0; a2 < d; a2++)
                    for (int b2 = 0; b2 < d; b2++) s += V[i * d + a2] * X[a2 * d + b2] * std::conj(V[j * d + b2]);
                P[i * d + j] = s.real();
            }
        for (int i = 0; i < d; i++)
            for (int j = i + 1; j < d; j++) {
                double s = 0.5 * (P[i * d + j] + P[j * d + i]);
                P[i * d + j] = P[j * d + i] = s;
            }
    }

    // balancing, normalised so that the first state (observed one) is unscaled
    balance_radix2(d, G, c.D);
    const double d0 = c.D[0];
    for (int i = 0; i < d; i++) c.D[i] /= d0;
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            c.G1[i * d + j] = G[i * d + j] * c.D[j] / c.D[i];
            c.P1[i * d + j] = P[i * d + j] / (c.D[i] * c.D[j]);
        }

    // expansion matrices of exp(s G1) in the balanced coordinates
    c.M.assign((size_t)d * d * d, 0.0);
    if (spec.kind != PSSGP_RBF) {
        double Nb[PSSGP_MAXD * PSSGP_MAXD];
        for (int i = 0; i < d * d; i++) Nb[i] = c.G1[i];
        for (int i = 0; i < d; i++) Nb[i * d + i] += c.lam;
        for (int i = 0; i < d; i++) c.M[i * d + i] = 1.0;
        for (int j = 1; j < d; j++)
            for (int a2 = 0; a2 < d; a2++)
                for (int b2 = 0; b2 < d; b2++) {
                    double s = 0.0;
                    for (int k = 0; k < d; k++) s += c.M[(size_t)(j - 1) * d * d + a2 * d + k] * Nb[k * d + b2];
                    c.M[(size_t)j * d * d + a2 * d + b2] = s / j;
                }
    } else {
        // eigen-projector of eigenvalue e (column e of V times row e of V^-1),
        // in balanced coordinates D^-1 (.) D
        auto proj = [&](int e, int a2, int b2) {
            return V[a2 * d + e] * Vi[e * d + b2] * (c.D[b2] / c.D[a2]);
        };
        for (int p = 0; p < c.npair; p++) {
            const int e = 2 * p;  // eig[2p] = alpha + i beta
            for (int a2 = 0; a2 < d; a2++)
                for (int b2 = 0; b2 < d; b2++) {
                    cd w = proj(e, a2, b2);
                    c.M[(size_t)(2 * p) * d * d + a2 * d + b2] = 2.0 * w.real();
                    c.M[(size_t)(2 * p + 1) * d * d + a2 * d + b2] = -2.0 * w.imag();
                }
        }
        for (int q = 0; q < c.nreal; q++) {
            const int e = 2 * c.npair + q;
            for (int a2 = 0; a2 < d; a2++)
                for (int b2 = 0; b2 < d; b2++)
                    c.M[(size_t)(2 * c.npair + q) * d * d + a2 * d + b2] = proj(e, a2, b2).real();
        }
    }
    return PSSGP_OK;
}

}  // namespace

void pssgp_set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

extern "C" const char *pssgp_last_error(void) { return g_err; }

int pssgp_build_devmodel(const pssgp_model *spec, DevModel *out, double *tdiag)
{
    if (!spec) {
        pssgp_set_error("model is NULL");
        return PSSGP_EINVAL;
    }
    if (spec->n_comp < 1 || spec->n_comp > PSSGP_MAXBLK) {
        pssgp_set_error("n_comp = %d: 1 or 2 components are supported", spec->n_comp);
        return PSSGP_EUNSUPPORTED;
    }
    if (!(spec->noise_var > 0.0) || !std::isfinite(spec->noise_var)) {
        pssgp_set_error("noise_var must be positive and finite");
        return PSSGP_EMODEL;
    }
    int d = 0;
    for (int c = 0; c < spec->n_comp; c++) {
        const pssgp_component &cp = spec->comp[c];
        if (cp.kind == PSSGP_QUASIPERIODIC) {
            pssgp_set_error("component %d: quasi-periodic models run through pssgp_predict and pssgp_loglik only", c);
            return PSSGP_EUNSUPPORTED;
        }
        if (cp.kind < PSSGP_MATERN12 || cp.kind > PSSGP_RBF) {
            pssgp_set_error("component %d: unknown kind %d", c, cp.kind);
            return PSSGP_EINVAL;
        }
        if (cp.kind == PSSGP_RBF && (cp.order < 1 || cp.order > 6)) {
            pssgp_set_error("component %d: RBF Taylor order %d outside 1..6", c, cp.order);
            return PSSGP_EUNSUPPORTED;
        }
        if (!(cp.lengthscale > 0.0) || !(cp.variance > 0.0) || !std::isfinite(cp.lengthscale) ||
            !std::isfinite(cp.variance)) {
            pssgp_set_error("component %d: lengthscale and variance must be positive and finite", c);
            return PSSGP_EMODEL;
        }
        d += comp_dim(cp.kind, cp.order);
    }
    if (d > PSSGP_MAXD) {
        pssgp_set_error("state size %d exceeds %d", d, PSSGP_MAXD);
        return PSSGP_EUNSUPPORTED;
    }
    if (!out && !tdiag) return d;
    DevModel m;
    std::memset(&m, 0, sizeof(m));
    m.d = d;
    m.nblk = spec->n_comp;
    m.R = spec->noise_var;
    int off = 0, fc = 0;
    for (int c = 0; c < spec->n_comp; c++) {
        Comp cp;
        int rc = build_component(spec->comp[c], cp);
        if (rc) return rc;
        const int dc = cp.dim;
        DevBlock &b = m.blk[c];
        b.kind = (cp.kind == PSSGP_RBF) ? BLK_RBF : BLK_MATERN;
        b.dim = dc;
        b.off = off;
        b.npair = cp.npair;
        b.nreal = cp.nreal;
        b.fc_off = fc;
        b.comp = c;
        b.ell = cp.ell;
        b.inv_ell = 1.0 / cp.ell;
        b.var = cp.var;
        b.lam = cp.lam;
        for (int r = 0; r < PSSGP_MAXRT; r++) { b.alpha[r] = cp.alpha[r]; b.beta[r] = cp.beta[r]; }
        if (fc + dc * dc * dc > PSSGP_FCOEF) {
            pssgp_set_error("expansion table too large for this model");
            return PSSGP_EUNSUPPORTED;
        }
        for (int i = 0; i < dc * dc * dc; i++) m.fcoef[fc + i] = cp.M[i];
        fc += dc * dc * dc;
        m.H[off] = 1.0;
        for (int i = 0; i < dc; i++)
            for (int j = 0; j < dc; j++) m.Pinf[(off + i) * d + off + j] = cp.var * cp.P1[i * dc + j];
        double gn = 0.0;
        for (int j = 0; j < dc; j++) {
            double col = 0.0;
            for (int i = 0; i < dc; i++) col += std::fabs(cp.G1[i * dc + j]);
            gn = std::fmax(gn, col);
            b.glast[j] = cp.G1[(dc - 1) * dc + j];
            b.gsup[j] = (j + 1 < dc) ? cp.G1[j * dc + j + 1] : 0.0;
        }
        b.gnorm = gn;
        if (tdiag)
            for (int i = 0; i < dc; i++) tdiag[off + i] = cp.D[i] * std::pow(cp.ell, -i);
        off += dc;
    }
    if (out) *out = m;
    return d;
}

void pssgp_layout(const DevModel &m, int *b0, int *b1)
{
    *b0 = m.blk[0].dim;
    *b1 = m.nblk > 1 ? m.blk[1].dim : 0;
}
