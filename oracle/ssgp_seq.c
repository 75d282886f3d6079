/*
 * Sequential state-space GP oracle (SSGP): Kalman filter, RTS smoother,
 * log-likelihood and its gradient, all in FP64 with plain scalar loops.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct
 * reference that the GPU path is checked against. Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it. It
 * shares no code with the GPU library.
 *
 * What it computes (paper: "Temporal Gaussian Process Regression in
 * Logarithmic Time", supplement):
 *  - discretisation of the continuous model dx/dt = G x + L w per step
 *    (eq. ss-gp-formation): F = exp(dt G) and
 *    Q = int_0^dt exp(sG) W exp(sG)^T ds with W = L Qc L^T, evaluated by
 *    Van Loan's block exponential; exp() is scaling-and-squaring with the
 *    degree-13 Pade approximant (Higham 2005).
 *  - Kalman filter with missing measurements (eqs. nomeas, withmeas1):
 *    predict m- = F m, P- = F P F^T + Q; if observed
 *    S = H P- H^T + R, K = P- H^T / S, m = m- + K (y - H m-),
 *    P = P- - K S K^T. The first step starts from m- = 0, P- = Pinf
 *    (the stationary covariance, section 4.1).
 *  - Rauch-Tung-Striebel smoother (eq. smoother).
 *  - log-likelihood by the prediction-error decomposition (the paper says
 *    the parameters are estimated "with standard state-space methods";
 *    this is the standard one):
 *    sum over observed steps of -1/2 (log 2 pi + log S + v^2 / S).
 *  - gradient by forward-mode sensitivities: every parameter's derivative
 *    of (m, P, loglik) is propagated alongside the filter, with dF and dQ
 *    from the derivative of the Van Loan exponential (block-triangular
 *    exponential of [[X, dX], [0, X]]).
 *
 * Layout: matrices are row-major d*d doubles. State outputs are in the
 * basis of the matrices passed in (the caller transforms them).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 18
#define MAXB (4 * MAXD)

/* ---------------------------------------------------------------- linear algebra */

static void mm(int n, const double *a, const double *b, double *c) /* c = a b */
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double s = 0.0;
            for (int k = 0; k < n; k++) s += a[i * n + k] * b[k * n + j];
            c[i * n + j] = s;
        }
}

static void mmt(int n, const double *a, const double *b, double *c) /* c = a b^T */
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double s = 0.0;
            for (int k = 0; k < n; k++) s += a[i * n + k] * b[j * n + k];
            c[i * n + j] = s;
        }
}

static void tmm(int n, const double *a, const double *b, double *c) /* c = a^T b */
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double s = 0.0;
            for (int k = 0; k < n; k++) s += a[k * n + i] * b[k * n + j];
            c[i * n + j] = s;
        }
}

static void symmetrize(int n, double *a)
{
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) {
            double s = 0.5 * (a[i * n + j] + a[j * n + i]);
            a[i * n + j] = s;
            a[j * n + i] = s;
        }
}

/* Solve A X = B in place (B overwritten by X), A n*n, B n*m.
 * Gaussian elimination with partial pivoting. Returns 0, or -1 if singular. */
static int solve(int n, int m, double *a, double *b)
{
    for (int c = 0; c < n; c++) {
        int p = c;
        double best = fabs(a[c * n + c]);
        for (int r = c + 1; r < n; r++)
            if (fabs(a[r * n + c]) > best) { best = fabs(a[r * n + c]); p = r; }
        if (best == 0.0) return -1;
        if (p != c) {
            for (int j = 0; j < n; j++) { double t = a[c * n + j]; a[c * n + j] = a[p * n + j]; a[p * n + j] = t; }
            for (int j = 0; j < m; j++) { double t = b[c * m + j]; b[c * m + j] = b[p * m + j]; b[p * m + j] = t; }
        }
        for (int r = c + 1; r < n; r++) {
            double f = a[r * n + c] / a[c * n + c];
            if (f == 0.0) continue;
            for (int j = c; j < n; j++) a[r * n + j] -= f * a[c * n + j];
            for (int j = 0; j < m; j++) b[r * m + j] -= f * b[c * m + j];
        }
    }
    for (int c = n - 1; c >= 0; c--)
        for (int j = 0; j < m; j++) {
            double s = b[c * m + j];
            for (int k = c + 1; k < n; k++) s -= a[c * n + k] * b[k * m + j];
            b[c * m + j] = s / a[c * n + c];
        }
    return 0;
}

/* Matrix exponential by scaling and squaring with the [13/13] Pade
 * approximant (Higham, SIAM J. Matrix Anal. Appl. 26(4), 2005). */
static int expm(int n, const double *a_in, double *out)
{
    static const double b[14] = {
        64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
        1187353796428800.0, 129060195264000.0, 10559470521600.0,
        670442572800.0, 33522128640.0, 1323241920.0, 40840800.0,
        960960.0, 16380.0, 182.0, 1.0};
    const double theta13 = 5.371920351148152;
    double a[MAXB * MAXB], a2[MAXB * MAXB], a4[MAXB * MAXB], a6[MAXB * MAXB];
    double u[MAXB * MAXB], v[MAXB * MAXB], t1[MAXB * MAXB], t2[MAXB * MAXB];
    int nn = n * n;
    double norm1 = 0.0;
    for (int j = 0; j < n; j++) {
        double s = 0.0;
        for (int i = 0; i < n; i++) s += fabs(a_in[i * n + j]);
        if (s > norm1) norm1 = s;
    }
    int sq = 0;
    if (norm1 > theta13) sq = (int)ceil(log2(norm1 / theta13));
    double scale = ldexp(1.0, -sq);
    for (int i = 0; i < nn; i++) a[i] = a_in[i] * scale;
    mm(n, a, a, a2);
    mm(n, a2, a2, a4);
    mm(n, a4, a2, a6);
    /* U = A [A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I] */
    for (int i = 0; i < nn; i++) t1[i] = b[13] * a6[i] + b[11] * a4[i] + b[9] * a2[i];
    mm(n, a6, t1, t2);
    for (int i = 0; i < nn; i++) t2[i] += b[7] * a6[i] + b[5] * a4[i] + b[3] * a2[i];
    for (int i = 0; i < n; i++) t2[i * n + i] += b[1];
    mm(n, a, t2, u);
    /* V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I */
    for (int i = 0; i < nn; i++) t1[i] = b[12] * a6[i] + b[10] * a4[i] + b[8] * a2[i];
    mm(n, a6, t1, v);
    for (int i = 0; i < nn; i++) v[i] += b[6] * a6[i] + b[4] * a4[i] + b[2] * a2[i];
    for (int i = 0; i < n; i++) v[i * n + i] += b[0];
    /* (V - U) X = (V + U) */
    for (int i = 0; i < nn; i++) { t1[i] = v[i] - u[i]; t2[i] = v[i] + u[i]; }
    if (solve(n, n, t1, t2) != 0) return -1;
    for (int s = 0; s < sq; s++) {
        mm(n, t2, t2, t1);
        memcpy(t2, t1, sizeof(double) * nn);
    }
    memcpy(out, t2, sizeof(double) * nn);
    return 0;
}

/* ---------------------------------------------------------------- discretisation */

/* Van Loan (1978): with X = [[-G, W], [0, G^T]] dt,
 * exp(X) = [[E11, E12], [0, E22]], F = E22^T and Q = F E12. */
static void vanloan_matrix(int d, const double *G, const double *W, double dt, double *X)
{
    int n = 2 * d;
    memset(X, 0, sizeof(double) * n * n);
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            X[i * n + j] = -G[i * d + j] * dt;
            X[i * n + d + j] = W[i * d + j] * dt;
            X[(d + i) * n + d + j] = G[j * d + i] * dt;
        }
}

/* Q is linear in W, so W is scaled to the size of G before exponentiating
 * and Q scaled back: a large W would otherwise force extra squarings and
 * lose accuracy (the result is the same in exact arithmetic). */
static double w_scale(int d, const double *G, const double *W)
{
    double ng = 0.0, nw = 0.0;
    for (int i = 0; i < d * d; i++) { ng += fabs(G[i]); nw += fabs(W[i]); }
    if (nw == 0.0 || ng == 0.0 || nw <= ng) return 1.0;
    return ldexp(1.0, (int)floor(log2(nw / ng)));
}

static int vanloan_step(int d, const double *G, const double *W, double dt, double *F, double *Q)
{
    if (dt == 0.0) {
        for (int i = 0; i < d * d; i++) { F[i] = 0.0; Q[i] = 0.0; }
        for (int i = 0; i < d; i++) F[i * d + i] = 1.0;
        return 0;
    }
    int n = 2 * d;
    double X[4 * MAXD * MAXD], E[4 * MAXD * MAXD], e12[MAXD * MAXD], Ws[MAXD * MAXD];
    const double c = w_scale(d, G, W);
    for (int i = 0; i < d * d; i++) Ws[i] = W[i] / c;
    vanloan_matrix(d, G, Ws, dt, X);
    if (expm(n, X, E) != 0) return -2;
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            F[i * d + j] = E[(d + j) * n + d + i];
            e12[i * d + j] = E[i * n + d + j];
        }
    mm(d, F, e12, Q);
    for (int i = 0; i < d * d; i++) Q[i] *= c;
    symmetrize(d, Q);
    return 0;
}

/* Derivative of (F, Q) along a parameter direction (dG, dW): the
 * derivative of exp(X) along dX is the upper-right block of
 * exp([[X, dX], [0, X]]) (Van Loan 1978, Theorem 1). */
static int vanloan_step_deriv(int d, const double *G, const double *W, const double *dG,
                              const double *dW, double dt, double *F, double *Q,
                              double *dF, double *dQ)
{
    if (dt == 0.0) {
        for (int i = 0; i < d * d; i++) { F[i] = 0.0; Q[i] = 0.0; dF[i] = 0.0; dQ[i] = 0.0; }
        for (int i = 0; i < d; i++) F[i * d + i] = 1.0;
        return 0;
    }
    int n = 2 * d, nb = 4 * d;
    double X[4 * MAXD * MAXD], dX[4 * MAXD * MAXD];
    double B[MAXB * MAXB], EB[MAXB * MAXB];
    double e12[MAXD * MAXD], de12[MAXD * MAXD], t1[MAXD * MAXD], t2[MAXD * MAXD];
    double Ws[MAXD * MAXD], dGs[MAXD * MAXD], dWs[MAXD * MAXD];
    /* (Q, dQ) are linear in (W, dW) jointly and the derivative block is
     * linear in (dG, dW): both are scaled to the size of G and the results
     * scaled back, as in ssgp_discretize. */
    const double c = w_scale(d, G, W);
    double ng = 0.0, nd = 0.0;
    for (int i = 0; i < d * d; i++) { ng += fabs(G[i]); nd += fabs(dG[i]) + fabs(dW[i]) / c; }
    const double cd = (nd > ng && ng > 0.0) ? ldexp(1.0, (int)floor(log2(nd / ng))) : 1.0;
    for (int i = 0; i < d * d; i++) { Ws[i] = W[i] / c; dGs[i] = dG[i] / cd; dWs[i] = dW[i] / (c * cd); }
    vanloan_matrix(d, G, Ws, dt, X);
    vanloan_matrix(d, dGs, dWs, dt, dX);
    memset(B, 0, sizeof(double) * nb * nb);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            B[i * nb + j] = X[i * n + j];
            B[i * nb + n + j] = dX[i * n + j];
            B[(n + i) * nb + n + j] = X[i * n + j];
        }
    if (expm(nb, B, EB) != 0) return -2;
    /* exp(X) = EB[0:n, 0:n], d exp(X) = EB[0:n, n:2n] */
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            F[i * d + j] = EB[(d + j) * nb + d + i];
            e12[i * d + j] = EB[i * nb + d + j];
            dF[i * d + j] = EB[(d + j) * nb + n + d + i];
            de12[i * d + j] = EB[i * nb + n + d + j];
        }
    for (int i = 0; i < d * d; i++) dF[i] *= cd;
    mm(d, F, e12, Q);
    mm(d, dF, e12, t1);
    mm(d, F, de12, t2);
    for (int i = 0; i < d * d; i++) {
        Q[i] *= c;
        dQ[i] = (t1[i] + t2[i] * cd) * c;
    }
    symmetrize(d, Q);
    symmetrize(d, dQ);
    return 0;
}

/* Long steps are split: with ||G||_1 dt > 1 the interval is halved j times,
 * Van Loan is evaluated on the short piece, and the pieces are composed by
 * the semigroup property of the discrete model,
 *   F(2h) = F(h) F(h),  Q(2h) = F(h) Q(h) F(h)^T + Q(h),
 * which follows from splitting the integral defining Q. Keeping the block
 * exponential's argument small keeps it accurate when exp(-G dt) is large. */
static int n_halvings(int d, const double *G, double dt)
{
    double g = 0.0;
    for (int j = 0; j < d; j++) {
        double s = 0.0;
        for (int i = 0; i < d; i++) s += fabs(G[i * d + j]);
        if (s > g) g = s;
    }
    double x = g * fabs(dt);
    return x > 1.0 ? (int)ceil(log2(x)) : 0;
}

int ssgp_discretize(int d, const double *G, const double *W, double dt, double *F, double *Q)
{
    if (d < 1 || d > MAXD) return -1;
    const int j = n_halvings(d, G, dt);
    int rc = vanloan_step(d, G, W, ldexp(dt, -j), F, Q);
    if (rc) return rc;
    double t1[MAXD * MAXD], t2[MAXD * MAXD];
    for (int r = 0; r < j; r++) {
        mm(d, F, Q, t1);
        mmt(d, t1, F, t2);
        for (int i = 0; i < d * d; i++) Q[i] += t2[i];
        symmetrize(d, Q);
        mm(d, F, F, t1);
        memcpy(F, t1, sizeof(double) * d * d);
    }
    return 0;
}

static int ssgp_discretize_deriv(int d, const double *G, const double *W, const double *dG,
                                 const double *dW, double dt, double *F, double *Q,
                                 double *dF, double *dQ)
{
    const int j = n_halvings(d, G, dt);
    int rc = vanloan_step_deriv(d, G, W, dG, dW, ldexp(dt, -j), F, Q, dF, dQ);
    if (rc) return rc;
    double t1[MAXD * MAXD], t2[MAXD * MAXD], t3[MAXD * MAXD], nQ[MAXD * MAXD], ndQ[MAXD * MAXD];
    const int dd = d * d;
    for (int r = 0; r < j; r++) {
        /* Q' = F Q F^T + Q ; dQ' = dF Q F^T + F Q dF^T + F dQ F^T + dQ */
        mm(d, F, Q, t1);
        mmt(d, t1, F, t2);
        for (int i = 0; i < dd; i++) nQ[i] = t2[i] + Q[i];
        mm(d, dF, Q, t1);
        mmt(d, t1, F, t2);
        mm(d, F, dQ, t1);
        mmt(d, t1, F, t3);
        for (int a = 0; a < d; a++)
            for (int b = 0; b < d; b++)
                ndQ[a * d + b] = t2[a * d + b] + t2[b * d + a] + t3[a * d + b] + dQ[a * d + b];
        /* F' = F F ; dF' = dF F + F dF */
        mm(d, dF, F, t1);
        mm(d, F, dF, t2);
        for (int i = 0; i < dd; i++) dF[i] = t1[i] + t2[i];
        mm(d, F, F, t1);
        memcpy(F, t1, sizeof(double) * dd);
        memcpy(Q, nQ, sizeof(double) * dd);
        memcpy(dQ, ndQ, sizeof(double) * dd);
        symmetrize(d, Q);
        symmetrize(d, dQ);
    }
    return 0;
}

/* ---------------------------------------------------------------- model */

typedef struct {
    int d;
    const double *G;    /* d*d */
    const double *W;    /* d*d, L Qc L^T */
    const double *Pinf; /* d*d */
    const double *H;    /* d */
    double R;           /* noise variance, used when noise_k is NULL */
    int np;             /* number of gradient parameters (0 = no gradient) */
    const double *dG;   /* np*d*d */
    const double *dW;   /* np*d*d */
    const double *dPinf;/* np*d*d */
    const double *dR;   /* np: derivative of the noise variance */
} ssgp_model;

/* One filter step from (m, P) with transition (F, Q); step 0 uses F = 0 and
 * Q = Pinf, i.e. m- = 0, P- = Pinf. Writes the predicted moments and returns
 * the log-likelihood term (0 for a missing step). */
typedef struct {
    double mp[MAXD], Pp[MAXD * MAXD]; /* predicted */
    double S, v, K[MAXD];
} kf_step_info;

static double kf_step(int d, const double *H, double R, int observed, double y,
                      const double *F, const double *Q, double *m, double *P, kf_step_info *info)
{
    double t1[MAXD * MAXD];
    /* predict */
    for (int i = 0; i < d; i++) {
        double s = 0.0;
        for (int j = 0; j < d; j++) s += F[i * d + j] * m[j];
        info->mp[i] = s;
    }
    mm(d, F, P, t1);
    mmt(d, t1, F, info->Pp);
    for (int i = 0; i < d * d; i++) info->Pp[i] += Q[i];
    symmetrize(d, info->Pp);
    memcpy(m, info->mp, sizeof(double) * d);
    memcpy(P, info->Pp, sizeof(double) * d * d);
    if (!observed) { info->S = 0.0; info->v = 0.0; return 0.0; }
    /* update */
    double PHt[MAXD];
    for (int i = 0; i < d; i++) {
        double s = 0.0;
        for (int j = 0; j < d; j++) s += info->Pp[i * d + j] * H[j];
        PHt[i] = s;
    }
    double S = R, hm = 0.0;
    for (int i = 0; i < d; i++) { S += H[i] * PHt[i]; hm += H[i] * info->mp[i]; }
    double v = y - hm;
    for (int i = 0; i < d; i++) info->K[i] = PHt[i] / S;
    for (int i = 0; i < d; i++) m[i] = info->mp[i] + info->K[i] * v;
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) P[i * d + j] = info->Pp[i * d + j] - info->K[i] * S * info->K[j];
    symmetrize(d, P);
    info->S = S;
    info->v = v;
    return -0.5 * (log(2.0 * M_PI) + log(S) + v * v / S);
}

/* Cholesky-based solve of the SPD system A X^T = B^T for X = B A^{-1}
 * (B is d*d, result in X). Returns -1 if A is not positive definite. */
static int right_solve_spd(int d, const double *A, const double *B, double *X)
{
    double Lc[MAXD * MAXD];
    memset(Lc, 0, sizeof(Lc));
    for (int j = 0; j < d; j++) {
        double s = A[j * d + j];
        for (int k = 0; k < j; k++) s -= Lc[j * d + k] * Lc[j * d + k];
        if (!(s > 0.0)) return -1;
        Lc[j * d + j] = sqrt(s);
        for (int i = j + 1; i < d; i++) {
            double r = A[i * d + j];
            for (int k = 0; k < j; k++) r -= Lc[i * d + k] * Lc[j * d + k];
            Lc[i * d + j] = r / Lc[j * d + j];
        }
    }
    /* each row x of X solves A x^T = b^T: forward then backward substitution */
    for (int r = 0; r < d; r++) {
        double z[MAXD];
        for (int i = 0; i < d; i++) {
            double s = B[r * d + i];
            for (int k = 0; k < i; k++) s -= Lc[i * d + k] * z[k];
            z[i] = s / Lc[i * d + i];
        }
        for (int i = d - 1; i >= 0; i--) {
            double s = z[i];
            for (int k = i + 1; k < d; k++) s -= Lc[k * d + i] * X[r * d + k];
            X[r * d + i] = s / Lc[i * d + i];
        }
    }
    return 0;
}

/*
 * Run the sequential filter (always), the smoother (when any smoother output
 * is requested) and the forward-mode gradient (when grad != NULL and np > 0).
 *
 * t[n] non-decreasing; y[n]; mask[n] (1 = observed); noise_k[n] or NULL.
 * Outputs (each nullable):
 *   mf[n*d], Pf[n*d*d]    filter moments
 *   ms[n*d], Ps[n*d*d]    smoother moments
 *   fmean[n], fvar[n]     H ms and H Ps H^T
 *   loglik[1], grad[np]
 * Returns 0 on success, negative on error (-1 bad args, -2 expm failure,
 * -3 out of memory, -4 smoother covariance not positive definite).
 */
int ssgp_run(const ssgp_model *mdl, int64_t n, const double *t, const double *y,
             const uint8_t *mask, const double *noise_k, double *mf, double *Pf,
             double *ms, double *Ps, double *fmean, double *fvar, double *loglik, double *grad)
{
    if (!mdl || n < 0 || mdl->d < 1 || mdl->d > MAXD) return -1;
    const int d = mdl->d, dd = d * d;
    const int np = (grad && mdl->np > 0) ? mdl->np : 0;
    if (np > 16) return -1;
    const int want_smooth = (ms || Ps || fmean || fvar);
    double *fm = mf, *fP = Pf;
    double *own_m = NULL, *own_P = NULL;
    if (want_smooth && (!fm || !fP)) {
        own_m = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * d);
        own_P = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * dd);
        if (!own_m || !own_P) { free(own_m); free(own_P); return -3; }
        if (!fm) fm = own_m;
        if (!fP) fP = own_P;
    }

    double m[MAXD] = {0}, P[MAXD * MAXD] = {0};
    double F[MAXD * MAXD], Q[MAXD * MAXD];
    double dm[16][MAXD], dP[16][MAXD * MAXD];
    memset(dm, 0, sizeof(dm));
    memset(dP, 0, sizeof(dP));
    double ll = 0.0, dll[16] = {0};
    double prev_dt = NAN;
    int rc = 0;

    for (int64_t k = 0; k < n; k++) {
        const int obs = mask ? (mask[k] != 0) : 1;
        const double R = noise_k ? noise_k[k] : mdl->R;
        kf_step_info info;
        double dFk[16][MAXD * MAXD], dQk[16][MAXD * MAXD];
        if (k == 0) {
            memset(F, 0, sizeof(F));
            memcpy(Q, mdl->Pinf, sizeof(double) * dd);
            for (int p = 0; p < np; p++) {
                memset(dFk[p], 0, sizeof(double) * dd);
                memcpy(dQk[p], mdl->dPinf + (size_t)p * dd, sizeof(double) * dd);
            }
        } else {
            const double dt = t[k] - t[k - 1];
            if (np > 0) {
                for (int p = 0; p < np; p++) {
                    rc = ssgp_discretize_deriv(d, mdl->G, mdl->W, mdl->dG + (size_t)p * dd,
                                               mdl->dW + (size_t)p * dd, dt, F, Q, dFk[p], dQk[p]);
                    if (rc) goto done;
                }
            } else if (!(dt == prev_dt)) {
                rc = ssgp_discretize(d, mdl->G, mdl->W, dt, F, Q);
                if (rc) goto done;
                prev_dt = dt;
            }
        }
        /* sensitivities use the moments before the step */
        double m_old[MAXD], P_old[MAXD * MAXD];
        memcpy(m_old, m, sizeof(double) * d);
        memcpy(P_old, P, sizeof(double) * dd);
        ll += kf_step(d, mdl->H, R, obs, y[k], F, Q, m, P, &info);

        for (int p = 0; p < np; p++) {
            /* d m- = dF m + F dm ; d P- = dF P F^T + F dP F^T + F P dF^T + dQ */
            double dmp[MAXD], dPp[MAXD * MAXD], t1[MAXD * MAXD], t2[MAXD * MAXD];
            for (int i = 0; i < d; i++) {
                double s = 0.0;
                for (int j = 0; j < d; j++) s += dFk[p][i * d + j] * m_old[j] + F[i * d + j] * dm[p][j];
                dmp[i] = s;
            }
            mm(d, dFk[p], P_old, t1);
            mmt(d, t1, F, t2); /* dF P F^T */
            for (int i = 0; i < dd; i++) dPp[i] = t2[i];
            for (int i = 0; i < d; i++)
                for (int j = 0; j < d; j++) dPp[i * d + j] += t2[j * d + i]; /* + F P dF^T */
            mm(d, F, dP[p], t1);
            mmt(d, t1, F, t2);
            for (int i = 0; i < dd; i++) dPp[i] += t2[i] + dQk[p][i];
            symmetrize(d, dPp);
            if (obs) {
                const double S = info.S, v = info.v;
                const double dR = (mdl->dR && !noise_k) ? mdl->dR[p] : 0.0;
                double dPHt[MAXD], dS = dR, dv = 0.0;
                for (int i = 0; i < d; i++) {
                    double s = 0.0;
                    for (int j = 0; j < d; j++) s += dPp[i * d + j] * mdl->H[j];
                    dPHt[i] = s;
                }
                for (int i = 0; i < d; i++) { dS += mdl->H[i] * dPHt[i]; dv -= mdl->H[i] * dmp[i]; }
                double dK[MAXD];
                for (int i = 0; i < d; i++) dK[i] = (dPHt[i] - info.K[i] * dS) / S;
                for (int i = 0; i < d; i++) dm[p][i] = dmp[i] + dK[i] * v + info.K[i] * dv;
                for (int i = 0; i < d; i++)
                    for (int j = 0; j < d; j++)
                        dP[p][i * d + j] = dPp[i * d + j] - dK[i] * S * info.K[j]
                                           - info.K[i] * dS * info.K[j] - info.K[i] * S * dK[j];
                symmetrize(d, dP[p]);
                dll[p] += -0.5 * (dS / S + 2.0 * v * dv / S - v * v * dS / (S * S));
            } else {
                memcpy(dm[p], dmp, sizeof(double) * d);
                memcpy(dP[p], dPp, sizeof(double) * dd);
            }
        }
        if (fm) memcpy(fm + (size_t)k * d, m, sizeof(double) * d);
        if (fP) memcpy(fP + (size_t)k * dd, P, sizeof(double) * dd);
    }
    if (loglik) *loglik = ll;
    for (int p = 0; p < np; p++) grad[p] = dll[p];

    if (want_smooth && n > 0) {
        /* RTS backward pass (eq. smoother). */
        double msn[MAXD], Psn[MAXD * MAXD];
        memcpy(msn, fm + (size_t)(n - 1) * d, sizeof(double) * d);
        memcpy(Psn, fP + (size_t)(n - 1) * dd, sizeof(double) * dd);
        for (int64_t k = n - 1; k >= 0; k--) {
            double mk[MAXD], Pk[MAXD * MAXD];
            if (k == n - 1) {
                memcpy(mk, msn, sizeof(double) * d);
                memcpy(Pk, Psn, sizeof(double) * dd);
            } else {
                const double *mfk = fm + (size_t)k * d, *Pfk = fP + (size_t)k * dd;
                const double dt = t[k + 1] - t[k];
                rc = ssgp_discretize(d, mdl->G, mdl->W, dt, F, Q);
                if (rc) goto done;
                double FP[MAXD * MAXD], Pp[MAXD * MAXD], Gk[MAXD * MAXD], mp[MAXD];
                mm(d, F, Pfk, FP);
                mmt(d, FP, F, Pp);
                for (int i = 0; i < dd; i++) Pp[i] += Q[i];
                symmetrize(d, Pp);
                /* G_k = P_k F^T (P-_{k+1})^{-1} = (F P_k)^T (P-)^{-1} */
                double PFt[MAXD * MAXD];
                for (int i = 0; i < d; i++)
                    for (int j = 0; j < d; j++) PFt[i * d + j] = FP[j * d + i];
                if (right_solve_spd(d, Pp, PFt, Gk) != 0) { rc = -4; goto done; }
                for (int i = 0; i < d; i++) {
                    double s = 0.0;
                    for (int j = 0; j < d; j++) s += F[i * d + j] * mfk[j];
                    mp[i] = s;
                }
                double dmv[MAXD], dPm[MAXD * MAXD], t1[MAXD * MAXD], t2[MAXD * MAXD];
                for (int i = 0; i < d; i++) dmv[i] = msn[i] - mp[i];
                for (int i = 0; i < dd; i++) dPm[i] = Psn[i] - Pp[i];
                for (int i = 0; i < d; i++) {
                    double s = 0.0;
                    for (int j = 0; j < d; j++) s += Gk[i * d + j] * dmv[j];
                    mk[i] = mfk[i] + s;
                }
                mm(d, Gk, dPm, t1);
                mmt(d, t1, Gk, t2);
                for (int i = 0; i < dd; i++) Pk[i] = Pfk[i] + t2[i];
                symmetrize(d, Pk);
                memcpy(msn, mk, sizeof(double) * d);
                memcpy(Psn, Pk, sizeof(double) * dd);
            }
            if (ms) memcpy(ms + (size_t)k * d, mk, sizeof(double) * d);
            if (Ps) memcpy(Ps + (size_t)k * dd, Pk, sizeof(double) * dd);
            double hm = 0.0, hph = 0.0;
            for (int i = 0; i < d; i++) {
                hm += mdl->H[i] * mk[i];
                for (int j = 0; j < d; j++) hph += mdl->H[i] * Pk[i * d + j] * mdl->H[j];
            }
            if (fmean) fmean[k] = hm;
            if (fvar) fvar[k] = hph;
        }
    }
done:
    free(own_m);
    free(own_P);
    return rc;
}

/* Exposed for tests: the oracle's own matrix exponential. */
int ssgp_expm(int n, const double *a, double *out)
{
    if (n < 1 || n > MAXB) return -1;
    return expm(n, a, out);
}

/* Batched driver: series s occupies steps [offsets[s], offsets[s+1]) of the
 * concatenated arrays, with its own model. Runs the series one after the
 * other on the calling thread (the Python wrapper spreads series over
 * threads). Outputs as in ssgp_run, at the concatenated positions; loglik
 * per series. */
int ssgp_run_batched(const ssgp_model *mdls, int64_t n_series, const int64_t *offsets,
                     const double *t, const double *y, const uint8_t *mask,
                     double *fmean, double *fvar, double *loglik)
{
    for (int64_t s = 0; s < n_series; s++) {
        int64_t a = offsets[s], b = offsets[s + 1];
        int rc = ssgp_run(&mdls[s], b - a, t + a, y + a, mask ? mask + a : NULL, NULL, NULL, NULL,
                          NULL, NULL, fmean ? fmean + a : NULL, fvar ? fvar + a : NULL,
                          loglik ? loglik + s : NULL, NULL);
        if (rc) return rc;
    }
    return 0;
}

/* Per-step log-likelihood terms of the sequential filter:
 * terms[k] = -1/2 (log 2 pi S_k + v_k^2 / S_k) for an observed step, 0 for
 * a missing one (prediction-error decomposition, as summed by ssgp_run).
 * Their absolute sum is the condition number of the log-likelihood as a
 * sum, used to state its error. Same arguments as ssgp_run. */
int ssgp_loglik_terms(const ssgp_model *mdl, int64_t n, const double *t, const double *y,
                      const uint8_t *mask, const double *noise_k, double *terms)
{
    if (!mdl || n < 0 || mdl->d < 1 || mdl->d > MAXD || (n > 0 && !terms)) return -1;
    const int d = mdl->d, dd = d * d;
    double m[MAXD] = {0}, P[MAXD * MAXD] = {0};
    double F[MAXD * MAXD], Q[MAXD * MAXD];
    for (int64_t k = 0; k < n; k++) {
        const int obs = mask ? (mask[k] != 0) : 1;
        const double R = noise_k ? noise_k[k] : mdl->R;
        kf_step_info info;
        if (k == 0) {
            memset(F, 0, sizeof(F));
            memcpy(Q, mdl->Pinf, sizeof(double) * dd);
        } else {
            int rc = ssgp_discretize(d, mdl->G, mdl->W, t[k] - t[k - 1], F, Q);
            if (rc) return rc;
        }
        terms[k] = kf_step(d, mdl->H, R, obs, y[k], F, Q, m, P, &info);
    }
    return 0;
}
