/*
 * pssgp -- parallel state-space Gaussian-process regression on MI355X (gfx950).
 *
 * C ABI of libpssgp.so. Implements the method of "Temporal Gaussian Process
 * Regression in Logarithmic Time" (Corenflos, Zhao, Sarkka): a temporal GP
 * with a state-space covariance (section 2, eq. ssmodel) is discretised per
 * time step (section 4.3, eq. ss-gp-formation of the supplement), the Kalman
 * filter is run as a parallel prefix scan over the associative elements
 * (A, b, C, eta, J) with missing measurements (section 3), the RTS smoother
 * as a reverse scan over (E, g, L) (supplement, Proposition 2), and the
 * log-likelihood and its gradient are reduced on the device.
 *
 * Conventions shared by every entry point:
 *  - Return value: 0 on success, a negative PSSGP_E* code on an argument
 *    error (detected on the host, nothing is launched; see
 *    pssgp_last_error()). Faults found in the data on the device (unsorted
 *    times, non-finite inputs, a non-positive innovation variance, a failed
 *    Cholesky factorisation) set bits of the status word in the workspace,
 *    read with pssgp_status().
 *  - Pointers named t, y, mask, noise_k, m, P, f_mean, f_var, F, Q, loglik,
 *    grad, ws and offsets are DEVICE pointers; pssgp_model, pssgp_options
 *    and the small host arrays named *_host are HOST memory. The caller owns
 *    every buffer; the library allocates nothing per call.
 *  - stream is a hipStream_t (NULL = the default stream). Calls are ordered
 *    on that stream and do not synchronise, except pssgp_status().
 *  - Time stamps t are FP64 and non-decreasing (equal times are allowed:
 *    a zero step has F = I, Q = 0). Test points are steps with mask 0
 *    (missing measurement, section 3); y there is ignored and may be NaN.
 *  - dtype selects the scan precision: PSSGP_F32 keeps the discretisation,
 *    the smoother elements, the conditioning on each measurement (the
 *    covariance update, whose subtraction cancels when the noise is small)
 *    and the log-likelihood terms and sums in FP64, and runs the scan
 *    algebra (predictions, combinations, stored moments) in FP32;
 *    PSSGP_F64 runs everything in FP64. y, m, P, f_mean, f_var use dtype.
 *  - State moments are in the library's state coordinates:
 *    x_canonical = diag(T) z with T from pssgp_state_basis(), where the
 *    canonical coordinates are the companion form (f, f', f'', ...) of
 *    each kernel component, concatenated for sums.
 *  - Covariances are stored packed: entry e of the upper triangle in
 *    row-major order ((0,0), (0,1), ..., (0,d-1), (1,1), ...), and arrays of
 *    per-step quantities are entry-major: X[e * n + k].
 *  - The workspace (ws, ws_bytes) must hold pssgp_workspace_bytes() bytes
 *    for the same model, n, dtype, operation and options; its contents
 *    need no initialisation and are scratch after the call, except the
 *    status word.
 *  - Calls that share a workspace must not overlap in time.
 */
#ifndef PSSGP_H
#define PSSGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PSSGP_OK = 0,
    PSSGP_EINVAL = -1,       /* bad argument (NULL pointer, n < 0, bad dtype, ...) */
    PSSGP_EUNSUPPORTED = -2, /* model shape not compiled in (see pssgp_model) */
    PSSGP_EWORKSPACE = -3,   /* workspace too small */
    PSSGP_EDEVICE = -4,      /* HIP runtime error */
    PSSGP_ENODEVICE = -5,    /* no HIP device */
    PSSGP_EMODEL = -6        /* hyperparameters out of range */
};

/* Kernel components (paper section 2: Matern covariances have an exact
 * state-space form; the RBF covariance is approximated in the spectral
 * domain by a Taylor series of the given order, section 5.1 uses order 6;
 * the quasi-periodic component is the periodic covariance times a
 * Matern-3/2, the product in the CO2 experiment of section 5, with the
 * periodic factor in its Taylor-series state-space form). */
enum { PSSGP_MATERN12 = 1, PSSGP_MATERN32 = 2, PSSGP_MATERN52 = 3, PSSGP_RBF = 4, PSSGP_QUASIPERIODIC = 5 };

typedef struct pssgp_component {
    int32_t kind;        /* PSSGP_MATERN12/32/52, PSSGP_RBF or PSSGP_QUASIPERIODIC */
    int32_t order;       /* RBF: Taylor order = state size, 1..6; quasi-periodic: J,
                            the harmonics beyond the constant (Taylor degree of the
                            periodic factor), 1..3; ignored otherwise */
    double lengthscale;  /* > 0; quasi-periodic: length-scale ell_p of the periodic
                            factor sigma^2 exp(-2 sin^2(pi tau / period) / ell_p^2) */
    double variance;     /* > 0 */
    double period;       /* quasi-periodic only: > 0 */
    double lengthscale2; /* quasi-periodic only: > 0, length-scale of the
                            Matern-3/2 factor */
} pssgp_component;

/* Sum of 1 or 2 components, total state size d <= 8 (e.g. Matern-3/2 +
 * RBF order 6 gives d = 8); noise_var > 0 is the measurement noise
 * variance sigma_n^2 of eq. gp-def (a per-step variance can be passed as
 * noise_k instead). Quasi-periodic models: component 0 quasi-periodic with
 * J = order harmonics beyond the constant, component 1 Matern-3/2, state
 * size d = 4 (J + 1) + 2 = 10, 14 or 18; they run through pssgp_predict
 * and pssgp_loglik (the other calls return PSSGP_EUNSUPPORTED). */
typedef struct pssgp_model {
    int32_t n_comp;
    int32_t reserved;
    pssgp_component comp[4];
    double noise_var;
} pssgp_model;

typedef enum { PSSGP_F32 = 0, PSSGP_F64 = 1 } pssgp_dtype;

typedef struct pssgp_options {
    uint32_t chunk;          /* steps per lane, 0 = default (16); 1..64 for FP64
                                scans, 4..64 for FP32 scans (PSSGP_EINVAL
                                otherwise) */
    uint32_t deterministic;  /* accepted for compatibility; every scan combines its
                                partial results in a fixed order, so results are
                                always bitwise reproducible for a given chunk */
    uint32_t reserved[6];    /* zero */
    void *pass_events[8];    /* optional hipEvent_t handles (NULL entries are skipped),
                                recorded on the stream before the fold pass, before
                                the carry pass, before the finish pass and after the
                                finish pass of the call's filter scan (entries 0-3:
                                pssgp_filter, pssgp_loglik, pssgp_loglik_grad,
                                pssgp_predict, the batched filter and batched
                                predict) and smoother scan (entries 0-3 for
                                pssgp_smooth and the batched smoother, entries 4-7
                                for pssgp_predict and the batched predict); for timing
                                the passes. Owned by the caller. */
} pssgp_options;

typedef enum {
    PSSGP_OP_FILTER = 1,
    PSSGP_OP_SMOOTH = 2,
    PSSGP_OP_LOGLIK = 3,
    PSSGP_OP_LOGLIK_GRAD = 4,
    PSSGP_OP_DISCRETIZE = 5,
    PSSGP_OP_PLAIN = 6,
    PSSGP_OP_PREDICT = 7
} pssgp_op;

/* Status word bits set on the device. */
enum {
    PSSGP_STATUS_UNSORTED = 1u,     /* t[k] < t[k-1] */
    PSSGP_STATUS_NONFINITE = 2u,    /* NaN/Inf in t or an observed y */
    PSSGP_STATUS_BAD_S = 4u,        /* innovation variance <= 0 or not finite */
    PSSGP_STATUS_CHOLESKY = 8u      /* smoother: predicted covariance not positive definite */
};

/* Library version (major * 10000 + minor * 100 + patch). */
int pssgp_version(void);

/* Message of the last error returned on this host thread (never NULL). */
const char *pssgp_last_error(void);

/* State size d of the model, or a negative error code. */
int pssgp_state_dim(const pssgp_model *model);

/* Diagonal basis change of the library's state coordinates:
 * x_canonical = diag(tdiag_host) z; tdiag_host has d entries (host). */
int pssgp_state_basis(const pssgp_model *model, double *tdiag_host);

/* The continuous model in the library's state coordinates (host arrays):
 * generator G (d*d row-major), stationary covariance Pinf (d*d) and
 * observation row H (d), i.e. dx/dt = G x + L w, f = H x with
 * G Pinf + Pinf G^T + L Qc L^T = 0 (paper section 2, eq. ssmodel, and
 * section 4.1). Any pointer may be NULL. For inspection and tests; the
 * kernels build the same matrices internally. */
int pssgp_model_matrices(const pssgp_model *model, double *G_host, double *Pinf_host, double *H_host);

/* Bytes of workspace needed by operation op (pssgp_op) for n steps. */
size_t pssgp_workspace_bytes(const pssgp_model *model, int64_t n, pssgp_dtype dtype, int op,
                             const pssgp_options *opts);

/*
 * Discretisation (supplement, eq. ss-gp-formation; paper section 4.3):
 * for every step k >= 1, F[k] = exp((t[k] - t[k-1]) G) and
 * Q[k] = int_0^dt exp(sG) L Qc L^T exp(sG)^T ds, computed in FP64 as
 * Q = Pinf - F Pinf F^T (stationarity). Step 0 has no predecessor and gets
 * F[0] = 0, Q[0] = Pinf, the first filter element of section 3.
 * F: device double[n][d][d] row-major; Q: device double[NS][n] packed
 * entry-major (NS = d(d+1)/2). Workspace: pssgp_workspace_bytes(...,
 * PSSGP_OP_DISCRETIZE) (holds the status word).
 */
int pssgp_discretize(const pssgp_model *model, const double *t, int64_t n, double *F, double *Q,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * Parallel Kalman filter (section 3): builds the elements (A, b, C, eta, J)
 * of every step (missing steps: A = F, b = 0, C = Q, eta = J = 0; observed:
 * supplement proof of Proposition 1; step 0: A = 0), runs the prefix scan
 * with the filtering operator (three stream-ordered passes: per-tile fold,
 * carry scan over the tiles, per-tile finish), and returns the
 * filter means m (device dtype[d][n], entry-major) and covariances P
 * (device dtype[NS][n], packed entry-major): b*_k and C*_k, Proposition 1.
 * m and P may be NULL (log-likelihood only). loglik (device double[1],
 * nullable) receives sum over observed steps of
 * -1/2 (log 2 pi + log S_k + v_k^2 / S_k) with the innovation v_k and its
 * variance S_k (prediction-error decomposition). noise_k (device
 * double[n], nullable) overrides model->noise_var per step (eq. gp-def).
 */
int pssgp_filter(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                 const double *noise_k, int64_t n, pssgp_dtype dtype, void *m, void *P,
                 double *loglik, void *ws, size_t ws_bytes, const pssgp_options *opts,
                 void *stream);

/*
 * Parallel RTS smoother (supplement, eq. smoother and Proposition 2): from
 * the filter moments (m, P) of pssgp_filter, builds (E_k, g_k, L_k)
 * (E_k = P_k F_k^T (F_k P_k F_k^T + Q_k)^-1, g_k = m_k - E_k F_k m_k,
 * L_k = P_k - E_k F_k P_k, last step (0, m, P)), runs the reverse scan
 * (the same three passes in reverse time order) and writes the posterior
 * mean and variance of
 * f = H x at every step (f_mean, f_var: device dtype[n]) -- at the test
 * (missing) steps these are the GP predictions (supplement, Lemma 1). ms,
 * Ps (nullable) receive the full smoothed state moments in the layout of
 * m, P.
 */
int pssgp_smooth(const pssgp_model *model, const double *t, const void *m, const void *P,
                 int64_t n, pssgp_dtype dtype, void *f_mean, void *f_var, void *ms, void *Ps,
                 void *ws, size_t ws_bytes, const pssgp_options *opts, void *stream);

/*
 * Plain FP64 GPU scan (reference point for the fused scans): the same
 * filter, log-likelihood and smoother with every element materialised in
 * HBM in FP64 and a work-efficient (Blelloch) scan, one launch per level of
 * the up-sweep and of the down-sweep (section 3 and supplement
 * Propositions 1-2 in their textbook parallel form). All data FP64: y
 * double[n], m double[d][n], P double[NS][n], f_mean, f_var double[n],
 * loglik double[1]. Workspace: pssgp_workspace_bytes(..., PSSGP_F64,
 * PSSGP_OP_PLAIN, NULL), which holds two element arrays padded to a power
 * of two.
 */
int pssgp_plain_predict(const pssgp_model *model, const double *t, const double *y,
                        const uint8_t *mask, int64_t n, double *m, double *P, double *f_mean,
                        double *f_var, double *loglik, void *ws, size_t ws_bytes, void *stream);

/*
 * Filter, log-likelihood and smoother in one call (section 3 and
 * supplement, Lemma 1; test points are missing steps): f_mean, f_var
 * dtype[n] and loglik double[1] as from pssgp_filter + pssgp_smooth,
 * but the filter builds the smoother element of every step from its own
 * FP64 prediction and hands the elements (and, for d <= 6, each lane's
 * composed smoother aggregate) to the smoother inside the workspace, in a
 * layout where every access of a wave is contiguous, instead of writing m
 * and P. Workspace: pssgp_workspace_bytes(..., PSSGP_OP_PREDICT, opts);
 * the same opts (chunk) must be passed. Errors as pssgp_filter.
 */
int pssgp_predict(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask, int64_t n,
                  pssgp_dtype dtype, void *f_mean, void *f_var, double *loglik, void *ws, size_t ws_bytes,
                  const pssgp_options *opts, void *stream);

/* Log-likelihood only: pssgp_filter without state outputs. */
int pssgp_loglik(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                 const double *noise_k, int64_t n, pssgp_dtype dtype, double *loglik, void *ws,
                 size_t ws_bytes, const pssgp_options *opts, void *stream);

/*
 * Log-likelihood and its gradient (the paper differentiates the parallel
 * filter by automatic differentiation, sections 2 and 4.4 item 6; here a
 * hand-written reverse-mode adjoint): a forward filter scan whose finish
 * pass stores the per-step forward quantities (predicted mean and
 * covariance, gain, innovation and its variance) in the workspace, then a
 * reverse scan over the affine adjoint maps (mbar_k, Pbar_k) ->
 * (mbar_{k-1}, Pbar_{k-1}) built from them, whose finish pass contracts the
 * adjoints with the parameter derivatives of F, Q, Pinf and R. grad (device double[2 n_comp
 * + 1]) receives d loglik / d (ell_0, var_0, ell_1, var_1, ..., noise_var).
 * The noise variance is the model's scalar noise_var (see
 * pssgp_loglik_grad_noise for per-step variances).
 */
int pssgp_loglik_grad(const pssgp_model *model, const double *t, const void *y,
                      const uint8_t *mask, int64_t n, pssgp_dtype dtype, double *loglik,
                      double *grad, void *ws, size_t ws_bytes, const pssgp_options *opts,
                      void *stream);

/*
 * pssgp_loglik_grad with heteroscedastic measurements: step k has the
 * noise variance noise_k[k] (device double[n], > 0 at observed steps),
 * fixed data rather than a hyperparameter, and the model's noise_var is
 * not used. grad has the same 2 n_comp + 1 entries; the last one (the
 * derivative with respect to noise_var) is 0. Workspace and errors as for
 * pssgp_loglik_grad; noise_k NULL with n > 0 is PSSGP_EINVAL.
 */
int pssgp_loglik_grad_noise(const pssgp_model *model, const double *t, const void *y,
                            const uint8_t *mask, const double *noise_k, int64_t n, pssgp_dtype dtype,
                            double *loglik, double *grad, void *ws, size_t ws_bytes,
                            const pssgp_options *opts, void *stream);

/*
 * Batched form: n_series independent series concatenated along the time
 * axis, series s occupying steps [offsets[s], offsets[s+1]) (offsets:
 * device int64[n_series + 1], offsets[0] = 0, non-decreasing; offsets_host:
 * the same values in host memory, used to lay out the launch). Series of
 * one state layout form a group: groups_host[g] gives the kernel kind
 * (single-component Matern-1/2, 3/2 or 5/2; lengthscale and variance
 * ignored) and the series range [series_begin, series_end) of group g;
 * n_groups is 1 or 2, the groups are contiguous, cover all series and have
 * ascending state sizes. params: device double[n_series][3], per series
 * (lengthscale, variance, noise_var). One set of scan launches (fold,
 * carry, finish) covers all series: a series start is a filter element with A = 0 (section 3) and a
 * series end a smoother element with E = 0, so both scans restart at series
 * boundaries without segment flags. m: device dtype[d_max][n_total], P:
 * device dtype[NS_max][n_total] (d_max, NS_max of the largest group); a
 * series of state size d uses rows [0, d) of m and the first d(d+1)/2 rows
 * of P in its own packing. loglik: device double[n_series]; an empty
 * series (offsets[s] = offsets[s+1]) gets 0. When the batch holds no steps
 * at all, the per-step arrays (t, y, mask, m, P, f_mean, f_var) may be NULL.
 */
typedef struct pssgp_batch_group {
    pssgp_component kind;
    int64_t series_begin;
    int64_t series_end;
} pssgp_batch_group;

size_t pssgp_batched_workspace_bytes(const pssgp_batch_group *groups_host, int n_groups,
                                     int64_t n_series, const int64_t *offsets_host,
                                     pssgp_dtype dtype, int op, const pssgp_options *opts);

int pssgp_batched_filter(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                         const int64_t *offsets, const int64_t *offsets_host, const double *params,
                         const double *t, const void *y, const uint8_t *mask, pssgp_dtype dtype,
                         void *m, void *P, double *loglik, void *ws, size_t ws_bytes,
                         const pssgp_options *opts, void *stream);

int pssgp_batched_smooth(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                         const int64_t *offsets, const int64_t *offsets_host, const double *params,
                         const double *t, const void *m, const void *P, pssgp_dtype dtype,
                         void *f_mean, void *f_var, void *ws, size_t ws_bytes,
                         const pssgp_options *opts, void *stream);

/*
 * Batched log-likelihood only: pssgp_batched_filter without the moment
 * outputs (m, P not written; they may be NULL). loglik: device
 * double[n_series]. Workspace: pssgp_batched_workspace_bytes(...,
 * PSSGP_OP_LOGLIK, opts). Errors as for pssgp_batched_filter.
 */
int pssgp_batched_loglik(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                         const int64_t *offsets, const int64_t *offsets_host, const double *params,
                         const double *t, const void *y, const uint8_t *mask, pssgp_dtype dtype,
                         double *loglik, void *ws, size_t ws_bytes, const pssgp_options *opts,
                         void *stream);

/*
 * Batched filter and smoother in one call (the batched form of
 * pssgp_predict; sections 3 and 4 with the series boundaries above): the
 * filter's finish pass writes the smoother element of every step into the
 * workspace and the smoother scans those elements, so no moments go to
 * caller memory. y, mask as for pssgp_batched_filter; f_mean, f_var: device
 * dtype[n_total]; loglik: device double[n_series]. Workspace size:
 * pssgp_batched_workspace_bytes(..., PSSGP_OP_PREDICT, opts).
 * opts->pass_events, when set, holds 8 events: the filter's 4, then the
 * smoother's 4. Errors as for pssgp_batched_filter.
 */
int pssgp_batched_predict(const pssgp_batch_group *groups_host, int n_groups, int64_t n_series,
                          const int64_t *offsets, const int64_t *offsets_host, const double *params,
                          const double *t, const void *y, const uint8_t *mask, pssgp_dtype dtype,
                          void *f_mean, void *f_var, double *loglik, void *ws, size_t ws_bytes,
                          const pssgp_options *opts, void *stream);

/*
 * Time grid of a prediction (section 4: test times enter the model as
 * steps without a measurement, the missing-measurement elements of
 * section 3): merges the sorted test times into the sorted training times
 * on the device (merge path over tiles of 2048 outputs). The merge is
 * stable: at equal times training steps precede test steps, and each
 * sequence keeps its own order.
 *  t_train   device double[n_train], non-decreasing
 *  y_train   device dtype[n_train]; may be NULL when y_out is NULL (no
 *            values merged) or n_train is 0
 *  mask_train device uint8[n_train] (1 = observed), or NULL (all observed)
 *  t_test    device double[n_test], non-decreasing
 * Outputs, n_out = n_train + n_test, in merged order:
 *  t_out     device double[n_out]
 *  y_out     device dtype[n_out] or NULL: y_train at training steps, 0 at
 *            test steps
 *  mask_out  device uint8[n_out]: mask_train (or 1) at training steps, 0 at
 *            test steps
 *  test_pos  device int64[n_test] or NULL: the merged index of each test time
 * Output buffers must not overlap the inputs. Needs no workspace. Errors:
 * PSSGP_EINVAL for n < 0, a total beyond 2^42 steps, a bad dtype, or a
 * missing pointer; PSSGP_EDEVICE for a launch failure. Unsorted inputs
 * give an unspecified order (every output is still written once and no
 * access leaves the buffers); the filter calls then report
 * PSSGP_STATUS_UNSORTED.
 */
int pssgp_merge_times(const double *t_train, const void *y_train, const uint8_t *mask_train,
                      int64_t n_train, const double *t_test, int64_t n_test, pssgp_dtype dtype,
                      double *t_out, void *y_out, uint8_t *mask_out, int64_t *test_pos, void *stream);

/* Status word of the most recent call that used workspace ws (read after
 * synchronising stream); bits: PSSGP_STATUS_*. */
int pssgp_status(void *ws, void *stream, uint32_t *bits_host);

/*
 * Plans (HIP graphs). pssgp_plan_create records one call, pssgp_predict
 * (op PSSGP_OP_PREDICT) or pssgp_loglik (op PSSGP_OP_LOGLIK, no per-step
 * noise), with the given arguments into a HIP graph on a stream of its own
 * (validation, planning and the kernel launches happen once, at creation);
 * pssgp_plan_launch replays it on `stream`, stream-ordered, with no other
 * host work; pssgp_plan_destroy releases the graph. The device buffers
 * (t, y, mask, outputs, ws) are bound at creation: a replay reads whatever
 * they hold when it runs (refill them between replays to process new data
 * of the same size) and every replay clears what must start at zero with a
 * kernel of its own (no memset node). Replays of one plan, or of plans that
 * share a workspace, must not overlap. options.pass_events must be NULL.
 * Errors: argument errors as the direct call (nothing is recorded);
 * PSSGP_EDEVICE for a HIP failure during capture or launch. The plan owns
 * its graph; the caller owns every buffer. Creation allocates host memory
 * and graph objects; launches allocate nothing.
 */
typedef struct pssgp_plan pssgp_plan;
int pssgp_plan_create(pssgp_plan **out, int op, const pssgp_model *model, const double *t, const void *y,
                      const uint8_t *mask, int64_t n, pssgp_dtype dtype, void *f_mean, void *f_var,
                      double *loglik, void *ws, size_t ws_bytes, const pssgp_options *opts);
int pssgp_plan_launch(pssgp_plan *plan, void *stream);
int pssgp_plan_destroy(pssgp_plan *plan);

/* Size of the device scratch array behind pssgp_loglik_static (per device). */
#define PSSGP_STATIC_SCRATCH_BYTES (64u << 20)

/*
 * pssgp_loglik without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving or
 * optimisation loops, harnesses that forbid hipMalloc. The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine): its
 * workspace is a device array of PSSGP_STATIC_SCRATCH_BYTES (64 MiB) that the
 * library holds on every device it runs on until the process ends; the
 * array's address on the current device is looked up on the first call on
 * that device. Arguments, layout, result and errors as pssgp_loglik (the
 * same kernels run, so the result equals pssgp_loglik's with the same
 * options), except:
 *  - an input whose workspace (pssgp_workspace_bytes with PSSGP_OP_LOGLIK)
 *    exceeds the scratch returns PSSGP_EWORKSPACE with nothing launched
 *    (about 2^22 steps fit at d <= 6 with chunk 64, 2^20 at d = 8 with
 *    chunk 32);
 *  - the stream must belong to the current device;
 *  - every call on a device shares that device's scratch, which keeps the
 *    last call's contents: calls that overlap on one device (on different
 *    streams, or from several host threads without ordering) race and give
 *    undefined results. Calls ordered on one stream are safe; each call
 *    clears what must start at zero with a kernel (no memset);
 *  - the device status word lives in the shared scratch and is not
 *    readable through pssgp_status; callers that need the status bits use
 *    pssgp_loglik with their own workspace.
 */
int pssgp_loglik_static(const pssgp_model *model, const double *t, const void *y, const uint8_t *mask,
                        const double *noise_k, int64_t n, pssgp_dtype dtype, double *loglik,
                        const pssgp_options *opts, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PSSGP_H */
