// Host-side launch interface between the C ABI (capi.cpp) and the kernel
// translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "model.h"

// Control block at the start of every workspace.
struct WsCtl {
    uint32_t done;     // tiles finished (last-block reduction)
    uint32_t status;   // PSSGP_STATUS_* bits
    uint32_t pad[62];
};

// Block layouts (state sizes of up to two kernel components) compiled in.
#ifndef PSSGP_LAYOUTS
#define PSSGP_LAYOUTS(X) X(1, 0) X(2, 0) X(3, 0) X(4, 0) X(6, 0) X(2, 6) X(1, 2)
#endif

// Room for the constants of the FP32 transition of one model in the
// workspace, in doubles (8 KB).
#define PSSGP_CONST_DOUBLES 1024

// Workspace pieces of one scan launch (all device pointers).
struct ScanWs {
    WsCtl *ctl;
    void *aggp;      // per-tile aggregates, contiguous (read by the carry pass)
    void *gagg;      // carry pass scratch: aggregates of groups of 64 tiles
    void *gcarry;    // carry pass scratch: moments entering each group
    void *inclp;     // per-tile carries (moments entering the tile)
    void *lanep;     // per-lane inclusive aggregates within the tile
    double *partials;  // per-tile partial sums (loglik, gradient)
    double *cst;       // model constants of the FP32 transition (8 KB per model)
    void *agg2;        // nullable: second buffer of tile aggregates (team carry of the filter)
};

struct FilterLaunch {
    void *const *ev;  // nullable: 4 events around the passes
    const double *t;
    const void *y;
    const uint8_t *mask;
    const double *noise_k;
    int64_t n;
    int chunk;
    int ntiles;
    void *m;         // nullable
    void *P;         // nullable
    double *loglik;  // nullable
    void *rec;       // nullable: per-step records of the adjoint (tile layout)
    int tiled;       // write smoother elements to m (P unused) in the tile layout of the handover
    void *slane;     // tiled: the smoother's lane records, written by the finish (lane_aggregate_handover)
    ScanWs ws;
};

struct SmoothLaunch {
    void *const *ev;  // nullable: 4 events around the passes
    const double *t;
    const void *m;
    const void *P;
    int64_t n;
    int chunk;
    int ntiles;
    void *f_mean;
    void *f_var;
    void *ms;  // nullable
    void *Ps;  // nullable
    int tiled; // m holds the smoother elements in the tile layout (P unused)
    const void *slane;  // tiled: the smoother's lane records written by the filter's finish
    ScanWs ws;
};

struct GradLaunch {
    const double *t;
    const void *y;
    const uint8_t *mask;
    int64_t n;
    int chunk;
    int ntiles;
    const void *rec;    // per-step records written by the forward filter
    int noise_fixed;    // per-step noise variances given: the noise-variance derivative is 0
    double *grad;       // device [2 n_comp + 1]
    ScanWs ws;
};

// Batched form: up to two groups of series sharing a single-component
// Matern layout (d <= 3, ascending d); per group a compact model whose
// covariance constants are for unit variance (the series variance is
// applied per step).
struct BatchModel {
    int32_t d;
    int32_t pad;
    DevBlock blk;
    double Pinf1[9];   // unit-variance stationary covariance, d*d row-major
    double fcoef[27];  // expansion matrices of the block
    double H[3];
};

struct BatchGroup {
    int64_t k_begin, k_end;  // step range of the group
    int64_t s_begin, s_end;  // series range of the group
    int ntiles;
    int slot_base;
};

struct BatchLaunch {
    void *const *ev;  // nullable: 4 events around the passes
    int ngroups;
    BatchGroup g[2];
    BatchModel bm[2];
    int total_tiles;
    const int64_t *offsets;   // device [n_series + 1]
    const double *params;     // device [n_series][3]
    int64_t n_series;
    int64_t n;                // total steps
    int chunk;
    const double *t;
    const void *y;
    const uint8_t *mask;
    void *m;
    void *P;
    void *f_mean;
    void *f_var;
    double *loglik;           // device [n_series]
    void *ll_terms;           // workspace [n]: log-likelihood partials at segment starts
    int tiled;                // m: smoother-element handover (filter then smoother in one call)
    void *slane;              // tiled: the smoother's lane records (written by the filter's finish)
    ScanWs ws;
};

int launch_batched_filter(const BatchLaunch &a, bool f64, hipStream_t s);
// the filter without moment outputs (log-likelihood only)
int launch_batched_loglik(const BatchLaunch &a, bool f64, hipStream_t s);
int launch_batched_smooth(const BatchLaunch &a, bool f64, hipStream_t s);
// filter writing the handover, then the smoother reading it (a.tiled = 1;
// a.ev, when set, holds 8 events: filter passes, then smoother passes)
int launch_batched_predict(const BatchLaunch &a, bool f64, hipStream_t s);

// Per-layout launchers, instantiated in one translation unit per layout.
template <int B0, int B1>
int launch_filter_layout(const DevModel &mdl, bool f64, const FilterLaunch &a, hipStream_t s);
template <int B0, int B1>
int launch_smoother_layout(const DevModel &mdl, bool f64, const SmoothLaunch &a, hipStream_t s);
template <int B0, int B1>
int launch_discretize_layout(const DevModel &mdl, const double *t, int64_t n, double *F, double *Q,
                             WsCtl *ctl, hipStream_t s);
template <int B0, int B1>
int launch_grad_layout(const DevModel &mdl, bool f64, const GradLaunch &a, hipStream_t s);
// Plain FP64 baseline: element arrays and outputs
struct PlainLaunch {
    const double *t;
    const double *y;
    const uint8_t *mask;
    int64_t n;
    int64_t n2;
    double *m;
    double *P;
    double *f_mean;
    double *f_var;
    double *loglik;
    void *X;      // n2 filter elements
    void *Xraw;   // n2 filter elements
    double *terms;
};
template <int B0, int B1>
int launch_plain_layout(const DevModel &mdl, const PlainLaunch &a, hipStream_t s);

// Dispatchers: return hipSuccess or an error; -1 when the layout (b0, b1) is
// not compiled in.
int launch_filter(const DevModel &mdl, int b0, int b1, bool f64, const FilterLaunch &a, hipStream_t s);
int launch_smoother(const DevModel &mdl, int b0, int b1, bool f64, const SmoothLaunch &a, hipStream_t s);
int launch_discretize(const DevModel &mdl, int b0, int b1, const double *t, int64_t n, double *F,
                      double *Q, WsCtl *ctl, hipStream_t s);
int launch_grad(const DevModel &mdl, int b0, int b1, bool f64, const GradLaunch &a, hipStream_t s);
int launch_plain(const DevModel &mdl, int b0, int b1, const PlainLaunch &a, hipStream_t s);
// Records pass event i (when given) on stream s.
inline void pass_event(void *const *ev, int i, hipStream_t s)
{
    if (ev && ev[i]) (void)hipEventRecord((hipEvent_t)ev[i], s);
}

// Zeroes the control block (keep_status: only the tile counter, so that a
// second pass of the same call keeps the first one's status bits) and
// zero_out[0, nzero).
int launch_ws_init(WsCtl *ctl, double *zero_out, int nzero, hipStream_t s, bool keep_status = false);
bool layout_supported(int b0, int b1);

// Merge of sorted test times into the sorted training grid (merge.hip).
struct MergeLaunch {
    const double *t_train;
    const void *y_train;         // nullable when y_out is NULL or n_train is 0
    const uint8_t *mask_train;   // nullable: every training step observed
    int64_t n_train;
    const double *t_test;
    int64_t n_test;
    bool f64;                    // y in FP64 (else FP32)
    double *t_out;
    void *y_out;
    uint8_t *mask_out;
    int64_t *test_pos;           // nullable
};
int64_t merge_tiles(int64_t total);
int launch_merge(const MergeLaunch &a, hipStream_t s);
