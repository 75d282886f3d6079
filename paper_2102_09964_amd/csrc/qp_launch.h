// Host interface of the large-state path (quasi-periodic models): model
// construction and the launch of the fused filter + smoother.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qp_team.h"

struct pssgp_model;

struct QPLaunch {
    void *const *ev;  // nullable: 8 events (filter fold, scan, finish, end; smoother fold, scan, finish, end)
    const double *t;
    const void *y;
    const uint8_t *mask;
    int64_t n;
    int chunk;
    int G;              // chunks of `chunk` steps
    void *fagg[2];      // G filter aggregates each (ping-pong)
    void *sagg[2];      // G smoother aggregates each (ping-pong)
    void *elem;         // n smoother elements; NULL: log-likelihood only
    double *partials;   // G
    double *loglik;     // device double[1]
    void *f_mean;
    void *f_var;
    uint32_t *status;
};

// Whether a model is a quasi-periodic one (first component PSSGP_QUASIPERIODIC).
bool qp_is_model(const pssgp_model *spec);
// Host construction: 0 or a negative pssgp status code (message through
// pssgp_set_error). tdiag (nullable, d entries): x_canonical = diag(tdiag) z.
int qp_build(const pssgp_model *spec, QPDev *out, double *tdiag);
// Generator G (d*d) and observation row H in the library's coordinates.
void qp_matrices(const QPDev &m, double *G, double *Pinf, double *H);
// Launch (stream-ordered); -1: layout not compiled in, else a hipError_t.
int qp_launch(const QPDev &m, bool f64, const QPLaunch &q, hipStream_t s);
