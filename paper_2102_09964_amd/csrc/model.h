// Model constants shared by the host construction and the device kernels.
//
// The device works in "normalised, balanced" state coordinates. For every
// kernel component c the state is the canonical companion state scaled so
// that the generator is G_c = G1_c / ell_c with G1_c independent of the
// length-scale, the stationary covariance is var_c * P1_c, and a constant
// radix-2 diagonal scaling (Osborne balancing, paper section 4.2) is
// applied to G1_c. The observation row H keeps a unit entry at the first
// state of each component. Sum kernels are block diagonal.
//
// The transition over a step of length dt is F_c = exp(s G1_c) with
// s = dt / ell_c; it is evaluated from a fixed expansion
//   F_c(s) = sum_r phi_r(s) M_r
// whose matrices M_r are precomputed on the host:
//  * Matern blocks: G1_c + lam I is nilpotent, so
//      F_c(s) = exp(-lam s) sum_j s^j Nb^j / j!   (M_j = Nb^j / j!, phi_j = e^{-lam s} s^j)
//  * RBF-Taylor blocks: G1_c has distinct eigenvalues rho = alpha +- i beta,
//      F_c(s) = sum_pairs e^{alpha s} (cos(beta s) M_cos + sin(beta s) M_sin)
//               + sum_real e^{alpha s} M_real.
// The expansion is cheap but cancels terms of size up to the eigenvalue
// condition numbers of G1 (about 1e4 for the RBF Taylor models), which costs
// about 1e-12 absolute accuracy in F; where full FP64 accuracy matters the
// kernels instead evaluate exp(s G1) by scaling and squaring a truncated
// Taylor series, multiplying by the sparse companion-structured G1.
// The process noise follows from stationarity: Q = Pinf - F Pinf F^T.
#pragma once
#include <stdint.h>

#define PSSGP_MAXD 8
#define PSSGP_MAXBLK 2
#define PSSGP_MAXRT 4
#define PSSGP_FCOEF 232

enum { BLK_MATERN = 1, BLK_RBF = 2 };

struct DevBlock {
    int32_t kind;    // BLK_MATERN or BLK_RBF
    int32_t dim;     // state size of the block
    int32_t off;     // first state index
    int32_t npair;   // RBF: complex-conjugate eigenvalue pairs
    int32_t nreal;   // RBF: real eigenvalues
    int32_t fc_off;  // first expansion matrix in DevModel::fcoef
    int32_t comp;    // index of the user component (gradient order)
    int32_t pad;
    double ell, inv_ell, var;
    double lam;                 // Matern: decay rate at unit length-scale
    double alpha[PSSGP_MAXRT];  // RBF: real parts (pairs first, then real roots)
    double beta[PSSGP_MAXRT];   // RBF: positive imaginary parts of the pairs
    // unit-length-scale generator G1 of the block in balanced coordinates:
    // companion structure, nonzero only on the superdiagonal and last row
    double gsup[PSSGP_MAXD];    // G1[i][i+1], i < dim-1
    double glast[PSSGP_MAXD];   // G1[dim-1][j]
    double gnorm;               // ||G1||_1
};

struct DevModel {
    int32_t d;
    int32_t nblk;
    int32_t pad[2];
    double R;                                // noise variance
    double H[PSSGP_MAXD];                    // observation row
    DevBlock blk[PSSGP_MAXBLK];
    double Pinf[PSSGP_MAXD * PSSGP_MAXD];    // stationary covariance (block diagonal)
    double fcoef[PSSGP_FCOEF];               // expansion matrices, block after block
};

static_assert(sizeof(DevModel) <= 3584, "model constants are passed by value as a kernel argument");

// Host construction. Returns 0 or a negative pssgp status code and writes an
// error message through pssgp_set_error. tdiag (nullable, d entries)
// receives the diagonal basis change: x_canonical = diag(tdiag) z.
struct pssgp_model;
int pssgp_build_devmodel(const struct pssgp_model *spec, DevModel *out, double *tdiag);
// block-dimension signature used to select a kernel instantiation: dims of
// up to two blocks, 0 for an absent block
void pssgp_layout(const DevModel &m, int *b0, int *b1);
void pssgp_set_error(const char *fmt, ...);
