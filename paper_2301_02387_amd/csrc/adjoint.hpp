// Launchers of the reverse-sweep kernels (adjoint.hip).  One instance, at
// most 4 orbitals; see adjoint.hip for the conventions.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace mh {

// Small complex n x n blocks of the per-step sensitivities, in one device
// array (index * n * n complex entries each).
enum {
  ADJ_XG = 0,    // ginv^T
  ADJ_XR,        // (regularised gamma)^T
  ADJ_LAM2,      // mixing matrix of the conjugated adjoint operator
  ADJ_LBAR,      // sensitivity of lambda, [q][p]
  ADJ_KH,        // sensitivity of h
  ADJ_KGAM,      // sensitivity of gamma
  ADJ_XL1, ADJ_XL2, ADJ_XH, ADJ_XD,  // mixing matrices of the reverse terms
  ADJ_NBLK
};

void launch_mix(const Batch& b, const double* in, const double* X, double beta, double* out, hipStream_t s);
void launch_q_accum(const Batch& b, const double* A, const double* B, double wr, double wi, double* Q,
                    hipStream_t s);
void launch_adj_mf(const Batch& b, const double* Q, const double* W, const double* phi, const double* ginv,
                   const double* Mr, const double* Kg, const int* colmap, double* Kw, double* Phib, hipStream_t s);
void launch_qw_gram(const Batch& b, const double* Q, const double* W, double* part, double* G2, hipStream_t s);
int64_t qw_part_doubles(const Batch& b);
void launch_caxpy(int64_t cnt, double wr, double wi, const double* x, double* y, hipStream_t s);
void launch_adj_prep(const double* ginv, const double* lam, int n, double* sm, hipStream_t s);
void launch_adj_quad(const double* Gz, const double* Sm, double wr, double wi, int n, double* ebar, double* sm,
                     hipStream_t s);
void launch_adj_terms(const double* z, const double* gam, double g, int n, double* ebar, double* sm, hipStream_t s);
void launch_adj_mf_small(const double* G2, const double* Mr, const double* ginv, const int* colmap, int n,
                         double* sm, double* KGam, hipStream_t s);
void launch_adj_ciprep(const double* sm, const double* KGam, int n, double* h, double* g, hipStream_t s);
void launch_adj_poisson_rhs(const Batch& b, const double* Kw, int ncol, double* y, double* sc, hipStream_t s);
void launch_adj_bnd(const Batch& b, const double* Kw, const double* u, int ncol, int nh, double* tb, double* qlm,
                    hipStream_t s);
void launch_krho(const Batch& b, const double* z, const double* qlm, int lmax, int ncol, const int* colmap,
                 const double* phi, double* Phib, hipStream_t s);
void launch_load_split(const Batch& b, const double* f, double* out, double* acc, hipStream_t s);

}  // namespace mh
