// Declarations of the double-precision vector and reduction launchers.
#pragma once

#include "pe_internal.hpp"

namespace pe {

constexpr int kMaxK = 256;  // max Krylov vectors in one multi-dot (restart + 1)

// Coefficients of the k = 0 constant of the split.
struct CkCoef {
  int reg;
  double inv_epsV;  // 1 / (eps V)
  double inv4xi2;   // 1 / (4 xi^2)
  double a;         // shell radius
};

void launch_moments(hipStream_t s, const double* q, const double* sig, double sig_const, int64_t n,
                    const CkCoef& cc, double* partial, double* ck, double* tot);
void launch_seg_sum(hipStream_t s, const int64_t* off, int64_t n_body, const double* x, double* out);
void launch_body_outputs(hipStream_t s, const int64_t* off, int64_t n_body, const double* rel, const double* q,
                         const double* f, const double* u, double* S, double* F, double* L, double* U);
void launch_mdot(hipStream_t s, const double* V, int64_t ldv, int K, const double* w, int64_t n,
                 double* partial, double* out, bool take_sqrt);
void launch_maxpy(hipStream_t s, const double* V, int64_t ldv, int K, const double* h, double* w, int64_t n,
                  double sign);
void launch_scale(hipStream_t s, const double* w, const double* nrm, double* vout, int64_t n);
void launch_axpby(hipStream_t s, double a, const double* x, double b, double* y, int64_t n);
void launch_sub(hipStream_t s, const double* x, const double* y, double* z, int64_t n);
void launch_givens(hipStream_t s, const double* h1, const double* h2, const double* nrm, double* st, int m,
                   int j, double* res);
// One classical Gram-Schmidt (CGS2) Arnoldi step of column j in four
// launches: h1 = V^T w, w -= V h1, h2 = V^T w, w -= V h2, *nrm = ||w||,
// vout = w / ||w||, then the Givens step (h1 + h2, ||w||) with the residual
// estimate in *res and, when res_host is given, in page-locked host memory.
// V holds K vectors of n (stride ldv); partial holds 2 kMaxK 1024 doubles.
void launch_cgs_step(hipStream_t s, const double* V, int64_t ldv, int K, double* w, int64_t n, double* partial,
                     double* h1, double* h2, double* nrm, double* vout, double* st, int m, int j, double* res,
                     double* res_host);
void launch_init_g(hipStream_t s, double* st, int m, const double* beta);
void launch_backsolve(hipStream_t s, const double* st, int m, int k, double* y);

// Sort every segment [start[k], start[k+1]) of keys ascending, in place.
// Sorts keys[start[k] .. start[k+1]) ascending for every k; max_len bounds
// the segment lengths (it sizes the LDS of each workgroup).
void launch_segment_sort(hipStream_t s, const int* start, int nseg, int* keys, int max_len);
// out[0] = 0, out[i+1] = in[0] + ... + in[i] (i < n), summed in 64 bits;
// tmp holds scan_workspace(n) values.
int64_t scan_workspace(int64_t n);
void launch_exclusive_scan(hipStream_t s, const int* in, int64_t n, int64_t* out, int64_t* tmp);

// per-particle kernels of the solve / force passes (solver unit)
void launch_rhs_top(hipStream_t s, int64_t n, const double* rel, const double* E0, const double* phi_ion,
                    double* b);
void launch_forces_energy(hipStream_t s, int64_t n, const double* chg, const double* pos, const double* E0v,
                          const double* phi, const double* E, double* f, double* u);

}  // namespace pe
