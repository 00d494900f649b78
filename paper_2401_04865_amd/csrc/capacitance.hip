// Grand capacitance tensor and effective permittivity.
//
// Section "Induced Surface Charge Distribution of Polarizable Bodies" (the
// rigid-body moment equation): the charges and dipoles of the bodies follow
// from their potentials and the applied field through
//     [Q; S] = C [Psi - Psi_0; E0],   C = Sigma' M^-1 Sigma'^T,
// Sigma' (4 N_b x N) being the summation tensor over the ones of body i
// (row i) and over the bead positions relative to the body centre (rows
// N_b + 3 i + d).  Section "Cubic array of spheres in an electric field":
// for neutral bodies in the mean field E0,
//     eps_eff = eps I + (1/V) sum_{i,j} [C_SE - C_SPsi C_qPsi^-1 C_qE]_{ij}.
//
// M is symmetric positive definite, so the 4 N_b right-hand sides (columns
// of Sigma'^T) are solved by preconditioned conjugate gradients, a block of
// columns at a time: each iteration applies the double spectral-Ewald
// operator of the loaded configuration (one cell sort, one set of FFT tables
// and pair structures for every column) to the block's unconverged columns,
// and does the vector work of the whole block in one launch per step
// (column dot products, updates whose per-column scalars stay on the
// device).  Preconditioner: block Jacobi with, per body, the inverse of its
// free-space self block M_ii (one per shape, rotation invariant), applied to
// all bodies of a shape as one dense product.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "pe_internal.hpp"
#include "vector.hpp"

namespace pe {

namespace {

constexpr int kBS = 256;

// Column j of the block (global column col0 + j) of Sigma'^T, bead part;
// the body-potential tail of every column is zero.
__global__ void cap_rhs_kernel(const int* __restrict__ body_of, const double* __restrict__ rel, int64_t nb,
                               int64_t nbody, int64_t col0, int64_t ld, double* __restrict__ B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= ld) return;
  const int64_t col = col0 + j;
  double v = 0.0;
  if (i < nb) {
    const int b = body_of[i];
    if (col < nbody) v = (b == col) ? 1.0 : 0.0;
    else {
      const int64_t body = (col - nbody) / 3, d = (col - nbody) % 3;
      v = (b == body) ? rel[3 * i + d] : 0.0;
    }
  }
  B[(int64_t)j * ld + i] = v;
}

// part[j * nchunk + c] = sum over chunk c of A_j . B_j (first n entries)
__global__ void coldot_partial_kernel(const double* __restrict__ A, const double* __restrict__ B, int64_t ld,
                                      int64_t n, int64_t chunk, int nchunk, double* __restrict__ part) {
  const int c = blockIdx.x, j = blockIdx.y;
  const double* a = A + (int64_t)j * ld;
  const double* b = B + (int64_t)j * ld;
  const int64_t i0 = (int64_t)c * chunk, i1 = min(n, i0 + chunk);
  double s = 0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) s += a[i] * b[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ double sh[kBS / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < kBS / 64; ++w) t += sh[w];
    part[(int64_t)j * nchunk + c] = t;
  }
}

__global__ void coldot_final_kernel(const double* __restrict__ part, int nchunk, double* __restrict__ out) {
  const int j = blockIdx.x;
  double s = 0;
  for (int c = threadIdx.x; c < nchunk; c += 64) s += part[(int64_t)j * nchunk + c];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) out[j] = s;
}

// Y holds -M p (the top of the saddle product with zero potentials):
// alpha = rz / (p . M p); x += alpha p; r -= alpha M p.
__global__ void cg_update_kernel(double* __restrict__ X, double* __restrict__ R, const double* __restrict__ P,
                                 const double* __restrict__ Y, int64_t ld, int64_t n, const double* __restrict__ rz,
                                 const double* __restrict__ pY, const int* __restrict__ active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n || !active[j]) return;
  const double alpha = rz[j] / (-pY[j]);
  const int64_t o = (int64_t)j * ld + i;
  X[o] += alpha * P[o];
  R[o] += alpha * Y[o];
}

// p = z + beta p, beta = rz_new / rz_old (first: p = z)
__global__ void cg_direction_kernel(double* __restrict__ P, const double* __restrict__ Z, int64_t ld, int64_t n,
                                    const double* __restrict__ rz_new, const double* __restrict__ rz_old,
                                    const int* __restrict__ active, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n || !active[j]) return;
  const int64_t o = (int64_t)j * ld + i;
  P[o] = first ? Z[o] : Z[o] + (rz_new[j] / rz_old[j]) * P[o];
}

// Rows of C for the block's columns: per (body i, column j) the charge
// sum_j x and the dipole sum_j r x of body i's beads.
__global__ void cap_moments_kernel(const int64_t* __restrict__ off, const double* __restrict__ rel,
                                   const double* __restrict__ X, int64_t ld, int64_t nbody, int64_t col0,
                                   double* __restrict__ C) {
  const int64_t i = blockIdx.x;
  const int j = blockIdx.y;
  const double* x = X + (int64_t)j * ld;
  double q = 0, sx = 0, sy = 0, sz = 0;
  for (int64_t k = off[i] + threadIdx.x; k < off[i + 1]; k += blockDim.x) {
    const double v = x[k];
    q += v;
    sx += rel[3 * k] * v;
    sy += rel[3 * k + 1] * v;
    sz += rel[3 * k + 2] * v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    q += __shfl_xor(q, o, 64);
    sx += __shfl_xor(sx, o, 64);
    sy += __shfl_xor(sy, o, 64);
    sz += __shfl_xor(sz, o, 64);
  }
  __shared__ double sh[4][kBS / 64];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = q; sh[1][w] = sx; sh[2][w] = sy; sh[3][w] = sz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[4] = {0, 0, 0, 0};
    for (int k = 0; k < kBS / 64; ++k)
      for (int m = 0; m < 4; ++m) t[m] += sh[m][k];
    const int64_t ldc = 4 * nbody, col = col0 + j;
    C[i * ldc + col] = t[0];
    for (int d = 0; d < 3; ++d) C[(nbody + 3 * i + d) * ldc + col] = t[1 + d];
  }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

struct ColDot {
  int nchunk;
  int64_t chunk;
  double* part;
};

ColDot coldot_plan(int64_t n, double* part, int kb, size_t part_cap) {
  ColDot d;
  d.chunk = std::max<int64_t>(4096, (n + 255) / 256);
  d.nchunk = (int)std::max<int64_t>(1, (n + d.chunk - 1) / d.chunk);
  require((size_t)d.nchunk * kb <= part_cap, "capacitance: reduction buffer too small");
  d.part = part;
  return d;
}

void coldot(hipStream_t s, const ColDot& d, const double* A, const double* B, int64_t ld, int64_t n, int kb,
            double* out) {
  hipLaunchKernelGGL(coldot_partial_kernel, dim3(d.nchunk, kb), dim3(kBS), 0, s, A, B, ld, n, d.chunk, d.nchunk,
                     d.part);
  hipLaunchKernelGGL(coldot_final_kernel, dim3(kb), dim3(64), 0, s, d.part, d.nchunk, out);
  PE_CHECK_LAUNCH();
}

// z = P^-1 r for one column (block Jacobi over the bodies' free-space self
// blocks; the identity when the context has no preconditioner)
void precondition(pe_context* c, const double* r, double* z) {
  hipStream_t s = c->stream;
  bool any = false;
  for (auto& t : c->pc.types)
    if (!t.bodies.empty() && t.have_inv) any = true;
  if (!c->p.precond || !any) {
    PE_HIP(hipMemcpyAsync(z, r, sizeof(double) * c->n_bead, hipMemcpyDeviceToDevice, s));
    return;
  }
  for (auto& t : c->pc.types) {
    if (t.bodies.empty()) continue;
    launch_body_gemm<double>(s, t.Minv.get(), t.N, false, false, t.dbodies.get(), (int)t.bodies.size(),
                             c->off.get(), c->n_bead, r, z, c->pc.gemm_ws.get());
  }
}

// Cholesky solve of the SPD system A x = b in place (n x n, row-major).
void host_cholesky_solve(std::vector<double>& A, int n, std::vector<double>& b, int nrhs) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(d > 0)) throw Error(PE_ERR_NUMERIC, "capacitance: C_qPsi is not positive definite");
    d = std::sqrt(d);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = v / d;
    }
  }
  for (int r = 0; r < nrhs; ++r) {
    double* x = b.data() + (size_t)r * n;
    for (int i = 0; i < n; ++i) {
      double v = x[i];
      for (int k = 0; k < i; ++k) v -= A[(size_t)i * n + k] * x[k];
      x[i] = v / A[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = x[i];
      for (int k = i + 1; k < n; ++k) v -= A[(size_t)k * n + i] * x[k];
      x[i] = v / A[(size_t)i * n + i];
    }
  }
}

}  // namespace

// eps_eff (row-major 3 x 3) from C (host, row-major (4 nb)^2): only the block
// sums enter, so with u_a[k] = sum_i C_SPsi[(i,a), k] and w_b[l] = sum_j
// C_qE[l, (j,b)], T_ab = sum_{ij} C_SE[(i,a),(j,b)] - u_a . C_qPsi^-1 w_b.
void effective_permittivity(const std::vector<double>& C, int64_t nb, double eps, double V, double* out) {
  const int64_t ld = 4 * nb;
  std::vector<double> A((size_t)nb * nb), w((size_t)3 * nb, 0.0);
  double T[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int64_t i = 0; i < nb; ++i)
    for (int64_t k = 0; k < nb; ++k)
      A[(size_t)i * nb + k] = 0.5 * (C[(size_t)i * ld + k] + C[(size_t)k * ld + i]);
  for (int b = 0; b < 3; ++b)
    for (int64_t l = 0; l < nb; ++l) {
      double s = 0;
      for (int64_t j = 0; j < nb; ++j) s += C[(size_t)l * ld + nb + 3 * j + b];
      w[(size_t)b * nb + l] = s;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int64_t i = 0; i < nb; ++i)
        for (int64_t j = 0; j < nb; ++j) s += C[(size_t)(nb + 3 * i + a) * ld + nb + 3 * j + b];
      T[a][b] = s;
    }
  std::vector<double> y = w;
  host_cholesky_solve(A, (int)nb, y, 3);
  for (int a = 0; a < 3; ++a) {
    std::vector<double> u(nb, 0.0);
    for (int64_t i = 0; i < nb; ++i)
      for (int64_t k = 0; k < nb; ++k) u[k] += C[(size_t)(nb + 3 * i + a) * ld + k];
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int64_t k = 0; k < nb; ++k) s += u[k] * y[(size_t)b * nb + k];
      T[a][b] -= s;
    }
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) out[3 * a + b] = (a == b ? eps : 0.0) + T[a][b] / V;
}

void grand_capacitance(pe_context* c, double* C_out, double* eps_out, pe_solve_info* info) {
  hipStream_t s = c->stream;
  const int64_t nb = c->n_bead, nbody = c->n_body, n = nb + nbody;
  require(nbody > 0, "capacitance: no bodies");
  const int64_t ncol = 4 * nbody;
  const int kb = (int)std::min<int64_t>(ncol, 32);
  const auto t0 = std::chrono::steady_clock::now();
  // block storage: X, R, Z, P, Y (kb columns of n each) and per-column scalars
  DevBuf<double> blk, sc, part, Cd;
  blk.ensure((size_t)5 * kb * n);
  double* X = blk.get();
  double* R = X + (size_t)kb * n;
  double* Z = R + (size_t)kb * n;
  double* P = Z + (size_t)kb * n;
  double* Y = P + (size_t)kb * n;
  sc.ensure((size_t)6 * kb);
  double* rz = sc.get();
  double* rz2 = rz + kb;
  double* pY = rz2 + kb;
  double* rr = pY + kb;
  DevBuf<int> act;
  act.ensure(kb);
  const ColDot cd = coldot_plan(nb, nullptr, kb, (size_t)1 << 40);
  part.ensure((size_t)cd.nchunk * kb);
  ColDot d = cd;
  d.part = part.get();
  double* C = C_out;
  if (!C) {
    Cd.ensure((size_t)ncol * ncol);
    C = Cd.get();
  }
  const double tol = c->p.rel_tol;
  int max_it = 0, mv = 0;
  double worst = 0;
  std::vector<double> h_rr(kb), h_b(kb);
  std::vector<int> h_act(kb);
  for (int64_t col0 = 0; col0 < ncol; col0 += kb) {
    const int k = (int)std::min<int64_t>(kb, ncol - col0);
    const dim3 g2(nblk(n, kBS), k);
    PE_HIP(hipMemsetAsync(blk.get(), 0, sizeof(double) * 5 * (size_t)kb * n, s));
    hipLaunchKernelGGL(cap_rhs_kernel, g2, dim3(kBS), 0, s, c->body_of.get(), c->rel.get(), nb, nbody, col0, n, R);
    PE_CHECK_LAUNCH();
    coldot(s, d, R, R, n, nb, k, rr);
    PE_HIP(hipMemcpyAsync(h_b.data(), rr, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    for (int j = 0; j < k; ++j) precondition(c, R + (size_t)j * n, Z + (size_t)j * n);
    coldot(s, d, R, Z, n, nb, k, rz);
    PE_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) {
      h_b[j] = std::sqrt(h_b[j]);
      h_act[j] = h_b[j] > 0 ? 1 : 0;
    }
    PE_HIP(hipMemcpyAsync(act.get(), h_act.data(), sizeof(int) * k, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(cg_direction_kernel, g2, dim3(kBS), 0, s, P, Z, n, nb, rz, rz, act.get(), 1);
    PE_CHECK_LAUNCH();
    int it = 0;
    for (; it < c->p.max_iters; ++it) {
      for (int j = 0; j < k; ++j)
        if (h_act[j]) {
          saddle_product(c, PE_FP64, P + (size_t)j * n, Y + (size_t)j * n);
          ++mv;
        }
      coldot(s, d, P, Y, n, nb, k, pY);
      hipLaunchKernelGGL(cg_update_kernel, g2, dim3(kBS), 0, s, X, R, P, Y, n, nb, rz, pY, act.get());
      PE_CHECK_LAUNCH();
      coldot(s, d, R, R, n, nb, k, rr);
      PE_HIP(hipMemcpyAsync(h_rr.data(), rr, sizeof(double) * k, hipMemcpyDeviceToHost, s));
      PE_HIP(hipStreamSynchronize(s));
      bool left = false, changed = false;
      for (int j = 0; j < k; ++j) {
        if (!h_act[j]) continue;
        const double rel = std::sqrt(h_rr[j]) / h_b[j];
        if (!std::isfinite(rel)) throw Error(PE_ERR_NUMERIC, "non-finite residual in the capacitance solves");
        if (rel <= tol) {
          h_act[j] = 0;
          changed = true;
          worst = std::max(worst, rel);
        } else {
          left = true;
        }
      }
      if (!left) {
        ++it;
        break;
      }
      if (changed) PE_HIP(hipMemcpyAsync(act.get(), h_act.data(), sizeof(int) * k, hipMemcpyHostToDevice, s));
      PE_HIP(hipMemcpyAsync(rz2, rz, sizeof(double) * k, hipMemcpyDeviceToDevice, s));
      for (int j = 0; j < k; ++j)
        if (h_act[j]) precondition(c, R + (size_t)j * n, Z + (size_t)j * n);
      coldot(s, d, R, Z, n, nb, k, rz);
      hipLaunchKernelGGL(cg_direction_kernel, g2, dim3(kBS), 0, s, P, Z, n, nb, rz, rz2, act.get(), 0);
      PE_CHECK_LAUNCH();
    }
    for (int j = 0; j < k; ++j)
      if (h_act[j]) {
        worst = std::max(worst, std::sqrt(h_rr[j]) / h_b[j]);
        if (info) info->iters = std::max(info->iters, it);
        if (info) info->matvecs_fp64 = mv;
        throw Error(PE_ERR_NOT_CONVERGED, "capacitance: conjugate gradients did not reach rel_tol within max_iters");
      }
    max_it = std::max(max_it, it);
    hipLaunchKernelGGL(cap_moments_kernel, dim3((unsigned)nbody, k), dim3(kBS), 0, s, c->off.get(), c->rel.get(), X,
                       n, nbody, col0, C);
    PE_CHECK_LAUNCH();
  }
  PE_HIP(hipStreamSynchronize(s));
  if (eps_out) {
    std::vector<double> hC((size_t)ncol * ncol);
    PE_HIP(hipMemcpy(hC.data(), C, sizeof(double) * hC.size(), hipMemcpyDeviceToHost));
    effective_permittivity(hC, nbody, c->p.eps, c->V, eps_out);
  }
  c->prof.flush();
  if (info) {
    info->iters = max_it;
    info->matvecs_fp64 = mv;
    info->rel_residual = worst;
    info->t_solve = info->t_total =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
}

}  // namespace pe
