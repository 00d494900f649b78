// Block-Jacobi preconditioner for the conductor saddle-point system.
//
// The saddle matrix couples each body's beads to every other bead through M,
// but the strongest coupling is within a body.  Keeping only the diagonal
// body blocks gives, per body, the small saddle matrix
//     A_i = [ -M_ii  1 ]
//           [  1^T   0 ]
// (the summation tensor is block diagonal by construction).  M_ii is taken in
// free space, so it depends only on the distances between the body's own
// beads: rigid bodies of one shape share one A_i whatever their position and
// orientation.  With M_ii SPD, u = M_ii^{-1} 1 and s = 1^T u,
//     A_i^{-1} = [ -M^{-1} + u u^T / s   u / s ]
//                [  u^T / s              1 / s ].
// Bodies are grouped into shape types (shapes.hip), M^{-1} is formed per type
// on the device by Gauss-Jordan elimination (no pivoting: M is SPD), and the
// preconditioner is applied to all bodies of a type at once as one dense
// product (N+1) x (N+1) times (N+1) x n_bodies.  Types are cached across
// configurations, so a rigid-body simulation builds them once.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pe_internal.hpp"
#include "precond.hpp"

namespace pe {

namespace {

constexpr double kInv4Pi = 0.07957747154594766788;
constexpr double kTwoOverSqrtPi = 1.12837916709551257390;

// Free-space regularized potential tensor of one body (N x N, row-major).
__global__ void build_self_block_kernel(const double* __restrict__ ref, const double* __restrict__ sig, int N,
                                        int reg, double a, double eps, double* __restrict__ M) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * N) return;
  const int i = (int)(t / N), j = (int)(t % N);
  const double dx = ref[3 * i] - ref[3 * j], dy = ref[3 * i + 1] - ref[3 * j + 1], dz = ref[3 * i + 2] - ref[3 * j + 2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double c = kInv4Pi / eps;
  double v;
  if (reg == PE_REG_GAUSSIAN) {
    const double b = 1.0 / sqrt(2.0 * (sig[i] * sig[i] + sig[j] * sig[j]));
    v = r > 0 ? c * erf(b * r) / r : c * kTwoOverSqrtPi * b;
  } else {
    v = r >= 2 * a ? c / r : c * (4 * a - r) / (4 * a * a);
  }
  M[t] = v;
}

// Gauss-Jordan step k, part 1: save column k, normalize row k.
__global__ void gj_pivot_kernel(double* __restrict__ A, int N, int k, double* __restrict__ f,
                                double* __restrict__ rowk) {
  const double p = A[(int64_t)k * N + k];
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    f[i] = (i == k) ? 0.0 : A[(int64_t)i * N + k];
    rowk[i] = (i == k) ? 1.0 / p : A[(int64_t)k * N + i] / p;
  }
}

// Part 2: eliminate column k from every other row, write row k.
__global__ void gj_update_kernel(double* __restrict__ A, int N, int k, const double* __restrict__ f,
                                 const double* __restrict__ rowk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * N) return;
  const int i = (int)(t / N), j = (int)(t % N);
  if (i == k) {
    A[t] = rowk[j];
  } else {
    const double base = (j == k) ? 0.0 : A[t];
    A[t] = base - f[i] * rowk[j];
  }
}

// u = Minv 1 (row sums), s = 1^T u
__global__ void rowsum_kernel(const double* __restrict__ Minv, int N, double* __restrict__ u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0;
  for (int j = 0; j < N; ++j) s += Minv[(int64_t)i * N + j];
  u[i] = s;
}

// Assemble the (N+1) x (N+1) inverse of the body saddle block (and a float copy).
__global__ void assemble_inverse_kernel(const double* __restrict__ Minv, const double* __restrict__ u, double s,
                                        int N, double* __restrict__ Ainv, float* __restrict__ Ainv32) {
  const int Np = N + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)Np * Np) return;
  const int i = (int)(t / Np), j = (int)(t % Np);
  double v;
  if (i < N && j < N) v = -Minv[(int64_t)i * N + j] + u[i] * u[j] / s;
  else if (i < N) v = u[i] / s;
  else if (j < N) v = u[j] / s;
  else v = 1.0 / s;
  Ainv[t] = v;
  Ainv32[t] = (float)v;
}

}  // namespace

void build_type_inverse(pe_context* c, BodyType& t) {
  hipStream_t s = c->stream;
  const int N = t.N, Np = N + 1;
  DevBuf<double> dref, dsig, M, f, rowk, u;
  dref.ensure(3 * N);
  dsig.ensure(N);
  M.ensure((size_t)N * N);
  f.ensure(N);
  rowk.ensure(N);
  u.ensure(N);
  PE_HIP(hipMemcpyAsync(dref.get(), t.ref.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
  PE_HIP(hipMemcpyAsync(dsig.get(), t.sig.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
  const int64_t NN = (int64_t)N * N;
  const unsigned nb = (unsigned)((NN + 255) / 256);
  hipLaunchKernelGGL(build_self_block_kernel, dim3(nb), dim3(256), 0, s, dref.get(), dsig.get(), N, c->p.reg,
                     c->p.shell_radius, c->p.eps, M.get());
  PE_CHECK_LAUNCH();
  for (int k = 0; k < N; ++k) {
    hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(256), 0, s, M.get(), N, k, f.get(), rowk.get());
    hipLaunchKernelGGL(gj_update_kernel, dim3(nb), dim3(256), 0, s, M.get(), N, k, f.get(), rowk.get());
  }
  PE_CHECK_LAUNCH();
  // keep M_ii^-1 itself (block-Jacobi preconditioner of M alone, e.g. for
  // the capacitance solves)
  t.Minv.ensure((size_t)NN);
  PE_HIP(hipMemcpyAsync(t.Minv.get(), M.get(), sizeof(double) * NN, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(rowsum_kernel, dim3((N + 255) / 256), dim3(256), 0, s, M.get(), N, u.get());
  PE_CHECK_LAUNCH();
  std::vector<double> hu(N);
  PE_HIP(hipMemcpyAsync(hu.data(), u.get(), sizeof(double) * N, hipMemcpyDeviceToHost, s));
  PE_HIP(hipStreamSynchronize(s));
  double ssum = 0;
  for (int i = 0; i < N; ++i) ssum += hu[i];
  if (!(ssum > 0) || !std::isfinite(ssum))
    throw Error(PE_ERR_NUMERIC, "body self block is not positive definite");
  const int64_t NpNp = (int64_t)Np * Np;
  t.Ainv.ensure(NpNp);
  t.Ainv32.ensure(NpNp);
  hipLaunchKernelGGL(assemble_inverse_kernel, dim3((unsigned)((NpNp + 255) / 256)), dim3(256), 0, s, M.get(),
                     u.get(), ssum, N, t.Ainv.get(), t.Ainv32.get());
  PE_CHECK_LAUNCH();
  PE_HIP(hipStreamSynchronize(s));
}

template <typename T>
void precond_apply(hipStream_t s, pe_context* c, const double* x, double* z) {
  for (auto& t : c->pc.types) {
    const int nbt = (int)t.bodies.size();
    if (nbt == 0) continue;
    const T* A;
    if constexpr (sizeof(T) == 8) A = t.Ainv.get();
    else A = t.Ainv32.get();
    launch_body_gemm<T>(s, A, t.N, true, false, t.dbodies.get(), nbt, c->off.get(), c->n_bead, x, z,
                        c->pc.gemm_ws.get());
  }
}

template void precond_apply<float>(hipStream_t, pe_context*, const double*, double*);
template void precond_apply<double>(hipStream_t, pe_context*, const double*, double*);

}  // namespace pe
