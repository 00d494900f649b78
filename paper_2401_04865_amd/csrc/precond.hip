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
// Bodies are grouped into shape types on the host (bead count, widths and the
// distances of every bead to three reference beads), M^{-1} is formed per type
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

// z = A^{-1} x for every body of one type: Y (Np x nb) = Ainv (Np x Np) X (Np x nb),
// column b of X is [x[off(b) .. off(b)+N); x[n_bead + body(b)]].
// 32 x 32 output tiles (a few hundred workgroups even for one shape of a few
// hundred beads), K staged through LDS 32 at a time; thread (tx, ty) of the
// 16 x 16 block owns rows {ty, ty + 16} and columns {tx, tx + 16} of the tile.
constexpr int kBM = 32, kBN = 32, kBK = 32;

template <typename T>
__global__ void __launch_bounds__(256) apply_type_kernel(const T* __restrict__ Ainv, int N,
                                                         const int* __restrict__ bodies, int nbt,
                                                         const int64_t* __restrict__ off, int64_t n_bead,
                                                         const double* __restrict__ x, double* __restrict__ z) {
  const int Np = N + 1;
  __shared__ T As[kBK][kBM + 1];
  __shared__ T Xs[kBK][kBN + 1];
  __shared__ int64_t boff[kBN];
  __shared__ int64_t bpsi[kBN];
  const int row0 = blockIdx.x * kBM;
  const int col0 = blockIdx.y * kBN;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (threadIdx.x < kBN) {
    const int b = col0 + threadIdx.x;
    if (b < nbt) {
      const int body = bodies[b];
      boff[threadIdx.x] = off[body];
      bpsi[threadIdx.x] = n_bead + body;
    } else {
      boff[threadIdx.x] = -1;
      bpsi[threadIdx.x] = -1;
    }
  }
  __syncthreads();
  T acc[2][2] = {{0, 0}, {0, 0}};
  for (int k0 = 0; k0 < Np; k0 += kBK) {
    for (int t = threadIdx.x; t < kBK * kBM; t += blockDim.x) {
      const int kk = t % kBK, r = t / kBK;
      const int gr = row0 + r, gk = k0 + kk;
      As[kk][r] = (gr < Np && gk < Np) ? Ainv[(int64_t)gr * Np + gk] : (T)0;
    }
    for (int t = threadIdx.x; t < kBK * kBN; t += blockDim.x) {
      const int cc = t / kBK, kk = t % kBK;
      const int gk = k0 + kk;
      T v = 0;
      if (boff[cc] >= 0 && gk < Np) v = (T)(gk < N ? x[boff[cc] + gk] : x[bpsi[cc]]);
      Xs[kk][cc] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kBK; ++kk) {
      const T a0 = As[kk][ty], a1 = As[kk][ty + 16];
      const T b0 = Xs[kk][tx], b1 = Xs[kk][tx + 16];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const int gr = row0 + ty + 16 * p;
    if (gr >= Np) continue;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int cc = tx + 16 * q;
      if (boff[cc] < 0) continue;
      const int64_t o = gr < N ? boff[cc] + gr : bpsi[cc];
      z[o] = (double)acc[p][q];
    }
  }
}

bool same_shape(const BodyType& t, const double* rel, const double* sig, int N) {
  if (t.N != N) return false;
  double scale = 0;
  for (int j = 0; j < 3 * N; ++j) scale = std::max(scale, std::fabs(t.ref[j]));
  const double tol = 1e-9 * std::max(scale, 1e-300);
  auto dist = [](const double* a, const double* b) {
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return std::sqrt(dx * dx + dy * dy + dz * dz);
  };
  const int nref = std::min(N, 3);
  for (int j = 0; j < N; ++j) {
    if (std::fabs(t.sig[j] - sig[j]) > 1e-12 * std::fabs(sig[j])) return false;
    for (int r = 0; r < nref; ++r)
      if (std::fabs(dist(&t.ref[3 * j], &t.ref[3 * r]) - dist(&rel[3 * j], &rel[3 * r])) > tol) return false;
  }
  return true;
}

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

}  // namespace

void precond_setup(pe_context* c) {
  Precond& pc = c->pc;
  for (auto& t : pc.types) t.bodies.clear();
  const int64_t nb = c->n_bead, nbody = c->n_body;
  if (nbody == 0) return;
  std::vector<double> rel(3 * nb), sig(nb);
  if (nb) {
    PE_HIP(hipMemcpyAsync(rel.data(), c->rel.get(), sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, c->stream));
    PE_HIP(hipMemcpyAsync(sig.data(), c->bead_sig.get(), sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
  }
  PE_HIP(hipStreamSynchronize(c->stream));
  for (int64_t i = 0; i < nbody; ++i) {
    const int64_t o = c->h_off[i];
    const int N = (int)(c->h_off[i + 1] - o);
    if (N == 0) continue;
    BodyType* found = nullptr;
    for (auto& t : pc.types)
      if (same_shape(t, &rel[3 * o], &sig[o], N)) {
        found = &t;
        break;
      }
    if (!found) {
      require(N <= 16384, "body too large for the block preconditioner (N > 16384)");
      pc.types.emplace_back();
      BodyType& t = pc.types.back();
      t.N = N;
      t.ref.assign(rel.begin() + 3 * o, rel.begin() + 3 * (o + N));
      t.sig.assign(sig.begin() + o, sig.begin() + o + N);
      build_type_inverse(c, t);
      found = &t;
    }
    found->bodies.push_back((int)i);
  }
  for (auto& t : pc.types) {
    t.dbodies.ensure(std::max<size_t>(1, t.bodies.size()));
    if (!t.bodies.empty())
      PE_HIP(hipMemcpyAsync(t.dbodies.get(), t.bodies.data(), sizeof(int) * t.bodies.size(), hipMemcpyHostToDevice,
                            c->stream));
  }
  PE_HIP(hipStreamSynchronize(c->stream));
}

template <typename T>
void precond_apply(hipStream_t s, pe_context* c, const double* x, double* z) {
  for (auto& t : c->pc.types) {
    const int nbt = (int)t.bodies.size();
    if (nbt == 0) continue;
    const int Np = t.N + 1;
    const T* A;
    if constexpr (sizeof(T) == 8) A = t.Ainv.get();
    else A = t.Ainv32.get();
    dim3 grid((unsigned)((Np + kBM - 1) / kBM), (unsigned)((nbt + kBN - 1) / kBN));
    hipLaunchKernelGGL(apply_type_kernel<T>, grid, dim3(256), 0, s, A, t.N, t.dbodies.get(), nbt, c->off.get(),
                       c->n_bead, x, z);
    PE_CHECK_LAUNCH();
  }
}

template void precond_apply<float>(hipStream_t, pe_context*, const double*, double*);
template void precond_apply<double>(hipStream_t, pe_context*, const double*, double*);

}  // namespace pe
