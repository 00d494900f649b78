// Double-precision reductions and vector kernels: charge moments for the k=0
// constant of the split, per-body segmented sums (the summation tensor
// Sigma and its transpose, appendix "Summation Tensors"), body outputs
// (dipole, force, torque, energy), and the GMRES building blocks (multi-dot
// and multi-axpy for classical Gram-Schmidt, Givens rotations, back
// substitution).  Every reduction is two-stage with a fixed order, so
// results are bitwise reproducible run to run.
#include <algorithm>

#include "pe_internal.hpp"
#include "vector.hpp"

namespace pe {

namespace {

constexpr int kBS = 256;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of K values per thread; result valid in thread 0 (out[k]).
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* out) {
  __shared__ double sh[kBS / 64][K > 0 ? K : 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wsum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[w][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// partial[blk*2 + {0,1}] = sum q, sum sigma^2 q over this block's range
__global__ void __launch_bounds__(kBS) moments_partial_kernel(const double* __restrict__ q,
                                                              const double* __restrict__ sig,
                                                              double sig_const, int64_t n,
                                                              double* __restrict__ partial) {
  double v[2] = {0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double s = sig ? sig[i] : sig_const;
    v[0] += q[i];
    v[1] += s * s * q[i];
  }
  __shared__ double o[2];
  block_sum<2>(v, o);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = o[0];
    partial[2 * blockIdx.x + 1] = o[1];
  }
}

// ck[0], ck[1]: the k=0 constant at a target of width sigma_t is
// ck[0] - ck[1] sigma_t^2 (see the split in the real-space unit).
__global__ void moments_final_kernel(const double* __restrict__ partial, int nb, CkCoef cc,
                                     double* __restrict__ ck, double* __restrict__ tot) {
  double v[2] = {0, 0};
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    v[0] += partial[2 * i];
    v[1] += partial[2 * i + 1];
  }
  __shared__ double o[2];
  block_sum<2>(v, o);
  if (threadIdx.x == 0) {
    const double Sq = o[0], Ssq = o[1];
    if (cc.reg == PE_REG_GAUSSIAN) {
      ck[0] = cc.inv_epsV * (Sq * cc.inv4xi2 - 0.5 * Ssq);
      ck[1] = cc.inv_epsV * 0.5 * Sq;
    } else if (cc.reg == PE_REG_SHELL_PAPER) {
      // (1 - h) j0^2 / k^2 -> 1 / (4 xi^2) as k -> 0
      ck[0] = cc.inv_epsV * cc.inv4xi2 * Sq;
      ck[1] = 0.0;
    } else {
      ck[0] = cc.inv_epsV * (cc.inv4xi2 - cc.a * cc.a / 3.0) * Sq;
      ck[1] = 0.0;
    }
    if (tot) {
      tot[0] = Sq;
      tot[1] = Ssq;
    }
  }
}

// out[b] = sum of x over the beads of body b (one block per body)
__global__ void __launch_bounds__(kBS) seg_sum_kernel(const int64_t* __restrict__ off,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ out) {
  const int b = blockIdx.x;
  double v[1] = {0};
  for (int64_t i = off[b] + threadIdx.x; i < off[b + 1]; i += blockDim.x) v[0] += x[i];
  __shared__ double o[1];
  block_sum<1>(v, o);
  if (threadIdx.x == 0) out[b] = o[0];
}

// Body outputs from bead data: S = sum r q, F = sum f, L = sum r x f, U = sum u.
__global__ void __launch_bounds__(kBS) body_outputs_kernel(
    const int64_t* __restrict__ off, const double* __restrict__ rel, const double* __restrict__ q,
    const double* __restrict__ f, const double* __restrict__ u, double* __restrict__ S,
    double* __restrict__ F, double* __restrict__ L, double* __restrict__ U) {
  const int b = blockIdx.x;
  double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = off[b] + threadIdx.x; i < off[b + 1]; i += blockDim.x) {
    const double rx = rel[3 * i], ry = rel[3 * i + 1], rz = rel[3 * i + 2];
    const double qi = q[i];
    v[0] += rx * qi;
    v[1] += ry * qi;
    v[2] += rz * qi;
    if (f) {
      const double fx = f[3 * i], fy = f[3 * i + 1], fz = f[3 * i + 2];
      v[3] += fx;
      v[4] += fy;
      v[5] += fz;
      v[6] += ry * fz - rz * fy;
      v[7] += rz * fx - rx * fz;
      v[8] += rx * fy - ry * fx;
      v[9] += u[i];
    }
  }
  __shared__ double o[10];
  block_sum<10>(v, o);
  if (threadIdx.x == 0) {
    if (S) { S[3 * b] = o[0]; S[3 * b + 1] = o[1]; S[3 * b + 2] = o[2]; }
    if (F) { F[3 * b] = o[3]; F[3 * b + 1] = o[4]; F[3 * b + 2] = o[5]; }
    if (L) { L[3 * b] = o[6]; L[3 * b + 1] = o[7]; L[3 * b + 2] = o[8]; }
    if (U) U[b] = o[9];
  }
}

// partial[k * gridDim.x + c] = V_k . w over chunk c (grid: chunks x K)
__global__ void __launch_bounds__(kBS) mdot_partial_kernel(const double* __restrict__ V, int64_t ldv,
                                                           const double* __restrict__ w, int64_t n,
                                                           int64_t chunk, double* __restrict__ partial) {
  const int k = blockIdx.y;
  const double* v = V + (int64_t)k * ldv;
  const int64_t b = (int64_t)blockIdx.x * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  double acc[1] = {0};
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) acc[0] += v[i] * w[i];
  __shared__ double o[1];
  block_sum<1>(acc, o);
  if (threadIdx.x == 0) partial[(int64_t)k * gridDim.x + blockIdx.x] = o[0];
}

__global__ void mdot_final_kernel(const double* __restrict__ partial, int nb, int K, double* __restrict__ out,
                                  int sqrt_flag) {
  // one wavefront per output
  const int k = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < nb; i += 64) s += partial[(int64_t)k * nb + i];
  s = wsum(s);
  if (threadIdx.x == 0) out[k] = sqrt_flag ? sqrt(s) : s;
}

// w -= sum_k h[k] V_k   (h on the device)
__global__ void __launch_bounds__(kBS) maxpy_kernel(const double* __restrict__ V, int64_t ldv, int K,
                                                    const double* __restrict__ h, double* __restrict__ w,
                                                    int64_t n, double sign) {
  __shared__ double hs[kMaxK];
  if (threadIdx.x < K) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int k = 0; k < K; ++k) s += hs[k] * V[k * ldv + i];
    w[i] -= sign * s;
  }
}

// vout = w / *nrm  (guarding a zero norm)
__global__ void scale_kernel(const double* __restrict__ w, const double* __restrict__ nrm,
                             double* __restrict__ vout, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = *nrm;
  vout[i] = d > 0 ? w[i] / d : 0.0;
}

// y = a*x + b*y
__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = a * x[i] + b * y[i];
}

// z = x - y
__global__ void sub_kernel(const double* __restrict__ x, const double* __restrict__ y, double* __restrict__ z,
                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  z[i] = x[i] - y[i];
}

// Arnoldi column j: h = h1 + h2 (two Gram-Schmidt passes), subdiagonal = norm.
// Apply the previous rotations, form the new one, update g; return |g[j+1]|.
// Layout of st (double): H[(m+1) x m] column-major at 0, cs[m], sn[m], g[m+1].
__device__ double givens_step(const double* __restrict__ h1, const double* __restrict__ h2, double nrm,
                              double* __restrict__ st, int m, int j) {
  double* H = st;
  double* cs = st + (m + 1) * m;
  double* sn = cs + m;
  double* g = sn + m;
  double* col = H + (int64_t)j * (m + 1);
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  col[j + 1] = nrm;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double r = hypot(a, b);
  const double c = r > 0 ? a / r : 1.0;
  const double s = r > 0 ? b / r : 0.0;
  cs[j] = c;
  sn[j] = s;
  col[j] = r;
  col[j + 1] = 0.0;
  const double gj = g[j];
  g[j] = c * gj;
  g[j + 1] = -s * gj;
  return fabs(g[j + 1]);
}

__global__ void givens_kernel(const double* __restrict__ h1, const double* __restrict__ h2,
                              const double* __restrict__ nrm, double* __restrict__ st, int m, int j,
                              double* __restrict__ res) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  *res = givens_step(h1, h2, *nrm, st, m, j);
}

// One Arnoldi step in four launches instead of a reduction kernel per pass:
// each kernel below starts by finishing the previous kernel's reduction
// itself (every workgroup sums the same partials in the same fixed order, so
// all of them hold the same values bit for bit), then updates its chunk of w
// and writes its own partial sums for the next one.  No workgroup waits on
// another inside a kernel.

// out[k] = sum of the nb partials of output k (partial[k * nb + i]): lane l
// takes i = l, l + 64, ..., then the wavefront tree; wavefront q of the
// workgroup takes k = q, q + 4, ...
__device__ void final_sums(const double* __restrict__ partial, int nb, int K, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = wv; k < K; k += nw) {
    double s = 0;
    for (int i = lane; i < nb; i += 64) s += partial[(int64_t)k * nb + i];
    s = wsum(s);
    if (lane == 0) out[k] = s;
  }
}

// Gram-Schmidt pass: h = the previous pass's dot products (from pin, nb
// partials each; workgroup 0 also stores them in hout), w -= V h over the
// workgroup's chunk, then the partial sums for the next reduction: V_k . w,
// k < K, or (NORM) w . w.
template <bool NORM>
__global__ void __launch_bounds__(kBS) cgs_pass_kernel(const double* __restrict__ V, int64_t ldv, int K,
                                                       const double* __restrict__ pin, double* __restrict__ hout,
                                                       double* __restrict__ w, int64_t n, int64_t chunk,
                                                       double* __restrict__ pout) {
  __shared__ double hs[kMaxK];
  final_sums(pin, (int)gridDim.x, K, hs);
  __syncthreads();
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < K; k += blockDim.x) hout[k] = hs[k];
  const int64_t b = (int64_t)blockIdx.x * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  if constexpr (NORM) {
    double acc[1] = {0};
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
      double s = 0;
      for (int k = 0; k < K; ++k) s += hs[k] * V[k * ldv + i];
      const double wi = w[i] - s;
      w[i] = wi;
      acc[0] += wi * wi;
    }
    __shared__ double o[1];
    block_sum<1>(acc, o);
    if (threadIdx.x == 0) pout[blockIdx.x] = o[0];
  } else {
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
      double s = 0;
      for (int k = 0; k < K; ++k) s += hs[k] * V[k * ldv + i];
      w[i] -= s;
    }
    // each thread reads back only the elements it wrote
    __shared__ double red[kMaxK][kBS / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < K; ++k) {
      double t = 0;
      for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) t += V[k * ldv + i] * w[i];
      t = wsum(t);
      if (lane == 0) red[k][wv] = t;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      double p = 0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) p += red[k][q];
      pout[(int64_t)k * gridDim.x + blockIdx.x] = p;
    }
  }
}

// End of the step: ||w|| from the norm partials, vout = w / ||w|| over the
// workgroup's chunk; workgroup 0 stores the norm and takes the Givens step of
// column j (h1 + h2, ||w||), writing the residual estimate to *res and, when
// given, to page-locked host memory (read by the host after the stream
// reaches an event recorded behind this kernel).
__global__ void __launch_bounds__(kBS) cgs_finish_kernel(const double* __restrict__ w, int64_t n, int64_t chunk,
                                                         const double* __restrict__ pnorm,
                                                         const double* __restrict__ h1,
                                                         const double* __restrict__ h2, double* __restrict__ nrm,
                                                         double* __restrict__ vout, double* __restrict__ st, int m,
                                                         int j, double* __restrict__ res, double* res_host) {
  __shared__ double ss[1];
  final_sums(pnorm, (int)gridDim.x, 1, ss);
  __syncthreads();
  const double d = sqrt(ss[0]);
  const int64_t b = (int64_t)blockIdx.x * chunk;
  const int64_t e = b + chunk < n ? b + chunk : n;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) vout[i] = d > 0 ? w[i] / d : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *nrm = d;
    const double r = givens_step(h1, h2, d, st, m, j);
    *res = r;
    if (res_host) {
      *res_host = r;
      __threadfence_system();
    }
  }
}

// g = [beta, 0, ...]
__global__ void init_g_kernel(double* __restrict__ st, int m, const double* __restrict__ beta) {
  double* g = st + (m + 1) * m + 2 * m;
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = (i == 0) ? *beta : 0.0;
}

// Back substitution R y = g for the first k columns; y -> ybuf.
__global__ void backsolve_kernel(const double* __restrict__ st, int m, int k, double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double* H = st;
  const double* g = st + (m + 1) * m + 2 * m;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < k; ++l) s -= H[(int64_t)l * (m + 1) + i] * y[l];
    const double d = H[(int64_t)i * (m + 1) + i];
    y[i] = d != 0 ? s / d : 0.0;
  }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
inline unsigned nred(int64_t n) {
  int64_t b = (n + kBS * 4 - 1) / (kBS * 4);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (unsigned)b;
}


// Segmented sort: one workgroup per segment.  Segments of up to kSortMax keys
// are sorted in LDS by a bitonic network in the form where every comparator
// puts the smaller key at the lower index, so padding with INT_MAX past the
// end needs no special case.  Longer segments (none at the workloads'
// densities) fall back to an insertion sort by one thread.
constexpr int kSortMax = 4096;

__global__ void __launch_bounds__(256) segment_sort_kernel(const int* __restrict__ start, int* __restrict__ keys) {
  extern __shared__ int key[];  // next power of two of the longest segment (at most kSortMax)
  const int b = start[blockIdx.x], e = start[blockIdx.x + 1];
  const int n = e - b;
  if (n <= 1) return;
  if (n > kSortMax) {
    if (threadIdx.x == 0) {
      for (int i = b + 1; i < e; ++i) {
        const int v = keys[i];
        int j = i - 1;
        while (j >= b && keys[j] > v) {
          keys[j + 1] = keys[j];
          --j;
        }
        keys[j + 1] = v;
      }
    }
    return;
  }
  int m = 1;
  while (m < n) m <<= 1;
  for (int i = threadIdx.x; i < m; i += blockDim.x) key[i] = i < n ? keys[b + i] : 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      // first stage of each merge compares mirrored pairs, later stages halves
      const int mask = (j == (k >> 1)) ? k - 1 : j;
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        if ((i & j) == 0) {
          const int p = i ^ mask;
          const int a = key[i], c = key[p];
          if (a > c) {
            key[i] = c;
            key[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) keys[b + i] = key[i];
}

// One wavefront per segment (segments of at most kWaveSortMax keys): up to
// 64 keys sit one per lane and are sorted by the same network with lane
// shuffles; longer ones in the wavefront's LDS slice, with wavefront-level
// ordering only.  Many short segments (cells, tiles) then cost a few dozen
// instructions each instead of a workgroup with a barrier per stage.
constexpr int kWaveSortMax = 1024;

__global__ void __launch_bounds__(256) segment_sort_wave_kernel(const int* __restrict__ start, int nseg,
                                                                int* __restrict__ keys) {
  __shared__ int buf[4][kWaveSortMax];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sg = blockIdx.x * 4 + wv;
  if (sg >= nseg) return;
  const int b = start[sg], e = start[sg + 1];
  const int n = e - b;
  if (n <= 1) return;
  if (n <= 64) {
    int v = lane < n ? keys[b + lane] : 0x7fffffff;
    for (int k = 2; k <= 64; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int mask = (j == (k >> 1)) ? k - 1 : j;
        const int p = lane ^ mask;
        const int o = __shfl(v, p, 64);
        v = lane < p ? min(v, o) : max(v, o);  // the lower lane keeps the smaller key
      }
    }
    if (lane < n) keys[b + lane] = v;
    return;
  }
  int m = 1;
  while (m < n) m <<= 1;
  int* key = buf[wv];
  for (int i = lane; i < m; i += 64) key[i] = i < n ? keys[b + i] : 0x7fffffff;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int mask = (j == (k >> 1)) ? k - 1 : j;
      for (int i = lane; i < m; i += 64) {
        if ((i & j) == 0) {
          const int p = i ^ mask;
          const int a = key[i], c = key[p];
          if (a > c) {
            key[i] = c;
            key[p] = a;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  for (int i = lane; i < n; i += 64) keys[b + i] = key[i];
}

}  // namespace

void launch_moments(hipStream_t s, const double* q, const double* sig, double sig_const, int64_t n,
                    const CkCoef& cc, double* partial, double* ck, double* tot) {
  const unsigned nb = nred(n);
  hipLaunchKernelGGL(moments_partial_kernel, dim3(nb), dim3(kBS), 0, s, q, sig, sig_const, n, partial);
  PE_CHECK_LAUNCH();
  hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(kBS), 0, s, partial, (int)nb, cc, ck, tot);
  PE_CHECK_LAUNCH();
}

void launch_seg_sum(hipStream_t s, const int64_t* off, int64_t n_body, const double* x, double* out) {
  if (n_body == 0) return;
  hipLaunchKernelGGL(seg_sum_kernel, dim3((unsigned)n_body), dim3(kBS), 0, s, off, x, out);
  PE_CHECK_LAUNCH();
}

void launch_body_outputs(hipStream_t s, const int64_t* off, int64_t n_body, const double* rel, const double* q,
                         const double* f, const double* u, double* S, double* F, double* L, double* U) {
  if (n_body == 0) return;
  hipLaunchKernelGGL(body_outputs_kernel, dim3((unsigned)n_body), dim3(kBS), 0, s, off, rel, q, f, u, S, F, L, U);
  PE_CHECK_LAUNCH();
}

void launch_mdot(hipStream_t s, const double* V, int64_t ldv, int K, const double* w, int64_t n,
                 double* partial, double* out, bool take_sqrt) {
  require(K >= 1 && K <= kMaxK, "mdot: too many vectors");
  int64_t chunk = 1024;
  if ((n + chunk - 1) / chunk > 1024) chunk = (n + 1023) / 1024;
  const unsigned nb = (unsigned)std::max<int64_t>(1, (n + chunk - 1) / chunk);
  hipLaunchKernelGGL(mdot_partial_kernel, dim3(nb, K), dim3(kBS), 0, s, V, ldv, w, n, chunk, partial);
  PE_CHECK_LAUNCH();
  hipLaunchKernelGGL(mdot_final_kernel, dim3(K), dim3(64), 0, s, partial, (int)nb, K, out, take_sqrt ? 1 : 0);
  PE_CHECK_LAUNCH();
}

void launch_maxpy(hipStream_t s, const double* V, int64_t ldv, int K, const double* h, double* w, int64_t n,
                  double sign) {
  require(K >= 1 && K <= kMaxK, "maxpy: too many vectors");
  unsigned nb = nblk(n, kBS);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(maxpy_kernel, dim3(nb), dim3(kBS), 0, s, V, ldv, K, h, w, n, sign);
  PE_CHECK_LAUNCH();
}

void launch_scale(hipStream_t s, const double* w, const double* nrm, double* vout, int64_t n) {
  hipLaunchKernelGGL(scale_kernel, dim3(nblk(n, kBS)), dim3(kBS), 0, s, w, nrm, vout, n);
  PE_CHECK_LAUNCH();
}

void launch_axpby(hipStream_t s, double a, const double* x, double b, double* y, int64_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(nblk(n, kBS)), dim3(kBS), 0, s, a, x, b, y, n);
  PE_CHECK_LAUNCH();
}

void launch_sub(hipStream_t s, const double* x, const double* y, double* z, int64_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(sub_kernel, dim3(nblk(n, kBS)), dim3(kBS), 0, s, x, y, z, n);
  PE_CHECK_LAUNCH();
}

namespace {
// chunks of the Krylov reductions: 1024 elements, or n / 1024 when that is
// larger, so there are at most 1024 partials per output
int64_t kchunk(int64_t n) {
  int64_t chunk = 1024;
  if ((n + chunk - 1) / chunk > 1024) chunk = (n + 1023) / 1024;
  return chunk;
}
unsigned kchunks(int64_t n, int64_t chunk) { return (unsigned)std::max<int64_t>(1, (n + chunk - 1) / chunk); }
}  // namespace

void launch_cgs_step(hipStream_t s, const double* V, int64_t ldv, int K, double* w, int64_t n, double* partial,
                     double* h1, double* h2, double* nrm, double* vout, double* st, int m, int j, double* res,
                     double* res_host) {
  require(K >= 1 && K <= kMaxK, "Gram-Schmidt: too many vectors");
  const int64_t chunk = kchunk(n);
  const unsigned nb = kchunks(n, chunk);
  double* p1 = partial;
  double* p2 = partial + (size_t)kMaxK * 1024;
  hipLaunchKernelGGL(mdot_partial_kernel, dim3(nb, K), dim3(kBS), 0, s, V, ldv, w, n, chunk, p1);
  PE_CHECK_LAUNCH();
  hipLaunchKernelGGL(cgs_pass_kernel<false>, dim3(nb), dim3(kBS), 0, s, V, ldv, K, p1, h1, w, n, chunk, p2);
  PE_CHECK_LAUNCH();
  hipLaunchKernelGGL(cgs_pass_kernel<true>, dim3(nb), dim3(kBS), 0, s, V, ldv, K, p2, h2, w, n, chunk, p1);
  PE_CHECK_LAUNCH();
  hipLaunchKernelGGL(cgs_finish_kernel, dim3(nb), dim3(kBS), 0, s, w, n, chunk, p1, h1, h2, nrm, vout, st, m, j,
                     res, res_host);
  PE_CHECK_LAUNCH();
}

void launch_givens(hipStream_t s, const double* h1, const double* h2, const double* nrm, double* st, int m,
                   int j, double* res) {
  hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, s, h1, h2, nrm, st, m, j, res);
  PE_CHECK_LAUNCH();
}

void launch_init_g(hipStream_t s, double* st, int m, const double* beta) {
  hipLaunchKernelGGL(init_g_kernel, dim3(1), dim3(64), 0, s, st, m, beta);
  PE_CHECK_LAUNCH();
}

void launch_backsolve(hipStream_t s, const double* st, int m, int k, double* y) {
  hipLaunchKernelGGL(backsolve_kernel, dim3(1), dim3(64), 0, s, st, m, k, y);
  PE_CHECK_LAUNCH();
}

void launch_segment_sort(hipStream_t s, const int* start, int nseg, int* keys, int max_len) {
  if (nseg <= 0 || max_len <= 1) return;
  if (max_len <= kWaveSortMax) {
    hipLaunchKernelGGL(segment_sort_wave_kernel, dim3((unsigned)((nseg + 3) / 4)), dim3(256), 0, s, start, nseg,
                       keys);
    PE_CHECK_LAUNCH();
    return;
  }
  int m = 1;
  while (m < std::min(max_len, kSortMax)) m <<= 1;
  hipLaunchKernelGGL(segment_sort_kernel, dim3((unsigned)nseg), dim3(256), sizeof(int) * (size_t)m, s, start, keys);
  PE_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ scan
//
// Exclusive prefix sum of int counts into 64-bit offsets in three launches:
// per-tile totals (kScanTile values per block), one block scanning the
// totals in order, then every tile scanned again locally and offset.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

__global__ void __launch_bounds__(kScanThreads) scan_tile_sum_kernel(const int* __restrict__ in, int64_t n,
                                                                     int64_t* __restrict__ tot) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t v = 0;
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) v += in[i];
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __shared__ int64_t sh[kScanThreads / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += sh[w];
    tot[blockIdx.x] = t;
  }
}

// One block: tot[b] <- sum of tot[0..b), tot[nt] <- total.  Each thread
// scans a contiguous run serially; the run totals are scanned in LDS.
__global__ void __launch_bounds__(1024) scan_tile_offsets_kernel(int64_t* __restrict__ tot, int64_t nt) {
  __shared__ int64_t run[1024];
  const int64_t per = (nt + 1023) / 1024;
  const int64_t b0 = threadIdx.x * per, b1 = min(nt, b0 + per);
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += tot[b];
  run[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int k = 0; k < 1024; ++k) {
      const int64_t t = run[k];
      run[k] = acc;
      acc += t;
    }
    tot[nt] = acc;
  }
  __syncthreads();
  int64_t acc = run[threadIdx.x];
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t t = tot[b];
    tot[b] = acc;
    acc += t;
  }
}

__global__ void __launch_bounds__(kScanThreads) scan_tile_write_kernel(const int* __restrict__ in, int64_t n,
                                                                       const int64_t* __restrict__ tot,
                                                                       int64_t* __restrict__ out) {
  // thread t owns the kScanPer consecutive values t * kScanPer .. of the tile
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int v[kScanPer];
  int64_t own = 0;
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    own += v[k];
  }
  // exclusive scan of the per-thread totals across the block
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = own;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  __shared__ int64_t wsum[kScanThreads / 64];
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int64_t pre = tot[blockIdx.x];
  for (int k = 0; k < w; ++k) pre += wsum[k];
  int64_t acc = pre + inc - own;
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = acc;
    acc += v[k];
  }
}

int64_t scan_workspace(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_exclusive_scan(hipStream_t s, const int* in, int64_t n, int64_t* out, int64_t* tmp) {
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  if (nt > 0) {
    hipLaunchKernelGGL(scan_tile_sum_kernel, dim3((unsigned)nt), dim3(kScanThreads), 0, s, in, n, tmp);
    PE_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(scan_tile_offsets_kernel, dim3(1), dim3(1024), 0, s, tmp, nt);
  PE_CHECK_LAUNCH();
  if (nt > 0) {
    hipLaunchKernelGGL(scan_tile_write_kernel, dim3((unsigned)nt), dim3(kScanThreads), 0, s, in, n, tmp, out);
    PE_CHECK_LAUNCH();
  }
  // out[n] = total
  PE_HIP(hipMemcpyAsync(out + n, tmp + nt, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
}

}  // namespace pe
