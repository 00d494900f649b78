// Gaussian spreading and contraction (section "Spectral Ewald
// implementation", steps 2 and 6; window of section "Wave-space sum").
//
// One 64-lane wavefront per particle.  Lanes 0..3P-1 first evaluate the
// separable window factors w_x[j], w_y[j], w_z[j] (3P exponentials per
// particle instead of P^3) and the wrapped grid indices into LDS; then the
// wavefront sweeps the P x P (y,z) lines of the support, lane t owning line
// (t / P, t % P) and looping over the P x-points.  Consecutive lanes touch
// consecutive z addresses.  Particles are visited in cell order, so
// neighbouring wavefronts work on neighbouring grid regions (cache reuse).
//
// Support (the P closest grid points per axis): even P takes
// m0-P/2+1 .. m0+P/2 with m0 = floor(x/h); odd P is centred on rint(x/h).
// Index and displacement are computed in double for both precisions, so
// the float and double paths use the same support.
#include "pe_internal.hpp"

namespace pe {

namespace {

constexpr int kWaves = 4;      // particles per 256-thread block
constexpr int kMaxP = 16;

template <typename T>
__device__ __forceinline__ void window_setup(const double4 p, const GridGeom& g, int lane,
                                             T* w_s, int* i_s, T* d_s) {
  const int P = g.P;
  if (lane < 3 * P) {
    const int ax = lane / P;
    const int j = lane - ax * P;
    const double x = ax == 0 ? p.x : (ax == 1 ? p.y : p.z);
    const double u = x * g.inv_h[ax];
    const long m0 = (P & 1) ? (long)rint(u) - (P - 1) / 2 : (long)floor(u) - P / 2 + 1;
    const long m = m0 + j;
    const double d = (double)m * g.h[ax] - x;
    const int N = g.N[ax];
    long mw = m % N;
    if (mw < 0) mw += N;
    w_s[lane] = (T)(g.wnorm * exp(-g.wexp * d * d));
    i_s[lane] = (int)mw;
    if (d_s) d_s[lane] = (T)d;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) spread_kernel(const double4* __restrict__ pos,
                                                     const int* __restrict__ idx,
                                                     const double* __restrict__ q, int64_t n,
                                                     T* __restrict__ grid, GridGeom g) {
  __shared__ T w_s[kWaves][3 * kMaxP];
  __shared__ int i_s[kWaves][3 * kMaxP];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kWaves + wv;
  const bool live = i < n;
  double4 p = make_double4(0, 0, 0, 0);
  T qi = 0;
  if (live) {
    p = pos[i];
    qi = (T)q[idx[i]];
    window_setup<T>(p, g, lane, w_s[wv], i_s[wv], (T*)nullptr);
  }
  __syncthreads();
  if (!live) return;
  const int P = g.P;
  const int PP = P * P;
  const int64_t sx = (int64_t)g.N[1] * g.N[2];
  for (int t = lane; t < PP; t += 64) {
    const int jy = t / P;
    const int jz = t - jy * P;
    const T wyz = qi * w_s[wv][P + jy] * w_s[wv][2 * P + jz];
    const int64_t off_yz = (int64_t)i_s[wv][P + jy] * g.N[2] + i_s[wv][2 * P + jz];
    for (int jx = 0; jx < P; ++jx) {
      const T v = wyz * w_s[wv][jx];
      atomicAdd(&grid[(int64_t)i_s[wv][jx] * sx + off_yz], v);
    }
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T, bool FIELD>
__global__ void __launch_bounds__(256) gather_kernel(const double4* __restrict__ pos,
                                                     const int* __restrict__ idx, int64_t n,
                                                     const T* __restrict__ grid, GridGeom g,
                                                     double* __restrict__ phi,
                                                     double* __restrict__ E, int accumulate) {
  __shared__ T w_s[kWaves][3 * kMaxP];
  __shared__ T d_s[kWaves][3 * kMaxP];
  __shared__ int i_s[kWaves][3 * kMaxP];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * kWaves + wv;
  const bool live = i < n;
  if (live) window_setup<T>(pos[i], g, lane, w_s[wv], i_s[wv], FIELD ? d_s[wv] : (T*)nullptr);
  __syncthreads();
  if (!live) return;
  const int P = g.P;
  const int PP = P * P;
  const int64_t sx = (int64_t)g.N[1] * g.N[2];
  T acc = 0, ax = 0, ay = 0, az = 0;
  for (int t = lane; t < PP; t += 64) {
    const int jy = t / P;
    const int jz = t - jy * P;
    const T wyz = w_s[wv][P + jy] * w_s[wv][2 * P + jz];
    const int64_t off_yz = (int64_t)i_s[wv][P + jy] * g.N[2] + i_s[wv][2 * P + jz];
    T lacc = 0, lx = 0;
    for (int jx = 0; jx < P; ++jx) {
      const T v = grid[(int64_t)i_s[wv][jx] * sx + off_yz] * w_s[wv][jx];
      lacc += v;
      if (FIELD) lx += v * d_s[wv][jx];
    }
    acc += lacc * wyz;
    if (FIELD) {
      ax += lx * wyz;
      ay += lacc * wyz * d_s[wv][P + jy];
      az += lacc * wyz * d_s[wv][2 * P + jz];
    }
  }
  acc = wave_sum(acc);
  if (FIELD) {
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    az = wave_sum(az);
  }
  if (lane == 0) {
    const int o = idx[i];
    const double ph = (double)acc * (g.h3 / g.eps);
    if (accumulate) phi[o] += ph; else phi[o] = ph;
    if (FIELD) {
      const double ex = g.fcoef * (double)ax, ey = g.fcoef * (double)ay, ez = g.fcoef * (double)az;
      if (accumulate) {
        E[3 * o] += ex; E[3 * o + 1] += ey; E[3 * o + 2] += ez;
      } else {
        E[3 * o] = ex; E[3 * o + 1] = ey; E[3 * o + 2] = ez;
      }
    }
  }
}

}  // namespace

template <typename T>
void launch_spread(hipStream_t s, const ParticleSet& ps, const double* q, T* grid, const GridGeom& g) {
  if (ps.n == 0) return;
  require(g.P <= kMaxP, "support P must be <= 16");
  const int64_t nb = (ps.n + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(spread_kernel<T>, dim3((unsigned)nb), dim3(256), 0, s, ps.pos.get(),
                     ps.idx.get(), q, ps.n, grid, g);
  PE_CHECK_LAUNCH();
}

template <typename T>
void launch_gather(hipStream_t s, const ParticleSet& ps, const T* grid, const GridGeom& g,
                   double* phi, double* E, bool accumulate) {
  if (ps.n == 0) return;
  require(g.P <= kMaxP, "support P must be <= 16");
  const int64_t nb = (ps.n + kWaves - 1) / kWaves;
  if (E)
    hipLaunchKernelGGL((gather_kernel<T, true>), dim3((unsigned)nb), dim3(256), 0, s,
                       ps.pos.get(), ps.idx.get(), ps.n, grid, g, phi, E, accumulate ? 1 : 0);
  else
    hipLaunchKernelGGL((gather_kernel<T, false>), dim3((unsigned)nb), dim3(256), 0, s,
                       ps.pos.get(), ps.idx.get(), ps.n, grid, g, phi, E, accumulate ? 1 : 0);
  PE_CHECK_LAUNCH();
}

template void launch_spread<float>(hipStream_t, const ParticleSet&, const double*, float*, const GridGeom&);
template void launch_spread<double>(hipStream_t, const ParticleSet&, const double*, double*, const GridGeom&);
template void launch_gather<float>(hipStream_t, const ParticleSet&, const float*, const GridGeom&, double*, double*, bool);
template void launch_gather<double>(hipStream_t, const ParticleSet&, const double*, const GridGeom&, double*, double*, bool);

}  // namespace pe
