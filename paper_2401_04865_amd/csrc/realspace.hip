// Real-space part of the Ewald split (section "Real-space sum"): linked
// cells of edge >= r_c, 27-cell stencil (one cell per axis when the box holds
// fewer than three, with the minimum image taking care of periodicity since
// r_c <= L/2).
//
// Kernel of the split (regularization entirely in real space, point-charge
// wave space):
//   Gaussian, s^2 = sigma_a^2 + sigma_b^2, b = 1/(sqrt2 s):
//     R(r) = [erf(b r) - erf(xi r)] / (4 pi eps r),  R(0) = (2/sqrt pi)(b - xi)/(4 pi eps)
//   Shell of radius a:
//     R(r) = M_shell(r) - erf(xi r)/(4 pi eps r), M_shell = 1/(4 pi eps r) (r >= 2a),
//            (4a - r)/(16 pi eps a^2) (r < 2a);  R(0) = 1/(4 pi eps a) - xi/(2 pi^1.5 eps)
// The difference of error functions is formed as erf - erf where both are
// small and as erfc - erfc where both are close to one, so neither loses
// digits to cancellation.
//
// Positions are fixed during a solve, so the bead-bead block is evaluated once
// per configuration and stored as a CSR matrix (rows in cell order, entries
// in traversal order).  Every Krylov iteration then applies it as a sparse
// matrix-vector product.  One-off passes (ion -> bead for the right-hand
// side, all pairs with fields for the forces) are evaluated on the fly.
#include <algorithm>
#include <numeric>

#include "pe_internal.hpp"
#include "vector.hpp"

namespace pe {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv4Pi = 0.07957747154594766788;
constexpr double kTwoOverSqrtPi = 1.12837916709551257390;

__device__ __forceinline__ int cell_coord(double x, double inv, int nc) {
  int c = (int)(x * inv);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ double min_img(double d, double L, double invL) {
  return d - L * rint(d * invL);
}

template <typename T>
__device__ __forceinline__ T erf_diff(T b, T xi, T r) {
  // erf(b r) - erf(xi r)
  if (b * r < (T)1.0) return erf(b * r) - erf(xi * r);
  return erfc(xi * r) - erfc(b * r);
}

// R(r) and dR/dr for one pair (r > 0).
template <typename T>
__device__ __forceinline__ void pair_kernel(T r, T s2, const RealGeom& g, T& R, T& dR, bool want_d) {
  const T xi = (T)g.xi;
  const T c = (T)(kInv4Pi / g.eps);
  const T inv_r = (T)1 / r;
  if (g.reg == PE_REG_GAUSSIAN) {
    const T b = rsqrt((T)2 * s2);
    const T D = erf_diff<T>(b, xi, r);
    R = c * D * inv_r;
    if (want_d) {
      // d/dr [D/r] = (D' r - D)/r^2, D' = (2/sqrt pi)(b e^{-b^2 r^2} - xi e^{-xi^2 r^2})
      const T Dp = (T)kTwoOverSqrtPi * (b * exp(-b * b * r * r) - xi * exp(-xi * xi * r * r));
      dR = c * (Dp * r - D) * inv_r * inv_r;
    }
  } else {
    const T a = (T)g.a;
    const T erfx = erf(xi * r);
    T Ms, dMs;
    if (r >= (T)2 * a) {
      // M_shell - erf/(4 pi r) = erfc/(4 pi r)
      const T ec = erfc(xi * r);
      R = c * ec * inv_r;
      if (want_d) {
        const T dec = -(T)kTwoOverSqrtPi * xi * exp(-xi * xi * r * r);
        dR = c * (dec * r - ec) * inv_r * inv_r;
      }
      return;
    }
    Ms = c * ((T)4 * a - r) / ((T)4 * a * a);
    dMs = -c / ((T)4 * a * a);
    R = Ms - c * erfx * inv_r;
    if (want_d) {
      const T de = (T)kTwoOverSqrtPi * xi * exp(-xi * xi * r * r);
      dR = dMs - c * (de * r - erfx) * inv_r * inv_r;
    }
  }
}

template <typename T>
__device__ __forceinline__ T self_value(T s2, const RealGeom& g) {
  const T c = (T)(kInv4Pi / g.eps);
  if (g.reg == PE_REG_GAUSSIAN) return c * (T)kTwoOverSqrtPi * (rsqrt((T)2 * s2) - (T)g.xi);
  return c * ((T)1 / (T)g.a - (T)2 * (T)g.xi / (T)sqrt(kPi));
}

// ---------------------------------------------------------------- cell list

__global__ void assign_cells_kernel(const double* __restrict__ pos, const double* __restrict__ sig,
                                    double sig_const, int64_t n, RealGeom g, double4* __restrict__ tmp,
                                    int* __restrict__ cell_of, int* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  x -= g.L[0] * floor(x * g.inv_L[0]);
  y -= g.L[1] * floor(y * g.inv_L[1]);
  z -= g.L[2] * floor(z * g.inv_L[2]);
  if (x >= g.L[0]) x -= g.L[0];
  if (y >= g.L[1]) y -= g.L[1];
  if (z >= g.L[2]) z -= g.L[2];
  const double s = sig ? sig[i] : sig_const;
  tmp[i] = make_double4(x, y, z, s);
  const int cx = cell_coord(x, g.cell_inv[0], g.nc[0]);
  const int cy = cell_coord(y, g.cell_inv[1], g.nc[1]);
  const int cz = cell_coord(z, g.cell_inv[2], g.nc[2]);
  const int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
  cell_of[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ void scatter_cells_kernel(const int* __restrict__ cell_of, int64_t n,
                                     int* __restrict__ cursor, int* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int slot = atomicAdd(&cursor[cell_of[i]], 1);
  idx[slot] = (int)i;
}

__global__ void gather_sorted_kernel(const double4* __restrict__ tmp, const int* __restrict__ idx,
                                     int64_t n, double4* __restrict__ pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pos[i] = tmp[idx[i]];
}

// ------------------------------------------------------------ pair traversal

// Visit every source within r_c of target point p: f(slot, dx, dy, dz, r2, src_sigma).
template <typename F>
__device__ __forceinline__ void for_neighbours(const double4 p, const double4* __restrict__ spos,
                                               const int* __restrict__ start, const RealGeom& g, F&& f) {
  const int cx = cell_coord(p.x, g.cell_inv[0], g.nc[0]);
  const int cy = cell_coord(p.y, g.cell_inv[1], g.nc[1]);
  const int cz = cell_coord(p.z, g.cell_inv[2], g.nc[2]);
  const int rx = g.nc[0] >= 3 ? 1 : 0, ry = g.nc[1] >= 3 ? 1 : 0, rz = g.nc[2] >= 3 ? 1 : 0;
  for (int ox = -rx; ox <= rx; ++ox) {
    int x = cx + ox;
    x += (x < 0) ? g.nc[0] : (x >= g.nc[0] ? -g.nc[0] : 0);
    for (int oy = -ry; oy <= ry; ++oy) {
      int y = cy + oy;
      y += (y < 0) ? g.nc[1] : (y >= g.nc[1] ? -g.nc[1] : 0);
      for (int oz = -rz; oz <= rz; ++oz) {
        int z = cz + oz;
        z += (z < 0) ? g.nc[2] : (z >= g.nc[2] ? -g.nc[2] : 0);
        const int c = (x * g.nc[1] + y) * g.nc[2] + z;
        const int e = start[c + 1];
        for (int s = start[c]; s < e; ++s) {
          const double4 q = spos[s];
          const double dx = min_img(p.x - q.x, g.L[0], g.inv_L[0]);
          const double dy = min_img(p.y - q.y, g.L[1], g.inv_L[1]);
          const double dz = min_img(p.z - q.z, g.L[2], g.inv_L[2]);
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 < g.rc2) f(s, dx, dy, dz, r2, q.w);
        }
      }
    }
  }
}

// Count bead neighbours (incl. the bead itself) of every sorted bead.
__global__ void count_pairs_kernel(const double4* __restrict__ pos, const int* __restrict__ start,
                                   int64_t n, RealGeom g, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int k = 0;
  for_neighbours(pos[i], pos, start, g, [&](int, double, double, double, double, double) { ++k; });
  cnt[i] = k;
}

__global__ void fill_pairs_kernel(const double4* __restrict__ pos, const int* __restrict__ idx,
                                  const int* __restrict__ start, int64_t n, RealGeom g,
                                  const int64_t* __restrict__ row_ptr, int* __restrict__ col,
                                  double* __restrict__ v64, float* __restrict__ v32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 p = pos[i];
  int64_t o = row_ptr[i];
  for_neighbours(p, pos, start, g, [&](int s, double, double, double, double r2, double sw) {
    const double s2 = p.w * p.w + sw * sw;
    double R;
    if (r2 == 0.0) {
      R = self_value<double>(s2, g);
    } else {
      double dR;
      pair_kernel<double>(sqrt(r2), s2, g, R, dR, false);
    }
    col[o] = idx[s];
    v64[o] = R;
    if (v32) v32[o] = (float)R;
    ++o;
  });
}

// y_top[b] = -(phi_wave[b] + sum_j R_bj q_j - ck0_b) + dpsi[body(b)] for every bead b.
// ck0_b = ck[0] - ck[1] * sigma_b^2 (the k = 0 constant of the split).
// CSR rows in cell order; 16 lanes per row read the row's entries
// contiguously and reduce with lane shuffles (4 rows per wavefront).
template <typename T>
__global__ void __launch_bounds__(256) spmv_assemble_kernel(
    const int64_t* __restrict__ row_ptr, const int* __restrict__ col, const T* __restrict__ val,
    const int* __restrict__ idx, const double4* __restrict__ pos, int64_t n,
    const double* __restrict__ q, const double* __restrict__ phi_wave, const double* __restrict__ ck,
    const double* __restrict__ dpsi, const int* __restrict__ body_of, double* __restrict__ y) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int sub = threadIdx.x & 15;
  T acc = 0;
  if (i < n) {
    const int64_t e = row_ptr[i + 1];
    for (int64_t o = row_ptr[i] + sub; o < e; o += 16) acc += val[o] * (T)q[col[o]];
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
  if (i < n && sub == 0) {
    const int b = idx[i];
    const double sg = pos[i].w;
    const double phi = (double)acc + phi_wave[b] - (ck[0] - ck[1] * sg * sg);
    y[b] = -phi + (dpsi ? dpsi[body_of[b]] : 0.0);
  }
}

// On-the-fly potential (and field) at targets from sources; adds into
// phi[idx_t] and E[3 idx_t + d].
template <typename T, bool FIELD>
__global__ void __launch_bounds__(256) pair_onfly_kernel(
    const double4* __restrict__ tpos, const int* __restrict__ tidx, int64_t nt,
    const double4* __restrict__ spos, const int* __restrict__ sidx, const int* __restrict__ sstart,
    const double* __restrict__ q, RealGeom g, double* __restrict__ phi, double* __restrict__ E) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const double4 p = tpos[i];
  T acc = 0, ex = 0, ey = 0, ez = 0;
  for_neighbours(p, spos, sstart, g, [&](int s, double dx, double dy, double dz, double r2, double sw) {
    const T qs = (T)q[sidx[s]];
    const T s2 = (T)(p.w * p.w + sw * sw);
    if (r2 == 0.0) {
      acc += self_value<T>(s2, g) * qs;
      return;
    }
    T R, dR = 0;
    const T r = (T)sqrt(r2);
    pair_kernel<T>(r, s2, g, R, dR, FIELD);
    acc += R * qs;
    if (FIELD) {
      const T f = -dR / r * qs;  // E = -grad_t R q = -R'(r) d/r q
      ex += f * (T)dx;
      ey += f * (T)dy;
      ez += f * (T)dz;
    }
  });
  const int o = tidx[i];
  phi[o] += (double)acc;
  if (FIELD) {
    E[3 * o] += (double)ex;
    E[3 * o + 1] += (double)ey;
    E[3 * o + 2] += (double)ez;
  }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void build_cells(hipStream_t s, ParticleSet& ps, const double* pos_caller, const double* sig_caller,
                 double sig_const, int64_t n, const RealGeom& rg) {
  ps.n = n;
  const int ncell = rg.nc[0] * rg.nc[1] * rg.nc[2];
  ps.pos.ensure(n);
  ps.idx.ensure(n);
  ps.tmp.ensure(n);
  ps.cell_of.ensure(n);
  ps.cell_start.ensure(ncell + 1);
  ps.cell_count.ensure(ncell);
  PE_HIP(hipMemsetAsync(ps.cell_count.get(), 0, sizeof(int) * ncell, s));
  if (n > 0) {
    hipLaunchKernelGGL(assign_cells_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, pos_caller, sig_caller,
                       sig_const, n, rg, ps.tmp.get(), ps.cell_of.get(), ps.cell_count.get());
    PE_CHECK_LAUNCH();
  }
  std::vector<int> cnt(ncell), start(ncell + 1, 0);
  PE_HIP(hipMemcpyAsync(cnt.data(), ps.cell_count.get(), sizeof(int) * ncell, hipMemcpyDeviceToHost, s));
  PE_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < ncell; ++c) start[c + 1] = start[c] + cnt[c];
  PE_HIP(hipMemcpyAsync(ps.cell_start.get(), start.data(), sizeof(int) * (ncell + 1), hipMemcpyHostToDevice, s));
  // cursor = start (reuse cell_count)
  PE_HIP(hipMemcpyAsync(ps.cell_count.get(), start.data(), sizeof(int) * ncell, hipMemcpyHostToDevice, s));
  if (n > 0) {
    hipLaunchKernelGGL(scatter_cells_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, ps.cell_of.get(), n,
                       ps.cell_count.get(), ps.idx.get());
    PE_CHECK_LAUNCH();
    // sort each cell's slice by caller index so the order (and every sum over
    // it) is the same on every run
    launch_segment_sort(s, ps.cell_start.get(), ncell, ps.idx.get());
    hipLaunchKernelGGL(gather_sorted_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, ps.tmp.get(),
                       ps.idx.get(), n, ps.pos.get());
    PE_CHECK_LAUNCH();
  }
  // the host vectors go out of scope after the copies above complete
  PE_HIP(hipStreamSynchronize(s));
}

void build_bead_matrix(pe_context* c) {
  hipStream_t s = c->stream;
  const int64_t n = c->n_bead;
  ParticleSet& B = c->B;
  c->cnt.ensure(n);
  if (n > 0) {
    hipLaunchKernelGGL(count_pairs_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, B.pos.get(),
                       B.cell_start.get(), n, c->rg, c->cnt.get());
    PE_CHECK_LAUNCH();
  }
  std::vector<int> cnt(n);
  if (n > 0) PE_HIP(hipMemcpyAsync(cnt.data(), c->cnt.get(), sizeof(int) * n, hipMemcpyDeviceToHost, s));
  PE_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> rp(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) rp[i + 1] = rp[i] + cnt[i];
  c->nnz = rp[n];
  c->row_ptr.ensure(n + 1);
  c->col.ensure(c->nnz);
  c->val64.ensure(c->nnz);
  c->have_val32 = c->p.precision == PE_MIXED;
  if (c->have_val32) c->val32.ensure(c->nnz);
  PE_HIP(hipMemcpyAsync(c->row_ptr.get(), rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
  if (n > 0) {
    hipLaunchKernelGGL(fill_pairs_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, B.pos.get(), B.idx.get(),
                       B.cell_start.get(), n, c->rg, c->row_ptr.get(), c->col.get(), c->val64.get(),
                       c->have_val32 ? c->val32.get() : (float*)nullptr);
    PE_CHECK_LAUNCH();
  }
  PE_HIP(hipStreamSynchronize(s));
}

template <typename T>
void launch_spmv_assemble(hipStream_t s, pe_context* c, const double* q, const double* dpsi,
                          const double* phi_wave, const double* ck0, double* y_top) {
  const int64_t n = c->n_bead;
  if (n == 0) return;
  const T* val;
  if constexpr (sizeof(T) == 8) val = c->val64.get();
  else {
    require(c->have_val32, "float real-space operator not built (precision is PE_FP64)");
    val = c->val32.get();
  }
  hipLaunchKernelGGL(spmv_assemble_kernel<T>, dim3(nblk(16 * n, 256)), dim3(256), 0, s, c->row_ptr.get(),
                     c->col.get(), val, c->B.idx.get(), c->B.pos.get(), n, q, phi_wave, ck0, dpsi,
                     c->body_of.get(), y_top);
  PE_CHECK_LAUNCH();
}

template <typename T>
void launch_pair_onfly(hipStream_t s, const ParticleSet& tgt, const ParticleSet& src, const double* q_src,
                       const RealGeom& rg, double* phi, double* E) {
  if (tgt.n == 0 || src.n == 0) return;
  if (E)
    hipLaunchKernelGGL((pair_onfly_kernel<T, true>), dim3(nblk(tgt.n, 256)), dim3(256), 0, s,
                       tgt.pos.get(), tgt.idx.get(), tgt.n, src.pos.get(), src.idx.get(),
                       src.cell_start.get(), q_src, rg, phi, E);
  else
    hipLaunchKernelGGL((pair_onfly_kernel<T, false>), dim3(nblk(tgt.n, 256)), dim3(256), 0, s,
                       tgt.pos.get(), tgt.idx.get(), tgt.n, src.pos.get(), src.idx.get(),
                       src.cell_start.get(), q_src, rg, phi, E);
  PE_CHECK_LAUNCH();
}

template void launch_spmv_assemble<float>(hipStream_t, pe_context*, const double*, const double*, const double*, const double*, double*);
template void launch_spmv_assemble<double>(hipStream_t, pe_context*, const double*, const double*, const double*, const double*, double*);
template void launch_pair_onfly<float>(hipStream_t, const ParticleSet&, const ParticleSet&, const double*, const RealGeom&, double*, double*);
template void launch_pair_onfly<double>(hipStream_t, const ParticleSet&, const ParticleSet&, const double*, const RealGeom&, double*, double*);

}  // namespace pe
