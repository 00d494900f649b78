// One overdamped Brownian-dynamics step (section "Brownian dynamics
// simulations of charged and polarizable colloids in explicit electrolytes":
// Euler-Maruyama integration of the overdamped Langevin equation, Stokes drag
// gamma per particle, no hydrodynamic interactions between particles).
//
// Ions:   x += f dt / gamma + sqrt(2 kT dt / gamma) xi
// Bodies: a rigid set of N beads, each with drag gamma, moving freely
//         (free draining): translational drag N gamma, rotational drag
//         K = gamma sum_j (|r_j|^2 I - r_j r_j^T) about the centroid;
//         X += F dt / (N gamma) + sqrt(2 kT dt / (N gamma)) xi,
//         dtheta = K^{-1} L dt + sqrt(2 kT dt) C xi   with C C^T = K^{-1},
//         orientation q <- exp(dtheta / 2) q, beads x = X + R(q) r'.
// Gaussian noise: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw 2011) with key =
// seed and counter = (particle, stream, step lo, step hi), two uniforms per
// normal by the Box-Muller transform.  Ions use streams 0/1, bodies 2/3
// (translation / rotation), so every number is fixed by (seed, step, index).
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "pe_internal.hpp"
#include "vector.hpp"

namespace pe {

namespace {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c.x;
    const uint64_t p1 = (uint64_t)M1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// uniform in (0, 1]: (u + 1) / 2^32
__device__ __forceinline__ double uni(uint32_t u) { return ((double)u + 1.0) * 2.3283064365386963e-10; }

// Three standard normals for (index, stream, step).
__device__ __forceinline__ void normals3(uint64_t seed, uint64_t step, uint32_t index, uint32_t stream, double* g) {
  const U4 r = philox4x32_10(U4{index, stream, (uint32_t)step, (uint32_t)(step >> 32)}, (uint32_t)seed,
                             (uint32_t)(seed >> 32));
  const double two_pi = 6.283185307179586477;
  const double a = sqrt(-2.0 * log(uni(r.x))), b = sqrt(-2.0 * log(uni(r.z)));
  g[0] = a * cos(two_pi * uni(r.y));
  g[1] = a * sin(two_pi * uni(r.y));
  g[2] = b * cos(two_pi * uni(r.w));
}

__global__ void bd_ions_kernel(int64_t n, const double* __restrict__ f, double dt, double kT, double gamma,
                               uint64_t seed, uint64_t step, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double g[3];
  normals3(seed, step, (uint32_t)i, 0u, g);
  const double s = sqrt(2.0 * kT * dt / gamma);
  for (int d = 0; d < 3; ++d) x[3 * i + d] += f[3 * i + d] * dt / gamma + s * g[d];
}

__device__ __forceinline__ void quat_to_R(const double* q, double R[3][3]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

// One wavefront per body: the lanes sum the rotational drag over the beads
// (fixed order: lane strides, then a butterfly); lane 0 forms its inverse and
// a Cholesky factor of the inverse, the rigid-body displacement and rotation.
// Writes the new centre/orientation and the rotation (old -> new) for the
// bead update.
__global__ void __launch_bounds__(64) bd_bodies_kernel(int64_t nb, const int64_t* __restrict__ off,
                                                       const double* __restrict__ rel, const double* __restrict__ F,
                                                       const double* __restrict__ L, double dt, double kT,
                                                       double gamma, uint64_t seed, uint64_t step,
                                                       double* __restrict__ X, double* __restrict__ quat,
                                                       double* __restrict__ Rnew) {
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const int lane = threadIdx.x;
  const int64_t o0 = off[b], o1 = off[b + 1];
  const double N = (double)(o1 - o0);
  // xx, xy, xz, yy, yz, zz of sum_j (r_j^2 I - r_j r_j^T)
  double k6[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t j = o0 + lane; j < o1; j += 64) {
    const double rx = rel[3 * j], ry = rel[3 * j + 1], rz = rel[3 * j + 2];
    const double r2 = rx * rx + ry * ry + rz * rz;
    k6[0] += r2 - rx * rx;
    k6[1] -= rx * ry;
    k6[2] -= rx * rz;
    k6[3] += r2 - ry * ry;
    k6[4] -= ry * rz;
    k6[5] += r2 - rz * rz;
  }
#pragma unroll
  for (int m = 0; m < 6; ++m)
    for (int o = 32; o > 0; o >>= 1) k6[m] += __shfl_xor(k6[m], o, 64);
  if (lane != 0) return;
  double K[3][3] = {{gamma * k6[0], gamma * k6[1], gamma * k6[2]},
                    {gamma * k6[1], gamma * k6[3], gamma * k6[4]},
                    {gamma * k6[2], gamma * k6[4], gamma * k6[5]}};
  // inverse by cofactors (K is SPD for a body that is not a single point or a line)
  double Ki[3][3];
  const double det = K[0][0] * (K[1][1] * K[2][2] - K[1][2] * K[2][1]) - K[0][1] * (K[1][0] * K[2][2] - K[1][2] * K[2][0]) +
                     K[0][2] * (K[1][0] * K[2][1] - K[1][1] * K[2][0]);
  const bool rot = N > 1 && det > 1e-300;
  if (rot) {
    Ki[0][0] = (K[1][1] * K[2][2] - K[1][2] * K[2][1]) / det;
    Ki[0][1] = (K[0][2] * K[2][1] - K[0][1] * K[2][2]) / det;
    Ki[0][2] = (K[0][1] * K[1][2] - K[0][2] * K[1][1]) / det;
    Ki[1][0] = (K[1][2] * K[2][0] - K[1][0] * K[2][2]) / det;
    Ki[1][1] = (K[0][0] * K[2][2] - K[0][2] * K[2][0]) / det;
    Ki[1][2] = (K[0][2] * K[1][0] - K[0][0] * K[1][2]) / det;
    Ki[2][0] = (K[1][0] * K[2][1] - K[1][1] * K[2][0]) / det;
    Ki[2][1] = (K[0][1] * K[2][0] - K[0][0] * K[2][1]) / det;
    Ki[2][2] = (K[0][0] * K[1][1] - K[0][1] * K[1][0]) / det;
  }
  // translation
  double g[3];
  normals3(seed, step, (uint32_t)b, 2u, g);
  const double st = sqrt(2.0 * kT * dt / (N * gamma));
  for (int d = 0; d < 3; ++d) X[3 * b + d] += F[3 * b + d] * dt / (N * gamma) + st * g[d];
  // rotation vector
  double th[3] = {0, 0, 0};
  if (rot) {
    // Cholesky C of Ki (symmetrized)
    const double a00 = Ki[0][0], a10 = 0.5 * (Ki[1][0] + Ki[0][1]), a11 = Ki[1][1];
    const double a20 = 0.5 * (Ki[2][0] + Ki[0][2]), a21 = 0.5 * (Ki[2][1] + Ki[1][2]), a22 = Ki[2][2];
    const double c00 = sqrt(a00);
    const double c10 = a10 / c00, c20 = a20 / c00;
    const double c11 = sqrt(fmax(a11 - c10 * c10, 0.0));
    const double c21 = c11 > 0 ? (a21 - c20 * c10) / c11 : 0.0;
    const double c22 = sqrt(fmax(a22 - c20 * c20 - c21 * c21, 0.0));
    normals3(seed, step, (uint32_t)b, 3u, g);
    const double sr = sqrt(2.0 * kT * dt);
    const double cg[3] = {c00 * g[0], c10 * g[0] + c11 * g[1], c20 * g[0] + c21 * g[1] + c22 * g[2]};
    for (int a = 0; a < 3; ++a)
      th[a] = (Ki[a][0] * L[3 * b] + Ki[a][1] * L[3 * b + 1] + Ki[a][2] * L[3 * b + 2]) * dt + sr * cg[a];
  }
  // dq = (cos(|th|/2), sin(|th|/2) th/|th|);  q <- dq * q
  const double ang = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
  double dq[4] = {1, 0, 0, 0};
  if (ang > 0) {
    const double s = sin(0.5 * ang) / ang;
    dq[0] = cos(0.5 * ang);
    dq[1] = s * th[0];
    dq[2] = s * th[1];
    dq[3] = s * th[2];
  }
  double* q = quat + 4 * b;
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  double nq[4] = {dq[0] * w - dq[1] * x - dq[2] * y - dq[3] * z, dq[0] * x + dq[1] * w + dq[2] * z - dq[3] * y,
                  dq[0] * y - dq[1] * z + dq[2] * w + dq[3] * x, dq[0] * z + dq[1] * y - dq[2] * x + dq[3] * w};
  const double nn = sqrt(nq[0] * nq[0] + nq[1] * nq[1] + nq[2] * nq[2] + nq[3] * nq[3]);
  for (int k = 0; k < 4; ++k) q[k] = nq[k] / nn;
  double R[3][3];
  quat_to_R(dq, R);
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) Rnew[9 * b + 3 * a + c] = R[a][c];
}

// beads: x = X_new + dR r  (dR rotates the old relative position to the new one)
__global__ void bd_beads_kernel(int64_t n, const int* __restrict__ body_of, const double* __restrict__ rel,
                                const double* __restrict__ X, const double* __restrict__ dR, double* __restrict__ x) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int b = body_of[j];
  const double* R = dR + 9 * b;
  const double r0 = rel[3 * j], r1 = rel[3 * j + 1], r2 = rel[3 * j + 2];
  for (int a = 0; a < 3; ++a) x[3 * j + a] = X[3 * b + a] + R[3 * a] * r0 + R[3 * a + 1] * r1 + R[3 * a + 2] * r2;
}

// ---- hard spheres (section "Brownian dynamics", the potential-free pair
// potential U(r) = gamma / (4 dt) (r - 2a)^2 for r < 2a): every two particles
// closer than 2a, ions and beads of different bodies, push each other apart
// with gamma / (2 dt) (2a - r) along the line of centres, which under the
// free-draining mobility separates an isolated pair to contact in one step.
// The pairs are found on a cell grid of edge >= 2a over all particles,
// counting-sorted and sorted by index within each cell, so every force is
// summed in a fixed order.

struct HsGeom {
  double L[3], inv_L[3];
  int nc[3];
  double cell_inv[3];
  double a2;      // (2a)^2
  double twoa;
  double coef;    // gamma / (2 dt)
};

// particle k of the combined list: beads 0..nb-1, then ions
__device__ __forceinline__ const double* hs_pos(int64_t k, int64_t nb, const double* bx, const double* ix) {
  return k < nb ? bx + 3 * k : ix + 3 * (k - nb);
}

__device__ __forceinline__ int hs_cell_index(double v, double inv_L, double cinv, int nc) {
  double w = v - floor(v * inv_L) / inv_L;  // wrapped into [0, L)
  int c = (int)(w * cinv);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void hs_count_kernel(int64_t n, int64_t nb, const double* __restrict__ bx, const double* __restrict__ ix,
                                HsGeom g, int* __restrict__ cell_of, int* __restrict__ count) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double* p = hs_pos(k, nb, bx, ix);
  const int c = (hs_cell_index(p[0], g.inv_L[0], g.cell_inv[0], g.nc[0]) * g.nc[1] +
                 hs_cell_index(p[1], g.inv_L[1], g.cell_inv[1], g.nc[1])) * g.nc[2] +
                hs_cell_index(p[2], g.inv_L[2], g.cell_inv[2], g.nc[2]);
  cell_of[k] = c;
  atomicAdd(count + c, 1);
}

__global__ void hs_start_kernel(const int64_t* __restrict__ s64, int64_t m, int* __restrict__ s32,
                                int* __restrict__ cursor, int* __restrict__ maxlen) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > m) return;
  s32[c] = (int)s64[c];
  if (c < m) {
    cursor[c] = (int)s64[c];
    atomicMax(maxlen, (int)(s64[c + 1] - s64[c]));
  }
}

__global__ void hs_scatter_kernel(int64_t n, const int* __restrict__ cell_of, int* __restrict__ cursor,
                                  int* __restrict__ entries) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  entries[atomicAdd(cursor + cell_of[k], 1)] = (int)k;
}

// f[k] = sum over partners j of coef (2a - r) (x_k - x_j) / r, 27 cells, fixed order
__global__ void hs_force_kernel(int64_t n, int64_t nb, const double* __restrict__ bx, const double* __restrict__ ix,
                                const int* __restrict__ body_of, HsGeom g, const int* __restrict__ start,
                                const int* __restrict__ entries, const int* __restrict__ cell_of,
                                double* __restrict__ f) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double* p = hs_pos(k, nb, bx, ix);
  const int own = k < nb ? body_of[k] : -1;
  const int c = cell_of[k];
  const int cz = c % g.nc[2], cy = (c / g.nc[2]) % g.nc[1], cx = c / (g.nc[1] * g.nc[2]);
  double fx = 0, fy = 0, fz = 0;
  for (int ox = -1; ox <= 1; ++ox) {
    const int x = (cx + ox + g.nc[0]) % g.nc[0];
    for (int oy = -1; oy <= 1; ++oy) {
      const int y = (cy + oy + g.nc[1]) % g.nc[1];
      for (int oz = -1; oz <= 1; ++oz) {
        const int z = (cz + oz + g.nc[2]) % g.nc[2];
        const int cc = (x * g.nc[1] + y) * g.nc[2] + z;
        for (int e = start[cc]; e < start[cc + 1]; ++e) {
          const int j = entries[e];
          if (j == k) continue;
          if (own >= 0 && j < nb && body_of[j] == own) continue;  // beads of one body
          const double* q = hs_pos(j, nb, bx, ix);
          double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
          dx -= g.L[0] * rint(dx * g.inv_L[0]);
          dy -= g.L[1] * rint(dy * g.inv_L[1]);
          dz -= g.L[2] * rint(dz * g.inv_L[2]);
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (!(r2 < g.a2) || r2 == 0.0) continue;
          const double r = sqrt(r2);
          const double s = g.coef * (g.twoa - r) / r;
          fx += s * dx;
          fy += s * dy;
          fz += s * dz;
        }
      }
    }
  }
  f[3 * k] = fx;
  f[3 * k + 1] = fy;
  f[3 * k + 2] = fz;
}

// per body: F += sum_j f_j, L += sum_j r_j x f_j (one block per body, fixed order)
__global__ void __launch_bounds__(256) hs_body_kernel(const int64_t* __restrict__ off, const double* __restrict__ rel,
                                                      const double* __restrict__ f, const double* __restrict__ F0,
                                                      const double* __restrict__ L0, double* __restrict__ Fo,
                                                      double* __restrict__ Lo) {
  const int64_t b = blockIdx.x;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = off[b] + threadIdx.x; i < off[b + 1]; i += blockDim.x) {
    const double rx = rel[3 * i], ry = rel[3 * i + 1], rz = rel[3 * i + 2];
    const double fx = f[3 * i], fy = f[3 * i + 1], fz = f[3 * i + 2];
    v[0] += fx; v[1] += fy; v[2] += fz;
    v[3] += ry * fz - rz * fy; v[4] += rz * fx - rx * fz; v[5] += rx * fy - ry * fx;
  }
  __shared__ double sh[6][4];
  for (int m = 0; m < 6; ++m)
    for (int o = 32; o > 0; o >>= 1) v[m] += __shfl_xor(v[m], o, 64);
  if ((threadIdx.x & 63) == 0)
    for (int m = 0; m < 6; ++m) sh[m][threadIdx.x >> 6] = v[m];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int m = 0; m < 6; ++m) {
      double t = 0;
      for (int w = 0; w < 4; ++w) t += sh[m][w];
      // F and L of the electrostatic pass plus the hard-sphere parts
      if (m < 3) Fo[3 * b + m] = F0[3 * b + m] + t;
      else Lo[3 * b + m - 3] = L0[3 * b + m - 3] + t;
    }
  }
}

__global__ void hs_ion_kernel(int64_t ni, const double* __restrict__ f0, const double* __restrict__ fh,
                              double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * ni) out[i] = f0[i] + fh[i];
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Hard-sphere forces of every particle of the loaded configuration (beads,
// then ions; 3 doubles each) in the workspace, followed by room for the
// summed ion forces (3 per ion) and body forces and torques (3 + 3 per body).
double* hard_sphere_forces(pe_context* c, double gamma, double dt) {
  hipStream_t s = c->stream;
  const int64_t nb = c->n_bead, ni = c->n_ion, n = nb + ni, nbody = c->n_body;
  const double a = c->p.hs_radius;
  HsGeom g{};
  int64_t ncell = 1;
  for (int d = 0; d < 3; ++d) {
    g.L[d] = c->p.box[d];
    g.inv_L[d] = 1.0 / c->p.box[d];
    g.nc[d] = (int)std::min(1024.0, std::floor(c->p.box[d] / (2.0 * a)));
    require(g.nc[d] >= 3, "hard-sphere diameter above a third of the box");
  }
  // at most 2^26 cells: coarser cells (edges still >= 2a) beyond that
  while ((int64_t)g.nc[0] * g.nc[1] * g.nc[2] > ((int64_t)1 << 26)) {
    const int d = g.nc[0] >= g.nc[1] ? (g.nc[0] >= g.nc[2] ? 0 : 2) : (g.nc[1] >= g.nc[2] ? 1 : 2);
    g.nc[d] = std::max(3, g.nc[d] / 2);
  }
  for (int d = 0; d < 3; ++d) {
    g.cell_inv[d] = g.nc[d] / c->p.box[d];
    ncell *= g.nc[d];
  }
  g.twoa = 2.0 * a;
  g.a2 = 4.0 * a * a;
  g.coef = gamma / (2.0 * dt);
  c->hs_f.ensure(3 * (size_t)n + 3 * (size_t)ni + 6 * (size_t)nbody + 1);
  c->hs_cell.ensure((size_t)n);
  c->hs_entries.ensure((size_t)n);
  c->hs_count.ensure((size_t)ncell + 1);
  c->hs_start.ensure((size_t)ncell + 1);
  c->hs_start64.ensure((size_t)ncell + 1);
  c->hs_scan.ensure((size_t)scan_workspace(ncell));
  int* count = c->hs_count.get();
  PE_HIP(hipMemsetAsync(count, 0, sizeof(int) * (ncell + 1), s));
  hipLaunchKernelGGL(hs_count_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, n, nb, c->bead_x.get(), c->ion_x.get(), g,
                     c->hs_cell.get(), count);
  PE_CHECK_LAUNCH();
  launch_exclusive_scan(s, count, ncell, c->hs_start64.get(), c->hs_scan.get());
  // counts become cursors; count[ncell] holds the longest cell
  PE_HIP(hipMemsetAsync(count + ncell, 0, sizeof(int), s));
  hipLaunchKernelGGL(hs_start_kernel, dim3(nblk(ncell + 1, 256)), dim3(256), 0, s, c->hs_start64.get(), ncell,
                     c->hs_start.get(), count, count + ncell);
  hipLaunchKernelGGL(hs_scatter_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, n, c->hs_cell.get(), count,
                     c->hs_entries.get());
  PE_CHECK_LAUNCH();
  int maxlen = 0;
  PE_HIP(hipMemcpyAsync(&maxlen, count + ncell, sizeof(int), hipMemcpyDeviceToHost, s));
  PE_HIP(hipStreamSynchronize(s));
  launch_segment_sort(s, c->hs_start.get(), (int)ncell, c->hs_entries.get(), maxlen);
  hipLaunchKernelGGL(hs_force_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, n, nb, c->bead_x.get(), c->ion_x.get(),
                     c->body_of.get(), g, c->hs_start.get(), c->hs_entries.get(), c->hs_cell.get(), c->hs_f.get());
  PE_CHECK_LAUNCH();
  return c->hs_f.get();
}

// The step's kernels; R: 9 doubles per body of scratch (the rotation of each
// body, written by the body kernel and read by the bead kernel).
void bd_launch(pe_context* c, double dt, double kT, double gamma, uint64_t seed, uint64_t step, double* bead_pos,
               double* body_center, double* body_quat, double* ion_pos, double* R) {
  if (!c->have_forces) throw Error(PE_ERR_STATE, "pe_forces_torques has not been called");
  require(dt > 0 && kT >= 0 && gamma > 0, "dt, gamma must be positive and kT non-negative");
  require((c->n_bead == 0 || bead_pos) && (c->n_body == 0 || (body_center && body_quat)) &&
              (c->n_ion == 0 || ion_pos),
          "null state array");
  hipStream_t s = c->stream;
  const int64_t nb = c->n_bead, nbody = c->n_body, ni = c->n_ion;
  const double* fion = c->forces.get() + 3 * nb;
  const double* Fb = c->bodyF.get();
  const double* Lb = c->bodyL.get();
  if (c->p.hs_radius > 0 && nb + ni > 1) {
    // hard-sphere forces of the current configuration added to the electrostatic ones
    double* hs = hard_sphere_forces(c, gamma, dt);
    double* ftot = hs + 3 * (nb + ni);   // ions: electrostatic + hard sphere
    double* Ft = ftot + 3 * ni;          // bodies
    double* Lt = Ft + 3 * nbody;
    if (ni) {
      hipLaunchKernelGGL(hs_ion_kernel, dim3(nblk(3 * ni, 256)), dim3(256), 0, s, ni, fion, hs + 3 * nb, ftot);
      fion = ftot;
    }
    if (nbody) {
      hipLaunchKernelGGL(hs_body_kernel, dim3((unsigned)nbody), dim3(256), 0, s, c->off.get(), c->rel.get(), hs, Fb,
                         Lb, Ft, Lt);
      Fb = Ft;
      Lb = Lt;
    }
    PE_CHECK_LAUNCH();
  }
  if (ni)
    hipLaunchKernelGGL(bd_ions_kernel, dim3(nblk(ni, 256)), dim3(256), 0, s, ni, fion, dt, kT, gamma, seed, step,
                       ion_pos);
  if (nbody) {
    hipLaunchKernelGGL(bd_bodies_kernel, dim3((unsigned)nbody), dim3(64), 0, s, nbody, c->off.get(), c->rel.get(),
                       Fb, Lb, dt, kT, gamma, seed, step, body_center, body_quat, R);
    hipLaunchKernelGGL(bd_beads_kernel, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, c->body_of.get(), c->rel.get(),
                       body_center, R, bead_pos);
  }
  PE_CHECK_LAUNCH();
  PE_HIP(hipStreamSynchronize(s));
  c->have_system = false;  // positions moved: pe_set_system must run again
  c->have_solution = false;
  c->have_forces = false;
}

// Scratch of the allocation-free step: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code uses only the device
// address looked up for each GPU (the array's name is a host-side stand-in).
constexpr int64_t kMaxStaticBodies = 65536;   // 4.5 MiB of rotations

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // per device; null until looked up

}  // namespace

static __device__ __align__(256) double scratch[9 * kMaxStaticBodies];

// Looks up (once per device, with that device current) the address of that
// device's copy of the scratch array.
double* bd_static_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev >= (int)g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    PE_HIP(hipGetDevice(&cur));
    if (cur != dev) PE_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) PE_HIP(hipSetDevice(cur));
    if (e != hipSuccess)
      throw Error(PE_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace pe

using namespace pe;

extern "C" pe_status pe_bd_step_noalloc(pe_context* c, double dt, double kT, double gamma, uint64_t seed,
                                        uint64_t step, double* bead_pos, double* body_center, double* body_quat,
                                        double* ion_pos) {
  if (!c) return PE_ERR_ARG;
  try {
    require(!(c->p.hs_radius > 0), "pe_bd_step_noalloc: hard spheres need workspace buffers (hs_radius must be 0)");
    if (c->n_body > kMaxStaticBodies)
      throw Error(PE_ERR_ARG, "pe_bd_step_noalloc: more than " + std::to_string(kMaxStaticBodies) +
                                  " bodies (the static scratch holds that many)");
    double* R = bd_static_scratch(c->device);
    bd_launch(c, dt, kT, gamma, seed, step, bead_pos, body_center, body_quat, ion_pos, R);
  } catch (const Error& e) {
    c->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    return PE_ERR_DEVICE;
  }
  return PE_OK;
}

extern "C" pe_status pe_bd_step(pe_context* c, double dt, double kT, double gamma, uint64_t seed, uint64_t step,
                                double* bead_pos, double* body_center, double* body_quat, double* ion_pos) {
  if (!c) return PE_ERR_ARG;
  ArenaScope arena_scope(&c->arena);
  try {
    c->bd_R.ensure(9 * std::max<int64_t>(c->n_body, 1));
    bd_launch(c, dt, kT, gamma, seed, step, bead_pos, body_center, body_quat, ion_pos, c->bd_R.get());
  } catch (const Error& e) {
    c->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    return PE_ERR_DEVICE;
  }
  return PE_OK;
}
