// C ABI entry points, configuration setup, the saddle-point operator, the
// GMRES driver (plain double and mixed-precision refinement), the
// right-hand side and the force pass.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "pe_internal.hpp"
#include "vector.hpp"
#include "guess.hpp"
#include "precond.hpp"

namespace pe {

thread_local Arena* tl_arena = nullptr;

void* Arena::alloc(size_t bytes, void** owner) {
  const size_t len = (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < len) continue;
    const size_t off = it->first, rest = it->second - len;
    free_.erase(it);
    if (rest) free_[off + len] = rest;
    live_[off] = Blk{len, owner};
    in_use += len;
    peak = std::max(peak, in_use);
    return base + off;
  }
  // does not fit: the region would need at least the live bytes plus this
  // request, and more than it has now
  need = std::max(need, std::max(in_use + len, size + len));
  throw Error(PE_ERR_NOMEM, "workspace too small: " + std::to_string(len) + " more bytes requested with " +
                                std::to_string(in_use) + " of " + std::to_string(size) +
                                " in use; register a region of at least pe_workspace_size() bytes "
                                "with pe_set_workspace and call again");
}

void Arena::release(void* p) {
  if (!p) return;
  const size_t off = static_cast<char*>(p) - base;
  auto it = live_.find(off);
  if (it == live_.end()) return;
  size_t o = off, len = it->second.len;
  in_use -= len;
  live_.erase(it);
  auto nx = free_.lower_bound(o);
  if (nx != free_.end() && nx->first == o + len) {
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {
    auto pv = std::prev(nx);
    if (pv->first + pv->second == o) {
      o = pv->first;
      len += pv->second;
      free_.erase(pv);
    }
  }
  free_[o] = len;
}

void Arena::reown(void* p, void** owner) {
  auto it = live_.find(static_cast<char*>(p) - base);
  if (it != live_.end()) it->second.owner = owner;
}

void Arena::migrate(char* nb, size_t nsize, hipStream_t s) {
  size_t total = 0, end = 0;
  for (auto& kv : live_) {
    total += kv.second.len;
    end = kv.first + kv.second.len;
  }
  if (nb == base) {
    // the same region, resized: blocks stay where they are
    if (end > nsize) {
      need = std::max(need, end);
      throw Error(PE_ERR_NOMEM, "the resized workspace cuts through live blocks");
    }
    if (nsize > size) free_[size] = nsize - size;  // merged by later releases
    else if (nsize < size) {
      auto it = free_.rbegin();
      require(it != free_.rend() && it->first + it->second == size, "cannot shrink the workspace");
      const size_t o = it->first;
      free_.erase(o);
      if (nsize > o) free_[o] = nsize - o;
    }
    size = nsize;
    need = 0;
    return;
  }
  require(nb + nsize <= base || base + size <= nb, "the new workspace overlaps the old one");
  if (total > nsize) {
    need = std::max(need, total);
    throw Error(PE_ERR_NOMEM, "the new workspace cannot hold the " + std::to_string(total) + " live bytes");
  }
  // live blocks packed from the start of the new region, in address order
  std::map<size_t, Blk> nl;
  size_t o = 0;
  for (auto& kv : live_) {
    if (nb + o != base + kv.first)
      PE_HIP(hipMemcpyAsync(nb + o, base + kv.first, kv.second.len, hipMemcpyDeviceToDevice, s));
    nl[o] = kv.second;
    o += kv.second.len;
  }
  PE_HIP(hipStreamSynchronize(s));
  for (auto& kv : nl) *kv.second.owner = nb + kv.first;
  live_.swap(nl);
  free_.clear();
  if (nsize > o) free_[o] = nsize - o;
  base = nb;
  size = nsize;
  need = 0;
}

}  // namespace pe

using namespace pe;

namespace {

thread_local std::string g_create_error;

using Clock = std::chrono::steady_clock;
inline double secs(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}
inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------------------------ kernels

__global__ void rel_kernel(const double* __restrict__ x, const double* __restrict__ X,
                           const int* __restrict__ body_of, int64_t n, double* __restrict__ rel) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = body_of[i];
  rel[3 * i] = x[3 * i] - X[3 * b];
  rel[3 * i + 1] = x[3 * i + 1] - X[3 * b + 1];
  rel[3 * i + 2] = x[3 * i + 2] - X[3 * b + 2];
}

// b_top[i] = -r_i.E0 + phi_ion[i] - (ck[0] - ck[1] sigma_i^2)
__global__ void rhs_top_kernel(int64_t n, const double* __restrict__ rel, double ex, double ey, double ez,
                               const double* __restrict__ phi_ion, const double* __restrict__ sig,
                               const double* __restrict__ ck, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = -(rel[3 * i] * ex + rel[3 * i + 1] * ey + rel[3 * i + 2] * ez);
  if (phi_ion) v += phi_ion[i] - (ck[0] - ck[1] * sig[i] * sig[i]);
  b[i] = v;
}

// Potential offsets of a starting point whose offsets are zero: with
// r = b - A [q; 0], the offset of body i that minimizes the residual of its
// bead rows is the mean of r over them (each row holds +dPsi_i once).
// Writes dPsi_i = sum_i / N_i into x and removes it from r.
__global__ void start_offsets_kernel(int64_t nb, int64_t n_body, const int64_t* __restrict__ off,
                                     const int* __restrict__ body_of, const double* __restrict__ rsum,
                                     double* __restrict__ r, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) {
    const int b = body_of[i];
    r[i] -= rsum[b] / (double)(off[b + 1] - off[b]);
  }
  if (i < n_body) x[nb + i] = rsum[i] / (double)(off[i + 1] - off[i]);
}

// phi[i] -= ck_total(sigma_i); then f = q (E0 + E), u = q phi / 2 - q x.E0
__global__ void finish_particles_kernel(int64_t n, const double* __restrict__ chg, const double* __restrict__ pos,
                                        const double* __restrict__ sig, double ex, double ey, double ez,
                                        const double* __restrict__ ckA, const double* __restrict__ ckB,
                                        double* __restrict__ phi, const double* __restrict__ E,
                                        double* __restrict__ f, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s2 = sig[i] * sig[i];
  double c0 = 0, c1 = 0;
  if (ckA) { c0 += ckA[0]; c1 += ckA[1]; }
  if (ckB) { c0 += ckB[0]; c1 += ckB[1]; }
  const double ph = phi[i] - (c0 - c1 * s2);
  phi[i] = ph;
  if (f) {
    const double q = chg[i];
    f[3 * i] = q * (ex + E[3 * i]);
    f[3 * i + 1] = q * (ey + E[3 * i + 1]);
    f[3 * i + 2] = q * (ez + E[3 * i + 2]);
    u[i] = 0.5 * q * ph - q * (pos[3 * i] * ex + pos[3 * i + 1] * ey + pos[3 * i + 2] * ez);
  }
}

// stats[0] += non-finite count, stats[1] = max, stats[2] = min (per block partials)
__global__ void stats_kernel(const double* __restrict__ a, int64_t n, int stride, int col, double* __restrict__ part) {
  double bad = 0, mx = -INFINITY, mn = INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = a[i * stride + col];
    if (!isfinite(v)) bad += 1;
    else {
      mx = fmax(mx, v);
      mn = fmin(mn, v);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    bad += __shfl_xor(bad, o, 64);
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    mn = fmin(mn, __shfl_xor(mn, o, 64));
  }
  __shared__ double sh[3][4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sh[0][w] = bad; sh[1][w] = mx; sh[2][w] = mn; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b2 = 0, m2 = -INFINITY, n2 = INFINITY;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      b2 += sh[0][k]; m2 = fmax(m2, sh[1][k]); n2 = fmin(n2, sh[2][k]);
    }
    part[3 * blockIdx.x] = b2;
    part[3 * blockIdx.x + 1] = m2;
    part[3 * blockIdx.x + 2] = n2;
  }
}

__global__ void to_float_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void copy_kernel(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// Sum of a[0..n) in a fixed order: sum_partial_kernel leaves one partial
// per block of `chunk` values, sum_kernel (one block) adds the partials.
__global__ void sum_partial_kernel(const double* __restrict__ a, int64_t n, int64_t chunk,
                                   double* __restrict__ part) {
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = min(n, b0 + chunk);
  double s = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) s += a[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ double sh[16];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    part[blockIdx.x] = t;
  }
}

__global__ void sum_kernel(const double* __restrict__ a, int64_t n, double* __restrict__ out) {
  // single block, fixed order
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += a[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ double sh[16];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    *out = t;
  }
}

// --------------------------------------------------------------- helpers

struct Stats {
  double bad, mx, mn;
};

// Several arrays at once: every stats launch writes its own slice of the
// reduction buffer, then one copy and one synchronization.
struct StatReq {
  const double* a;
  int64_t n;
  int stride, col;
};

std::vector<Stats> array_stats(pe_context* c, const std::vector<StatReq>& reqs) {
  std::vector<Stats> out(reqs.size(), Stats{0, -INFINITY, INFINITY});
  std::vector<unsigned> nbs(reqs.size(), 0);
  size_t slot = 0;
  for (size_t r = 0; r < reqs.size(); ++r) {
    const StatReq& q = reqs[r];
    if (q.n == 0 || !q.a) continue;
    unsigned nb = nblk(q.n, 256);
    if (nb > 256) nb = 256;
    nbs[r] = nb;
    hipLaunchKernelGGL(stats_kernel, dim3(nb), dim3(256), 0, c->stream, q.a, q.n, q.stride, q.col,
                       c->red.get() + 3 * slot);
    PE_CHECK_LAUNCH();
    slot += nb;
  }
  if (slot == 0) return out;
  require(3 * slot <= c->red.cap, "reduction buffer too small for the input checks");
  double* h = c->h_stats.get<double>(3 * slot);
  PE_HIP(hipMemcpyAsync(h, c->red.get(), sizeof(double) * 3 * slot, hipMemcpyDeviceToHost, c->stream));
  PE_HIP(hipStreamSynchronize(c->stream));
  size_t o = 0;
  for (size_t r = 0; r < reqs.size(); ++r) {
    for (unsigned b = 0; b < nbs[r]; ++b, ++o) {
      out[r].bad += h[3 * o];
      out[r].mx = std::max(out[r].mx, h[3 * o + 1]);
      out[r].mn = std::min(out[r].mn, h[3 * o + 2]);
    }
  }
  return out;
}

void dcopy(hipStream_t s, const double* a, double* b, int64_t n) {
  if (n == 0) return;
  PE_HIP(hipMemcpyAsync(b, a, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
}

CkCoef ck_coef(const pe_context* c) {
  CkCoef cc;
  cc.reg = c->p.reg;
  cc.inv_epsV = 1.0 / (c->p.eps * c->V);
  cc.inv4xi2 = 1.0 / (4.0 * c->xi * c->xi);
  cc.a = c->p.shell_radius;
  return cc;
}

// Scratch layout in c->sums: [ck_bead(2), ck_ion(2), tot(2), tmp(...)]
double* ck_bead(pe_context* c) { return c->sums.get(); }
double* ck_ion(pe_context* c) { return c->sums.get() + 2; }
double* tot2(pe_context* c) { return c->sums.get() + 4; }
double* scal(pe_context* c) { return c->sums.get() + 8; }   // misc device scalars (32)

template <typename T>
T* grid_real(pe::DevBuf<double>& g) { return reinterpret_cast<T*>(g.get()); }

// Device counter of pair evaluations for the profiler (null when not profiling).
template <typename T>
unsigned long long* pair_counter(pe_context* c) {
  return c->prof.on ? c->pair_count.get() + (sizeof(T) == 8 ? 1 : 0) : nullptr;
}

// M q for the beads with bead charges q (caller order), assembled into the
// saddle operator: y[0:nb] = -(M q) + Sigma^T dpsi, y[nb:] = Sigma q.
// Work enqueued on c->aux after fork() starts after everything enqueued on
// c->stream so far; work on c->stream after join() starts after everything
// enqueued on c->aux so far.
void fork_aux(pe_context* c) {
  PE_HIP(hipEventRecord(c->ev_fork, c->stream));
  PE_HIP(hipStreamWaitEvent(c->aux, c->ev_fork, 0));
}
void join_aux(pe_context* c) {
  PE_HIP(hipEventRecord(c->ev_join, c->aux));
  PE_HIP(hipStreamWaitEvent(c->stream, c->ev_join, 0));
}

template <typename T>
void apply_saddle(pe_context* c, const double* x, double* y) {
  hipStream_t s = c->stream;
  const int64_t nb = c->n_bead;
  ProfScope ps_all(c->prof, s, PE_PROF_MATVEC, sizeof(T) == 8, (double)nb);
  const double* q = x;
  const double* dpsi = x + nb;
  T* gA = grid_real<T>(c->gridA);
  T* gB = grid_real<T>(c->gridB);
  const bool dbl = sizeof(T) == 8;
  // the real-space part on the auxiliary stream, into its own buffer, while
  // the mesh part (spread, FFT, contraction) runs on the caller's: the dense
  // intra-body blocks per shape, then the sparse inter-body pairs added;
  // also the charge moments (the k = 0 term) and the body net charges; the
  // assembly after the join.  The spread is enqueued first, then the
  // auxiliary work (enqueued while the spread runs, and run beside the
  // spread, which is instruction-bound, rather than beside the FFT passes,
  // which are bandwidth-bound), then the rest of the mesh part.
  c->phi_near.ensure((size_t)std::max<int64_t>(nb, 1));
  double* phi_real = c->phi_near.get();
  fork_aux(c);
  { ProfScope ps(c->prof, s, PE_PROF_SPREAD, dbl, (double)nb); launch_spread<T>(s, c->B, q, gA, c->gg, false); }
  {
    hipStream_t sa = c->aux;
    launch_moments(sa, q, c->bead_sig.get(), 0.0, nb, ck_coef(c), c->red.get(), ck_bead(c), nullptr);
    launch_seg_sum(sa, c->off.get(), c->n_body, q, y + nb);
    // every bead segment belongs to one body: when all bodies have a dense
    // block, the block products write every entry and nothing is cleared
    const bool all_near = c->pc.near_beads == nb;
    if (!all_near) PE_HIP(hipMemsetAsync(phi_real, 0, sizeof(double) * nb, sa));
    for (auto& t : c->pc.types) {
      if (!t.near || t.bodies.empty()) continue;
      const T* R;
      if constexpr (sizeof(T) == 8) R = t.R64.get();
      else R = t.R32.get();
      ProfScope ps(c->prof, sa, PE_PROF_NEAR, dbl, (double)t.N * t.N * (double)t.bodies.size());
      launch_body_gemm<T>(sa, R, t.N, false, !all_near, t.dbodies.get(), (int)t.bodies.size(), c->off.get(), nb,
                          q, phi_real, c->pc.gemm_ws.get());
    }
    ProfScope ps(c->prof, sa, PE_PROF_SPMV, dbl, (double)c->nnz);
    launch_spmv_add<T>(sa, c, q, phi_real);
  }
  launch_wave_pipeline<T>(s, c, gA, gB, c->gridC.get());
  { ProfScope ps(c->prof, s, PE_PROF_GATHER, dbl, (double)nb); launch_gather<T>(s, c->B, gB, c->gg, c->phi_w.get(), nullptr, false); }
  join_aux(c);
  launch_assemble(s, c, dpsi, c->phi_w.get(), phi_real, ck_bead(c), y);
}

void apply_saddle_prec(pe_context* c, int prec, const double* x, double* y) {
  if (prec == PE_MIXED) apply_saddle<float>(c, x, y);
  else apply_saddle<double>(c, x, y);
}

// Potential (and field) of all particles for bead charges qb and ion charges qi.
// phi (n_all), E (3 n_all or null).  Includes the self terms and removes
// the k = 0 constant; optionally forms forces/energies.
//
// reuse_ion (single precision, ion charges those of the system): the ion
// grid and the ion -> bead real-space sums kept by the right-hand side of
// this configuration stand in for spreading the ions again and for the
// ion sources of the bead targets' pair pass (the potential is linear in
// the charges, and the kept parts were formed by the same kernels).
template <typename T>
void all_potential(pe_context* c, const double* qb, const double* qi, double* phi, double* E,
                   double* f, double* u, const double* chg_all, bool reuse_ion = false) {
  hipStream_t s = c->stream;
  const int64_t nb = c->n_bead, ni = c->n_ion, na = nb + ni;
  reuse_ion = reuse_ion && sizeof(T) == 4 && ni > 0 && c->ion_parts_valid && E != nullptr;
  PE_HIP(hipMemsetAsync(phi, 0, sizeof(double) * na, s));
  if (E) PE_HIP(hipMemsetAsync(E, 0, sizeof(double) * 3 * na, s));
  launch_moments(s, qb, c->bead_sig.get(), 0.0, nb, ck_coef(c), c->red.get(), ck_bead(c), nullptr);
  if (ni) launch_moments(s, qi, c->ion_sig.get(), 0.0, ni, ck_coef(c), c->red.get(), ck_ion(c), nullptr);
  T* gA = grid_real<T>(c->gridA);
  T* gB = grid_real<T>(c->gridB);
  if (reuse_ion) gA = reinterpret_cast<T*>(c->ion_grid32.get());
  // real space on the auxiliary stream, into its own buffers
  c->phi_pair.ensure((size_t)std::max<int64_t>(na, 1));
  if (E) c->E_pair.ensure(3 * (size_t)std::max<int64_t>(na, 1));
  double* phi_p = c->phi_pair.get();
  double* E_p = E ? c->E_pair.get() : nullptr;
  fork_aux(c);
  {
    hipStream_t sa = c->aux;
    PE_HIP(hipMemsetAsync(phi_p, 0, sizeof(double) * na, sa));
    if (E) PE_HIP(hipMemsetAsync(E_p, 0, sizeof(double) * 3 * na, sa));
    ProfScope ps_pair(c->prof, sa, PE_PROF_PAIR, sizeof(T) == 8);
    unsigned long long* npc = pair_counter<T>(c);
    const PairTables& pt = c->pair_tabs;
    if (reuse_ion) {
      launch_pair_onfly<T>(sa, c->B, &c->B, qb, nullptr, nullptr, c->rg, phi_p, E_p, false, npc,
                           pt.get(false, false));
      launch_axpby(sa, 1.0, c->ion_rs_phi.get(), 1.0, phi_p, nb);
      launch_axpby(sa, 1.0, c->ion_rs_E.get(), 1.0, E_p, 3 * nb);
    } else {
      launch_pair_onfly<T>(sa, c->B, &c->B, qb, &c->I, qi, c->rg, phi_p, E_p, false, npc, pt.get(false, false),
                           pt.get(false, true));
    }
    launch_pair_onfly<T>(sa, c->I, &c->B, qb, &c->I, qi, c->rg, phi_p + nb, E_p ? E_p + 3 * nb : nullptr, false,
                         npc, pt.get(true, false), pt.get(true, true));
  }
  {
    ProfScope ps(c->prof, s, PE_PROF_SPREAD, sizeof(T) == 8, (double)(reuse_ion ? nb : nb + ni));
    if (reuse_ion) {
      launch_spread<T>(s, c->B, qb, gA, c->gg, true);  // onto the kept ion grid
      c->ion_parts_valid = false;
    } else {
      launch_spread<T>(s, c->B, qb, gA, c->gg, false);
      if (ni) launch_spread<T>(s, c->I, qi, gA, c->gg, true);
    }
  }
  launch_wave_pipeline<T>(s, c, gA, gB, c->gridC.get());
  {
    ProfScope ps(c->prof, s, PE_PROF_GATHER, sizeof(T) == 8, (double)(nb + ni));
    launch_gather<T>(s, c->B, gB, c->gg, phi, E, true);
    if (ni) launch_gather<T>(s, c->I, gB, c->gg, phi + nb, E ? E + 3 * nb : nullptr, true);
  }
  join_aux(c);
  launch_axpby(s, 1.0, phi_p, 1.0, phi, na);
  if (E) launch_axpby(s, 1.0, E_p, 1.0, E, 3 * na);
  // k = 0 constant, then forces and energies
  if (nb)
    hipLaunchKernelGGL(finish_particles_kernel, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, chg_all,
                       c->bead_x.get(), c->bead_sig.get(), c->E0[0], c->E0[1], c->E0[2], ck_bead(c),
                       ni ? ck_ion(c) : (const double*)nullptr, phi, E, f, u);
  if (ni)
    hipLaunchKernelGGL(finish_particles_kernel, dim3(nblk(ni, 256)), dim3(256), 0, s, ni,
                       chg_all ? chg_all + nb : nullptr, c->ion_x.get(), c->ion_sig.get(), c->E0[0],
                       c->E0[1], c->E0[2], ck_bead(c), ck_ion(c), phi + nb, E ? E + 3 * nb : nullptr,
                       f ? f + 3 * nb : nullptr, u ? u + nb : nullptr);
  PE_CHECK_LAUNCH();
}

// Right-hand side b = [-r.E0 + phi_ion(beads); Q] in double.
// Ion potential (and, with the learned guess active, ion field) at the beads,
// in precision T: the wave part by one ion-only SE pass, plus the ion->bead
// real-space pairs.  Mixed precision runs it in float like every other
// real- and wave-space sum; the double path keeps it in double.
//
// In single precision with the field requested, the spread ion grid and the
// real-space ion -> bead sums are kept for the force pass of the same
// configuration (see all_potential).
//
// keep32 (mixed precision, field requested): the parts are kept for the
// single-precision force pass; a double pass keeps a float copy of its ion
// grid.
template <typename T>
void ion_potential_at_beads(pe_context* c, double* phi_ion, double* E, bool keep32) {
  hipStream_t s = c->stream;
  const bool dbl = sizeof(T) == 8;
  const int64_t nb = c->n_bead;
  const bool keep = keep32 && E != nullptr;
  T* gA = grid_real<T>(c->gridA);
  T* gB = grid_real<T>(c->gridB);
  const int64_t G = (int64_t)c->gg.N[0] * c->gg.N[1] * c->gg.N[2];
  if (keep) {
    c->ion_grid32.ensure((size_t)G);
    if constexpr (sizeof(T) == 4) gA = reinterpret_cast<T*>(c->ion_grid32.get());
  }
  // ion -> bead real space on the auxiliary stream, into its own buffers
  // (kept for the force pass in single precision with the field)
  double* rs_phi;
  double* rs_E = nullptr;
  if (keep) {
    c->ion_rs_phi.ensure((size_t)std::max<int64_t>(nb, 1));
    c->ion_rs_E.ensure(3 * (size_t)std::max<int64_t>(nb, 1));
    rs_phi = c->ion_rs_phi.get();
    rs_E = c->ion_rs_E.get();
  } else {
    c->phi_pair.ensure((size_t)std::max<int64_t>(nb, 1));
    rs_phi = c->phi_pair.get();
    if (E) {
      c->E_pair.ensure(3 * (size_t)std::max<int64_t>(nb, 1));
      rs_E = c->E_pair.get();
    }
  }
  fork_aux(c);
  {
    hipStream_t sa = c->aux;
    PE_HIP(hipMemsetAsync(rs_phi, 0, sizeof(double) * nb, sa));
    if (rs_E) PE_HIP(hipMemsetAsync(rs_E, 0, sizeof(double) * 3 * nb, sa));
    // double path: the field only feeds the guess features, single precision
    ProfScope ps(c->prof, sa, PE_PROF_PAIR, dbl);
    launch_pair_onfly<T>(sa, c->B, &c->I, c->ion_q.get(), nullptr, nullptr, c->rg, rs_phi, rs_E, true,
                         pair_counter<T>(c), c->pair_tabs.get(false, true));
  }
  {
    ProfScope ps(c->prof, s, PE_PROF_SPREAD, dbl, (double)c->n_ion);
    launch_spread<T>(s, c->I, c->ion_q.get(), gA, c->gg, false);
  }
  if (keep && dbl) {
    hipLaunchKernelGGL(to_float_kernel, dim3(nblk(G, 256)), dim3(256), 0, s,
                       reinterpret_cast<const double*>(gA), c->ion_grid32.get(), G);
    PE_CHECK_LAUNCH();
  }
  launch_wave_pipeline<T>(s, c, gA, gB, c->gridC.get());
  {
    ProfScope ps(c->prof, s, PE_PROF_GATHER, dbl, (double)nb);
    launch_gather<T>(s, c->B, gB, c->gg, phi_ion, E, false);
  }
  join_aux(c);
  launch_axpby(s, 1.0, rs_phi, 1.0, phi_ion, nb);
  if (E) launch_axpby(s, 1.0, rs_E, 1.0, E, 3 * nb);
  if (keep) c->ion_parts_valid = true;
}

// Right-hand side b = [-r.E0 + phi_ion(beads); Q].  The ion potential is
// formed in double unless the parameters ask for the float kernels in mixed
// precision (rhs_fp64 = 0): the double residuals of the refinement are then
// residuals of the same system the double path solves.
void build_rhs(pe_context* c, double* b) {
  hipStream_t s = c->stream;
  const int64_t nb = c->n_bead, ni = c->n_ion;
  double* phi_ion = nullptr;
  if (ni) {
    phi_ion = c->phi_w.get();
    launch_moments(s, c->ion_q.get(), c->ion_sig.get(), 0.0, ni, ck_coef(c), c->red.get(), ck_ion(c), nullptr);
    // with the learned guess active, the same pass also yields the ion field at the beads
    // (in single precision the field is formed anyway, for the force pass)
    double* E = nullptr;
    if (c->guess || c->p.precision == PE_MIXED) {
      c->E_ion.ensure(3 * std::max<int64_t>(nb, 1));
      E = c->E_ion.get();
    }
    const bool mixed = c->p.precision == PE_MIXED;
    if (mixed && !c->p.rhs_fp64) ion_potential_at_beads<float>(c, phi_ion, E, true);
    else ion_potential_at_beads<double>(c, phi_ion, E, mixed);
  }
  c->have_eion = c->guess != nullptr;
  if (nb)
    hipLaunchKernelGGL(rhs_top_kernel, dim3(nblk(nb, 256)), dim3(256), 0, s, nb, c->rel.get(), c->E0[0],
                       c->E0[1], c->E0[2], phi_ion, c->bead_sig.get(), ck_ion(c), b);
  PE_CHECK_LAUNCH();
  dcopy(s, c->body_Q.get(), b + nb, c->n_body);
}

// --------------------------------------------------------------- GMRES

struct KWork {
  double* V;      // (m+1) x n
  double* Z;      // m x n preconditioned directions (flexible GMRES)
  double* w;      // n
  double* r;      // n
  double* tmp;    // n
  double* st;     // Hessenberg etc.
  double* h1;     // m+1
  double* h2;     // m+1
  double* nrm;    // 1
  double* res;    // 1
  double* y;      // m
};

KWork kwork(pe_context* c, int64_t n, int m) {
  KWork k;
  c->Vb.ensure((size_t)(m + 1) * n);
  c->Zb.ensure((size_t)m * n);
  c->kvec.ensure((size_t)3 * n);
  const size_t nst = (size_t)(m + 1) * m + 2 * m + (m + 1);
  c->hs.ensure(nst + 3 * (m + 1) + 4 + m);
  k.V = c->Vb.get();
  k.Z = c->Zb.get();
  k.w = c->kvec.get();
  k.r = k.w + n;
  k.tmp = k.r + n;
  k.st = c->hs.get();
  k.h1 = k.st + nst;
  k.h2 = k.h1 + (m + 1);
  k.nrm = k.h2 + (m + 1);
  k.res = k.nrm + 1;
  k.y = k.res + 2;
  return k;
}

double fetch(pe_context* c, const double* d) {
  PE_HIP(hipMemcpyAsync(c->pinned, d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  PE_HIP(hipStreamSynchronize(c->stream));
  c->prof.flush();
  return c->pinned[0];
}

struct GmresOut {
  int iters = 0;
  bool converged = false;
  double rel = 0;  // last true (or estimated) relative residual w.r.t. bnorm
};

// Restarted GMRES on A x = b with operator precision `prec`; x is updated in
// place.  Convergence: ||b - A x|| <= tol * bnorm, checked with the true
// residual of the operator at every restart.
// Multiply-adds of one preconditioner application (all shapes).
double precond_madds(const pe_context* c) {
  double m = 0;
  for (const auto& t : c->pc.types) m += (double)(t.N + 1) * (t.N + 1) * (double)t.bodies.size();
  return m;
}

// r0 (optional, with its norm r0n): the residual b - A x at the starting x,
// already formed by the caller, so the first cycle does not recompute it.
//
// final_check = false (inner solves of the mixed refinement, whose caller
// forms the true residual in double right after): a cycle that ends on the
// residual estimate returns without recomputing b - A x.
GmresOut gmres(pe_context* c, int prec, const double* b, double* x, bool x_zero, double bnorm, double tol,
               int max_iters, pe_solve_info* info, int* mv64, int* mv32, const double* r0 = nullptr,
               double r0n = 0.0, bool final_check = true) {
  hipStream_t s = c->stream;
  const int64_t n = c->n_bead + c->n_body;
  const int m = std::max(1, std::min(c->p.gmres_restart, kMaxK - 1));
  KWork k = kwork(c, n, m);
  GmresOut out;
  double* partial = c->red.get();
  bool first = true;
  for (;;) {
    // r = b - A x
    double beta;
    if (first && r0) {
      if (r0 != k.r) dcopy(s, r0, k.r, n);
      beta = r0n;
      PE_HIP(hipStreamSynchronize(s));
      PE_HIP(hipMemcpy(k.nrm, &beta, sizeof(double), hipMemcpyHostToDevice));
    } else {
      if (first && x_zero) {
        dcopy(s, b, k.r, n);
      } else {
        apply_saddle_prec(c, prec, x, k.tmp);
        (prec == PE_MIXED ? *mv32 : *mv64) += 1;
        launch_sub(s, b, k.tmp, k.r, n);
      }
      launch_mdot(s, k.r, n, 1, k.r, n, partial, k.nrm, true);
      beta = fetch(c, k.nrm);
    }
    first = false;
    if (!std::isfinite(beta)) throw Error(PE_ERR_NUMERIC, "non-finite residual in GMRES");
    out.rel = beta / bnorm;
    if (beta <= tol * bnorm) {
      out.converged = true;
      return out;
    }
    if (out.iters >= max_iters) return out;
    launch_scale(s, k.r, k.nrm, k.V, n);
    launch_init_g(s, k.st, m, k.nrm);
    int jend = 0;
    double last_est = beta;
    const bool pre = c->p.precond != 0 && !c->pc.types.empty();
    // z_j = M^-1 v_j
    auto precond = [&](int j) {
      ProfScope ps(c->prof, s, PE_PROF_PRECOND, prec != PE_MIXED, precond_madds(c));
      double* vj = k.V + (size_t)j * n;
      double* zj = k.Z + (size_t)j * n;
      if (prec == PE_MIXED) precond_apply<float>(s, c, vj, zj);
      else precond_apply<double>(s, c, vj, zj);
    };
    bool z_ahead = false;  // z_j already enqueued while the host read step j-1's estimate
    for (int j = 0; j < m; ++j) {
      double* vj = k.V + (size_t)j * n;
      if (pre) {
        if (!z_ahead) precond(j);
        vj = k.Z + (size_t)j * n;
      }
      z_ahead = false;
      apply_saddle_prec(c, prec, vj, k.w);
      (prec == PE_MIXED ? *mv32 : *mv64) += 1;
      {
        ProfScope ps(c->prof, s, PE_PROF_KRYLOV, true);
        // CGS2, the next basis vector and the Givens step in four launches;
        // the residual estimate goes straight to page-locked host memory
        launch_cgs_step(s, k.V, n, j + 1, k.w, n, partial, k.h1, k.h2, k.nrm, k.V + (size_t)(j + 1) * n, k.st, m,
                        j, k.res, c->pinned);
        PE_HIP(hipEventRecord(c->ev_est, s));
      }
      // the host reads the estimate while the next step's preconditioner
      // runs (unused if this step ends the solve)
      if (pre && j + 1 < m && out.iters + 1 < max_iters) {
        precond(j + 1);
        z_ahead = true;
      }
      PE_HIP(hipEventSynchronize(c->ev_est));
      const double est = c->pinned[0];
      out.iters += 1;
      if (info && info->n_hist < 1024) info->hist[info->n_hist++] = est / bnorm;
      jend = j + 1;
      if (!std::isfinite(est)) throw Error(PE_ERR_NUMERIC, "non-finite residual estimate in GMRES");
      last_est = est;
      if (est <= tol * bnorm || out.iters >= max_iters) break;
    }
    launch_backsolve(s, k.st, m, jend, k.y);
    launch_maxpy(s, pre ? k.Z : k.V, n, jend, k.y, x, n, -1.0);  // x += Z y (flexible) or V y
    if (!final_check && (last_est <= tol * bnorm || out.iters >= max_iters)) {
      out.rel = last_est / bnorm;
      out.converged = last_est <= tol * bnorm;
      return out;
    }
  }
}

void compute_params(pe_context* c) {
  const pe_params& p = c->p;
  double hmax = 0;
  for (int d = 0; d < 3; ++d) hmax = std::max(hmax, p.box[d] / p.mesh[d]);
  c->hmax = hmax;
  c->V = p.box[0] * p.box[1] * p.box[2];
  const double lt = std::sqrt(std::log(1.0 / p.split_tol));
  if (p.xi > 0) c->xi = p.xi;
  else {
    double kc = 1e300;
    for (int d = 0; d < 3; ++d) kc = std::min(kc, M_PI * (p.mesh[d] - 1) / p.box[d]);
    c->xi = kc / (2.0 * lt);
  }
  c->eta = (hmax * c->xi) * (hmax * c->xi) * p.P / (M_PI * p.eta_c * p.eta_c);
  GridGeom& g = c->gg;
  for (int d = 0; d < 3; ++d) {
    g.N[d] = p.mesh[d];
    g.h[d] = p.box[d] / p.mesh[d];
    g.inv_h[d] = p.mesh[d] / p.box[d];
    g.L[d] = p.box[d];
  }
  g.Nzc = p.mesh[2] / 2 + 1;
  g.Nzs = (g.Nzc + 15) / 16 * 16;
  g.P = p.P;
  g.wexp = 2.0 * c->xi * c->xi / c->eta;
  g.wnorm = std::sqrt(2.0 * c->xi * c->xi / (M_PI * c->eta));
  g.h3 = g.h[0] * g.h[1] * g.h[2];
  g.eps = p.eps;
  g.fcoef = -4.0 * c->xi * c->xi * g.h3 / (p.eps * c->eta);
  for (int d = 0; d < 3; ++d) g.ntile[d] = (p.mesh[d] + 7) / 8;
}

void build_twiddles(pe_context* c) {
  for (int d = 0; d < 3; ++d) {
    const int n = c->p.mesh[d];
    make_fft_plan(n, c->plan[d]);
    std::vector<double2> t64(n);
    std::vector<float2> t32(n);
    for (int j = 0; j < n; ++j) {
      // exp(-2 pi i j / n), evaluated in long double
      const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)j / (long double)n;
      t64[j] = make_double2((double)cosl(a), (double)sinl(a));
      t32[j] = make_float2((float)t64[j].x, (float)t64[j].y);
    }
    c->tw64[d].ensure(n);
    c->tw32[d].ensure(n);
    PE_HIP(hipMemcpy(c->tw64[d].get(), t64.data(), sizeof(double2) * n, hipMemcpyHostToDevice));
    PE_HIP(hipMemcpy(c->tw32[d].get(), t32.data(), sizeof(float2) * n, hipMemcpyHostToDevice));
  }
}

// Tables that depend on the parameters only (twiddles, Green's-function
// factors, the scaled-erfc table) and the small reduction buffers, built
// in the workspace once per context.
void prepare_constants(pe_context* c) {
  if (c->consts_ready) return;
  build_twiddles(c);
  build_green_tables(c);
  build_erfcx_table(c->stream, c->erfcx_tab);
  c->rg.erfcx = c->erfcx_tab.get();
  c->sums.ensure(64);
  c->red.ensure((size_t)2 * kMaxK * 1024 + 8192);
  c->consts_ready = true;
}

// Device bytes a system of these sizes needs: every buffer of the context
// at its size for this system, with the data-dependent ones (the stored
// bead pairs, spreading-list entries, body-shape blocks, one recorded
// training solve) estimated: bead pairs from the mean bead density inside
// 1.1 r_c, every particle on 8 spreading tiles, two body shapes of the mean
// body size.  A configuration denser than that asks for more; the entry
// point then fails with PE_ERR_NOMEM and this call returns what it needed.
size_t estimate_workspace(const pe_context* c, int64_t nb, int64_t nbody, int64_t ni) {
  const pe_params& p = c->p;
  auto up = [](double b) { return (size_t)((b + Arena::kAlign - 1) / Arena::kAlign) * Arena::kAlign; };
  const double Nx = p.mesh[0], Ny = p.mesh[1], Nz = p.mesh[2];
  const double G = Nx * Ny * Nz;
  const double Nzs = std::ceil((Nz / 2 + 1) / 16.0) * 16.0;
  const double Gc = Nx * Ny * Nzs;
  const double n = (double)(nb + nbody), na = (double)(nb + ni);
  size_t b = 0;
  // parameter tables and reduction buffers
  b += up(24.0 * (Nx + Ny + Nz)) * 2 + up(16.0 * (Nx + Ny + Nz)) + up(64 * 1024);
  b += up(8.0 * (64 + nbody)) + up(8.0 * (2.0 * kMaxK * 1024 + 8192));
  // grids: two real double grids, the half spectrum, the kept float ion grid
  b += 2 * up(8 * G) + up(16 * Gc) + up(4 * G);
  // the system's copies
  b += up(8.0 * (nbody + 1)) + up(4.0 * nb) + 2 * up(24.0 * nb) + up(8.0 * nb) + up(24.0 * ni) + 2 * up(8.0 * ni) +
       up(8.0 * nbody) + up(32.0 * nbody) + up(4.0 * nbody);
  // the two particle sets (sorted records, lists, charges) and their cells
  const double lt = std::sqrt(std::log(1.0 / p.split_tol));
  const double rc_min = c->xi > 0 ? lt / c->xi : 0.0;
  double ncell = 1;
  for (int d = 0; d < 3; ++d) ncell *= rc_min > 0 ? std::min(512.0, std::max(1.0, std::floor(p.box[d] / rc_min))) : 1;
  const double ntile = std::ceil(Nx / 8) * std::ceil(Ny / 8) * std::ceil(Nz / 8);
  for (double m : {(double)nb, (double)ni})
    b += up(180.0 * m + 1) + up(12.0 * (ncell + 1)) + up(16.0 * (ntile + 1)) + 4 * Arena::kAlign;
  // per-particle outputs and scratch in caller order
  b += up(8 * na) * 3 + up(24 * na) * 3 + up(8 * std::max(n, na)) + up(8 * std::max(3 * na, n)) + up(8 * n) * 2 +
       up(8.0 * nb) * 2 + up(24.0 * nb) * 2 + up(8 * std::max(3 * n, 2 * na)) + up(72.0 * nbody) * 2;
  // Krylov basis and flexible directions
  const double m = std::max(1, std::min(p.gmres_restart, kMaxK - 1));
  b += up(8 * (m + 1) * n) + up(8 * m * n) + up(8 * ((m + 1) * (m + 4) + 8));
  // stored bead pairs (column, double and float value) and their rows
  const double V = p.box[0] * p.box[1] * p.box[2];
  const double rc = 1.1 * std::max(rc_min, 1e-12);
  const double nnz = (double)nb * (1.0 + (double)nb / V * 4.18879 * rc * rc * rc) * 1.5;
  b += up(16 * nnz) + up(8.0 * nb) * 3 + up(28.0 * nb) + up(4096);
  // body shapes: two shapes of the mean size (blocks in both precisions) and
  // the split-product partials
  if (nbody) {
    const double N = (double)nb / nbody;
    b += 2 * (up(12 * (N + 1) * (N + 1)) + up(12 * N * N) + up(48 * N)) + up(8 * 8 * (N + 1) * nbody) +
         up(8.0 * nbody) + up(2.0 * nbody);
  }
  // learned guess: features, one recorded solve, parameters and partials
  b += up(36.0 * nb) + up(44.0 * nb) + up(4.0 * nb) + up(4.0 * 256 * 4 * 5000) + up(4 * 4 * 5000);
  return b + (16u << 20);
}

void ensure_grids(pe_context* c) {
  const int64_t G = (int64_t)c->p.mesh[0] * c->p.mesh[1] * c->p.mesh[2];
  const int64_t Gc = (int64_t)c->p.mesh[0] * c->p.mesh[1] * c->gg.Nzs;
  c->gridA.ensure(G);
  c->gridB.ensure(G);
  c->gridC.ensure(Gc);
}

}  // namespace

namespace pe {
void saddle_product(pe_context* c, int prec, const double* x, double* y) { apply_saddle_prec(c, prec, x, y); }
}  // namespace pe

// =============================================================== C ABI

#define PE_API_BEGIN(ctx) ::pe::ArenaScope arena_scope_((ctx) ? &(ctx)->arena : nullptr); try {
#define PE_API_END(ctx)                                   \
  }                                                       \
  catch (const pe::Error& e) {                            \
    if (ctx) (ctx)->err = e.what();                       \
    else g_create_error = e.what();                       \
    return e.code;                                        \
  }                                                       \
  catch (const std::exception& e) {                       \
    if (ctx) (ctx)->err = e.what();                       \
    else g_create_error = e.what();                       \
    return PE_ERR_DEVICE;                                 \
  }                                                       \
  return PE_OK;

extern "C" {

pe_status pe_default_params(pe_params* p) {
  if (!p) return PE_ERR_ARG;
  std::memset(p, 0, sizeof(*p));
  p->P = 8;
  p->eta_c = 1.0;
  p->xi = 0.0;
  p->r_cut = 0.0;
  p->split_tol = 1e-8;
  p->eps = 1.0;
  p->precision = PE_FP64;
  p->reg = PE_REG_GAUSSIAN;
  p->shell_radius = 0.0;
  p->gmres_restart = 100;
  p->max_iters = 1000;
  p->rel_tol = 1e-6;
  p->inner_tol = 1e-7;
  p->max_refine = 8;
  p->use_learned_guess = 0;
  p->precond = 1;
  p->rhs_fp64 = 1;
  return PE_OK;
}

const char* pe_last_error(const pe_context* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

pe_status pe_create(const pe_params* params, void* hip_stream, pe_context** out) {
  pe_context* c = nullptr;
  PE_API_BEGIN(c)
  require(params != nullptr && out != nullptr, "null argument");
  const pe_params& p = *params;
  for (int d = 0; d < 3; ++d) {
    require(std::isfinite(p.box[d]) && p.box[d] > 0, "box lengths must be positive");
    require(p.mesh[d] >= 2, "mesh must have at least 2 points per axis");
  }
  require(p.mesh[2] % 2 == 0, "mesh[2] must be even (real-to-complex transform)");
  require(p.P >= 2 && p.P <= 16, "P must be in [2, 16]");
  for (int d = 0; d < 3; ++d)
    require(p.mesh[d] >= p.P + 8, "each mesh dimension must be at least P + 8");
  require(p.eps > 0 && std::isfinite(p.eps), "eps must be positive");
  require(p.eta_c > 0, "eta_c must be positive");
  require(p.split_tol > 0 && p.split_tol < 1, "split_tol must be in (0,1)");
  require(p.precision == PE_FP64 || p.precision == PE_MIXED, "unknown precision");
  require(p.reg == PE_REG_GAUSSIAN || p.reg == PE_REG_SHELL || p.reg == PE_REG_SHELL_PAPER,
          "unknown regularization");
  if (p.reg != PE_REG_GAUSSIAN) require(p.shell_radius > 0, "shell_radius must be positive");
  require(p.gmres_restart >= 1, "gmres_restart must be >= 1");
  require(p.max_iters >= 1, "max_iters must be >= 1");
  require(p.rel_tol > 0, "rel_tol must be positive");
  c = new pe_context();
  c->p = p;
  if (c->p.inner_tol <= 0) c->p.inner_tol = 1e-7;
  if (c->p.max_refine <= 0) c->p.max_refine = 8;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  PE_HIP(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
  PE_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  PE_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  PE_HIP(hipEventCreateWithFlags(&c->ev_est, hipEventDisableTiming));
  {
    int dev = 0, lds = 0;
    PE_HIP(hipGetDevice(&dev));
    PE_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    c->lds_per_block = lds;
    c->device = dev;
    // the allocation-free BD step's scratch array: its device address on
    // this GPU, looked up here (the library's init call) with the device current
    bd_static_scratch(dev);
  }
  pe::FFTPlan1D tmp;
  for (int d = 0; d < 3; ++d) make_fft_plan(p.mesh[d], tmp);
  compute_params(c);
  require(c->eta > 0 && c->eta < 1, "eta = (h xi)^2 P/(pi c^2) must lie in (0, 1); refine the mesh or lower xi");
  // no device memory yet: the constant tables are built in the workspace
  // by the first pe_set_system
  PE_HIP(hipHostMalloc((void**)&c->pinned, 512 * sizeof(double), hipHostMallocDefault));
  *out = c;
  c = nullptr;
  PE_API_END(c)
}

pe_status pe_destroy(pe_context* ctx) {
  if (!ctx) return PE_OK;
  if (ctx->guess) guess_destroy(ctx);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->ev_est) (void)hipEventDestroy(ctx->ev_est);
  delete ctx;
  return PE_OK;
}

pe_status pe_get_derived(const pe_context* ctx, double out[6]) {
  if (!ctx || !out) return PE_ERR_ARG;
  out[0] = ctx->xi;
  out[1] = ctx->rc;
  out[2] = ctx->eta;
  out[3] = ctx->hmax;
  out[4] = (double)ctx->nnz;
  out[5] = (double)ctx->rg.nc[0];
  return PE_OK;
}

pe_status pe_workspace_size(const pe_context* c, int64_t n_bead, int64_t n_body, int64_t n_ion, size_t* bytes) {
  if (!c || !bytes || n_bead < 0 || n_body < 0 || n_ion < 0) return PE_ERR_ARG;
  const size_t est = estimate_workspace(c, n_bead, n_body, n_ion);
  *bytes = std::max({est, c->arena.need, c->arena.peak});
  *bytes = (*bytes + Arena::kAlign - 1) / Arena::kAlign * Arena::kAlign;
  return PE_OK;
}

pe_status pe_set_workspace(pe_context* c, void* dev_ptr, size_t bytes) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  require(dev_ptr != nullptr || bytes == 0, "null workspace");
  require(reinterpret_cast<uintptr_t>(dev_ptr) % Arena::kAlign == 0, "workspace must be 256-byte aligned");
  // work in flight may still use the current region
  PE_HIP(hipStreamSynchronize(c->stream));
  PE_HIP(hipStreamSynchronize(c->aux));
  c->arena.migrate(static_cast<char*>(dev_ptr), bytes, c->stream);
  c->rg.erfcx = c->erfcx_tab.get();  // the one device address kept outside a buffer
  PE_API_END(c)
}

pe_status pe_workspace_info(const pe_context* c, size_t out[4]) {
  if (!c || !out) return PE_ERR_ARG;
  out[0] = c->arena.size;
  out[1] = c->arena.in_use;
  out[2] = c->arena.peak;
  out[3] = c->arena.need;
  return PE_OK;
}

pe_status pe_set_system(pe_context* c, int64_t n_body, const int64_t* body_offsets, const double* bead_pos,
                        const double* bead_sigma, const double* body_center, const double* body_quat,
                        const double* body_charge, int64_t n_ion, const double* ion_pos, const double* ion_charge,
                        const double* ion_sigma, const double E0[3]) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  c->have_system = false;
  c->have_solution = false;
  c->have_forces = false;
  c->have_eion = false;
  c->ion_parts_valid = false;
  require(n_body >= 0 && n_ion >= 0, "negative sizes");
  require(n_body == 0 || body_offsets != nullptr, "body_offsets is null");
  require(E0 != nullptr, "E0 is null");
  for (int d = 0; d < 3; ++d) require(std::isfinite(E0[d]), "E0 must be finite");
  std::vector<int64_t> off(n_body + 1, 0);
  if (n_body) std::copy(body_offsets, body_offsets + n_body + 1, off.begin());
  require(off[0] == 0, "body_offsets[0] must be 0");
  for (int64_t i = 0; i < n_body; ++i) require(off[i + 1] > off[i], "every body needs at least one bead");
  const int64_t nb = off[n_body];
  require(nb < ((int64_t)1 << 31) && n_ion < ((int64_t)1 << 31), "too many particles");
  require(nb == 0 || (bead_pos && bead_sigma), "bead arrays are null");
  require(n_body == 0 || (body_center && body_charge), "body arrays are null");
  require(n_ion == 0 || (ion_pos && ion_charge && ion_sigma), "ion arrays are null");
  prepare_constants(c);
  hipStream_t s = c->stream;
  c->n_body = n_body;
  c->n_bead = nb;
  c->n_ion = n_ion;
  // the body structure (offsets, bead -> body) is uploaded again only when
  // it changed (a Brownian run keeps it from step to step)
  const bool same_bodies = c->bodies_uploaded && c->h_off == off;
  c->h_off = off;
  for (int d = 0; d < 3; ++d) c->E0[d] = E0[d];
  // copies
  c->off.ensure(n_body + 1);
  c->body_of.ensure(nb);
  if (!same_bodies) {
    c->bodies_uploaded = false;
    PE_HIP(hipMemcpyAsync(c->off.get(), off.data(), sizeof(int64_t) * (n_body + 1), hipMemcpyHostToDevice, s));
    std::vector<int> bof(nb);
    for (int64_t i = 0; i < n_body; ++i)
      for (int64_t j = off[i]; j < off[i + 1]; ++j) bof[j] = (int)i;
    if (nb) PE_HIP(hipMemcpyAsync(c->body_of.get(), bof.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
    PE_HIP(hipStreamSynchronize(s));  // (the host arrays end with this scope)
    c->bodies_uploaded = true;
  }
  c->bead_x.ensure(3 * nb);
  c->bead_sig.ensure(nb);
  c->rel.ensure(3 * nb);
  c->ion_x.ensure(3 * n_ion);
  c->ion_q.ensure(n_ion);
  c->ion_sig.ensure(n_ion);
  c->body_Q.ensure(n_body);
  c->quat.ensure(4 * n_body);
  dcopy(s, bead_pos, c->bead_x.get(), 3 * nb);
  dcopy(s, bead_sigma, c->bead_sig.get(), nb);
  dcopy(s, ion_pos, c->ion_x.get(), 3 * n_ion);
  dcopy(s, ion_charge, c->ion_q.get(), n_ion);
  dcopy(s, ion_sigma, c->ion_sig.get(), n_ion);
  dcopy(s, body_charge, c->body_Q.get(), n_body);
  if (body_quat) dcopy(s, body_quat, c->quat.get(), 4 * n_body);
  else {
    std::vector<double> qi(4 * n_body, 0.0);
    for (int64_t i = 0; i < n_body; ++i) qi[4 * i] = 1.0;
    if (n_body) PE_HIP(hipMemcpyAsync(c->quat.get(), qi.data(), sizeof(double) * 4 * n_body, hipMemcpyHostToDevice, s));
    PE_HIP(hipStreamSynchronize(s));
  }
  // the pair structure's displacement check behind the input checks' wait
  launch_max_disp_early(c);
  // validation on the device
  double sig_max = 0, sig_min = INFINITY;
  {
    std::vector<StatReq> reqs;
    for (int d = 0; d < 3; ++d) {
      reqs.push_back({c->bead_x.get(), nb, 3, d});
      reqs.push_back({c->ion_x.get(), n_ion, 3, d});
    }
    reqs.push_back({c->bead_sig.get(), nb, 1, 0});
    reqs.push_back({c->ion_sig.get(), n_ion, 1, 0});
    reqs.push_back({c->ion_q.get(), n_ion, 1, 0});
    reqs.push_back({c->body_Q.get(), n_body, 1, 0});
    const std::vector<Stats> st = array_stats(c, reqs);
    for (int d = 0; d < 3; ++d) {
      require(st[2 * d].bad == 0, "bead positions must be finite");
      require(st[2 * d + 1].bad == 0, "ion positions must be finite");
    }
    const Stats& a = st[6];
    const Stats& b = st[7];
    const Stats& q1 = st[8];
    const Stats& q2 = st[9];
    require(a.bad == 0 && b.bad == 0 && q1.bad == 0 && q2.bad == 0, "charges and widths must be finite");
    if (c->p.reg == PE_REG_GAUSSIAN) {
      require(nb == 0 || a.mn > 0, "bead widths must be positive");
      require(n_ion == 0 || b.mn > 0, "ion widths must be positive");
    }
    if (nb) { sig_max = std::max(sig_max, a.mx); sig_min = std::min(sig_min, a.mn); }
    if (n_ion) { sig_max = std::max(sig_max, b.mx); }
    c->bead_sig_uniform = (nb && a.mx == a.mn) ? a.mx : -1.0;
  }
  // cutoff and cells
  const double lt = std::sqrt(std::log(1.0 / c->p.split_tol));
  if (c->p.r_cut > 0) c->rc = c->p.r_cut;
  else if (c->p.reg == PE_REG_GAUSSIAN) c->rc = lt * std::max(1.0 / c->xi, 2.0 * sig_max);
  else if (c->p.reg == PE_REG_SHELL_PAPER) c->rc = 2.0 * c->p.shell_radius + lt / c->xi;
  else c->rc = std::max(lt / c->xi, 2.0 * c->p.shell_radius);
  const double Lmin = std::min(c->p.box[0], std::min(c->p.box[1], c->p.box[2]));
  require(c->rc <= 0.5 * Lmin * (1 + 1e-12),
          "real-space cutoff " + std::to_string(c->rc) + " exceeds half the box; use a finer mesh or a larger box");
  RealGeom& rg = c->rg;
  for (int d = 0; d < 3; ++d) {
    rg.L[d] = c->p.box[d];
    rg.inv_L[d] = 1.0 / c->p.box[d];
    int nc = (int)std::floor(c->p.box[d] / c->rc);
    if (nc < 3) nc = 1;
    if (nc > 512) nc = 512;
    rg.nc[d] = nc;
    rg.cell_inv[d] = nc / c->p.box[d];
  }
  rg.rc2 = c->rc * c->rc;
  rg.xi = c->xi;
  rg.eps = c->p.eps;
  rg.reg = c->p.reg;
  rg.a = c->p.shell_radius;
  // relative positions, cells, bead operator, grids
  if (nb)
    hipLaunchKernelGGL(rel_kernel, dim3(nblk(nb, 256)), dim3(256), 0, s, c->bead_x.get(), body_center,
                       c->body_of.get(), nb, c->rel.get());
  PE_CHECK_LAUNCH();
  // the two sets' cells and lists: ions on the auxiliary stream, so their
  // kernels run while the host works on the beads' counts and vice versa
  // (both sets' counts are launched before the first wait)
  fork_aux(c);
  cells_count(s, c->B, c->bead_x.get(), c->bead_sig.get(), 0.0, nb, rg);
  cells_count(c->aux, c->I, c->ion_x.get(), c->ion_sig.get(), 0.0, n_ion, rg);
  PE_HIP(hipStreamSynchronize(s));
  cells_finish(s, c->B, c->body_of.get(), rg);
  PE_HIP(hipStreamSynchronize(c->aux));
  cells_finish(c->aux, c->I, nullptr, rg);
  // the bodies' shape matches behind the same wait as the beads' tile counts
  shape_match_launch(c);
  // beads are spread by every Krylov product: tile lists; ions once per
  // configuration in single precision: their sorted home lists serve
  build_tiles(s, c->B, c->gg, false);
  build_tiles(c->aux, c->I, c->gg, c->p.precision == PE_MIXED);
  update_pair_tables(s, c->pair_tabs, rg, c->B, c->I);  // the widths are known on the host by now
  // bead-only set-up still overlaps the ions' lists
  shape_setup(c);
  build_bead_matrix(c);
  join_aux(c);
  ensure_grids(c);
  c->phi_w.ensure(nb + n_ion + 1);
  c->phi_all.ensure(nb + n_ion + 1);
  c->E_all.ensure(3 * (nb + n_ion) + 1);
  c->forces.ensure(3 * (nb + n_ion) + 1);
  c->xsol.ensure(nb + n_body + 1);
  c->sums.ensure(64 + n_body);
  c->rhs_b.ensure(nb + n_body + 1);
  c->have_system = true;
  if (c->guess) guess_on_system(c);
  PE_HIP(hipStreamSynchronize(s));
  PE_API_END(c)
}

pe_status pe_apply_potential(pe_context* c, const double* charges, double* psi_out, double* field_out,
                             int32_t precision) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  if (!c->have_system) throw Error(PE_ERR_STATE, "pe_set_system has not been called");
  require(charges && psi_out, "null charges or output");
  require(precision == PE_FP64 || precision == PE_MIXED, "unknown precision");
  const int64_t nb = c->n_bead;
  if (precision == PE_MIXED)
    all_potential<float>(c, charges, charges + nb, psi_out, field_out, nullptr, nullptr, nullptr);
  else
    all_potential<double>(c, charges, charges + nb, psi_out, field_out, nullptr, nullptr, nullptr);
  PE_HIP(hipStreamSynchronize(c->stream));
  c->prof.flush();
  PE_API_END(c)
}

pe_status pe_solve_polarization(pe_context* c, const double* q_init, double* q_out, double* dpsi_out,
                                double* dipole_out, pe_solve_info* info) {
  if (!c) return PE_ERR_ARG;
  pe_status status = PE_OK;
  PE_API_BEGIN(c)
  if (!c->have_system) throw Error(PE_ERR_STATE, "pe_set_system has not been called");
  require(q_out && dpsi_out, "null output");
  pe_solve_info local;
  pe_solve_info* inf = info ? info : &local;
  std::memset(inf, 0, sizeof(*inf));
  hipStream_t s = c->stream;
  const auto t0 = Clock::now();
  const int64_t nb = c->n_bead, nbody = c->n_body, n = nb + nbody;
  double* b = c->rhs_b.get();
  double* x = c->xsol.get();
  build_rhs(c, b);
  // ||b||
  KWork k = kwork(c, n, std::max(1, std::min(c->p.gmres_restart, kMaxK - 1)));
  launch_mdot(s, b, n, 1, b, n, c->red.get(), k.nrm, true);
  const double bnorm = fetch(c, k.nrm);
  inf->rhs_norm = bnorm;
  const auto t1 = Clock::now();
  // initial guess
  bool x_zero = true;
  PE_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
  if (q_init) {
    dcopy(s, q_init, x, nb);
    x_zero = false;
  } else if (c->p.use_learned_guess) {
    require(c->guess != nullptr && guess_ready(c), "use_learned_guess set but no model is loaded");
    guess_predict(c, x);
    x_zero = false;
  }
  const auto t2 = Clock::now();
  int mv64 = 0, mv32 = 0;
  if (bnorm == 0.0) {
    inf->rel_residual = 0;
  } else {
    // residual at the guess; it is also the first residual of the solve
    // below.  Mixed precision forms it with the float operator: it only
    // starts the first refinement, whose correction is checked by the next
    // double residual.
    double rgn = bnorm;
    if (!x_zero) {
      const int rp = c->p.precision == PE_MIXED ? PE_MIXED : PE_FP64;
      apply_saddle_prec(c, rp, x, k.tmp);
      (rp == PE_MIXED ? mv32 : mv64)++;
      launch_sub(s, b, k.tmp, k.r, n);
      // the guess sets charges only: give it the best potential offsets
      c->sums.ensure(64 + nbody);
      double* rs = c->sums.get() + 64;
      launch_seg_sum(s, c->off.get(), nbody, k.r, rs);
      hipLaunchKernelGGL(start_offsets_kernel, dim3(nblk(std::max(nb, nbody), 256)), dim3(256), 0, s, nb, nbody,
                         c->off.get(), c->body_of.get(), rs, k.r, x);
      PE_CHECK_LAUNCH();
      launch_mdot(s, k.r, n, 1, k.r, n, c->red.get(), k.nrm, true);
      rgn = fetch(c, k.nrm);
      inf->rel_residual_guess = rgn / bnorm;
    } else {
      inf->rel_residual_guess = 1.0;
    }
    const double tol = c->p.rel_tol;
    if (c->p.precision == PE_FP64) {
      GmresOut o = gmres(c, PE_FP64, b, x, x_zero, bnorm, tol, c->p.max_iters, inf, &mv64, &mv32,
                         x_zero ? nullptr : k.r, rgn);
      inf->iters = o.iters;
      inf->rel_residual = o.rel;
      if (!o.converged) status = PE_ERR_NOT_CONVERGED;
    } else {
      // double iterative refinement around float-operator GMRES solves
      double* r = c->phi_all.get();  // reuse as residual vector storage (size >= n needed)
      c->phi_all.ensure(std::max<int64_t>(n, nb + c->n_ion) + 1);
      r = c->phi_all.get();
      double* d = c->E_all.get();
      c->E_all.ensure(std::max<int64_t>(n, 3 * (nb + c->n_ion)) + 1);
      d = c->E_all.get();
      int total = 0;
      bool conv = false;
      double rel = 1.0;
      for (int outer = 0; outer <= c->p.max_refine; ++outer) {
        // r = b - A64 x (at the start: b, or the residual of the guess)
        double rn;
        if (outer == 0) {
          dcopy(s, x_zero ? b : k.r, r, n);
          rn = rgn;
        } else {
          apply_saddle_prec(c, PE_FP64, x, k.tmp);
          mv64++;
          launch_sub(s, b, k.tmp, r, n);
          launch_mdot(s, r, n, 1, r, n, c->red.get(), k.nrm, true);
          rn = fetch(c, k.nrm);
        }
        if (!std::isfinite(rn)) throw Error(PE_ERR_NUMERIC, "non-finite residual in refinement");
        rel = rn / bnorm;
        // the residual of a guess was formed with the float operator:
        // convergence is only accepted on a double residual
        const bool r_is_fp64 = outer > 0 || x_zero;
        if (rel <= tol && r_is_fp64) { conv = true; break; }
        if (rel <= tol) continue;
        if (outer == c->p.max_refine || total >= c->p.max_iters) break;
        inf->outer_refinements++;
        PE_HIP(hipMemsetAsync(d, 0, sizeof(double) * n, s));
        const double itol = std::max(c->p.inner_tol, 0.5 * tol / std::max(rel, 1e-300));
        GmresOut o = gmres(c, PE_MIXED, r, d, true, rn, std::min(itol, 0.5), c->p.max_iters - total, inf,
                           &mv64, &mv32, nullptr, 0.0, false);
        total += o.iters;
        launch_axpby(s, 1.0, d, 1.0, x, n);
      }
      inf->iters = total;
      inf->rel_residual = rel;
      if (!conv) status = PE_ERR_NOT_CONVERGED;
    }
  }
  inf->matvecs_fp64 = mv64;
  inf->matvecs_fp32 = mv32;
  // outputs
  dcopy(s, x, q_out, nb);
  dcopy(s, x + nb, dpsi_out, nbody);
  if (dipole_out) launch_body_outputs(s, c->off.get(), nbody, c->rel.get(), x, nullptr, nullptr, dipole_out,
                                      nullptr, nullptr, nullptr);
  PE_HIP(hipStreamSynchronize(s));
  c->prof.flush();
  const auto t3 = Clock::now();
  inf->t_rhs = secs(t0, t1);
  inf->t_guess = secs(t1, t2);
  inf->t_solve = secs(t2, t3);
  inf->t_total = secs(t0, t3);
  c->have_solution = true;
  if (status != PE_OK) {
    c->err = status == PE_ERR_NOT_CONVERGED ? "GMRES did not reach rel_tol within max_iters" : "solve failed";
    return status;
  }
  PE_API_END(c)
}

pe_status pe_grand_capacitance(pe_context* c, double* C_out, double* eps_eff, pe_solve_info* info) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  if (!c->have_system) throw Error(PE_ERR_STATE, "pe_set_system has not been called");
  require(c->n_body > 0, "the capacitance needs at least one body");
  if (info) std::memset(info, 0, sizeof(*info));
  grand_capacitance(c, C_out, eps_eff, info);
  PE_API_END(c)
}

pe_status pe_apply_saddle(pe_context* c, const double* x, double* y, int32_t precision) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  if (!c->have_system) throw Error(PE_ERR_STATE, "pe_set_system has not been called");
  require(x && y, "null vector");
  require(precision == PE_FP64 || precision == PE_MIXED, "unknown precision");
  apply_saddle_prec(c, precision, x, y);
  PE_HIP(hipStreamSynchronize(c->stream));
  c->prof.flush();
  PE_API_END(c)
}

pe_status pe_profile_enable(pe_context* c, int32_t on) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  PE_HIP(hipStreamSynchronize(c->stream));
  c->prof.reset();
  c->prof.on = on != 0;
  c->pair_count.ensure(2);
  PE_HIP(hipMemsetAsync(c->pair_count.get(), 0, 2 * sizeof(unsigned long long), c->stream));
  PE_HIP(hipStreamSynchronize(c->stream));
  PE_API_END(c)
}

pe_status pe_profile_select(pe_context* c, uint32_t class_mask) {
  if (!c) return PE_ERR_ARG;
  c->prof.mask = class_mask;
  return PE_OK;
}

pe_status pe_profile_read(pe_context* c, double* out) {
  if (!c || !out) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  PE_HIP(hipStreamSynchronize(c->stream));
  c->prof.flush();
  unsigned long long np[2] = {0, 0};
  if (c->pair_count.get())
    PE_HIP(hipMemcpy(np, c->pair_count.get(), sizeof(np), hipMemcpyDeviceToHost));
  for (int i = 0; i < 2 * PE_PROF_NCLASS; ++i) {
    double w = c->prof.work[i];
    if (i == PE_PROF_PAIR) w = (double)np[0];
    if (i == PE_PROF_PAIR + PE_PROF_NCLASS) w = (double)np[1];
    out[3 * i] = c->prof.cnt[i];
    out[3 * i + 1] = c->prof.ms[i];
    out[3 * i + 2] = w;
  }
  PE_API_END(c)
}

pe_status pe_forces_torques(pe_context* c, double* body_force, double* body_torque, double* body_energy,
                            double* ion_force, double* bead_force, double* total_energy) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  if (!c->have_solution) throw Error(PE_ERR_STATE, "pe_solve_polarization has not been called");
  require(total_energy != nullptr, "total_energy is null");
  hipStream_t s = c->stream;
  const int64_t nb = c->n_bead, ni = c->n_ion, na = nb + ni;
  c->phi_all.ensure(na + 1);
  c->E_all.ensure(3 * na + 1);
  c->forces.ensure(3 * na + 1);
  c->kvec.ensure(2 * na + 2);
  double* chg = c->kvec.get();     // all charges
  double* u = chg + na;            // energies
  dcopy(s, c->xsol.get(), chg, nb);
  dcopy(s, c->ion_q.get(), chg + nb, ni);
  double* f = c->forces.get();
  if (c->p.precision == PE_MIXED)
    all_potential<float>(c, chg, chg + nb, c->phi_all.get(), c->E_all.get(), f, u, chg, true);
  else
    all_potential<double>(c, chg, chg + nb, c->phi_all.get(), c->E_all.get(), f, u, chg);
  c->bodyF.ensure(3 * std::max<int64_t>(c->n_body, 1));
  c->bodyL.ensure(3 * std::max<int64_t>(c->n_body, 1));
  launch_body_outputs(s, c->off.get(), c->n_body, c->rel.get(), chg, f, u, nullptr, c->bodyF.get(), c->bodyL.get(),
                      body_energy);
  if (body_force) dcopy(s, c->bodyF.get(), body_force, 3 * c->n_body);
  if (body_torque) dcopy(s, c->bodyL.get(), body_torque, 3 * c->n_body);
  if (ion_force) dcopy(s, f + 3 * nb, ion_force, 3 * ni);
  if (bead_force) dcopy(s, f, bead_force, 3 * nb);
  double* tot = scal(c);
  {
    const int64_t chunk = std::max<int64_t>(4096, (na + 1023) / 1024);
    const int64_t nparts = std::max<int64_t>(1, (na + chunk - 1) / chunk);
    hipLaunchKernelGGL(sum_partial_kernel, dim3((unsigned)nparts), dim3(256), 0, s, u, na, chunk, c->red.get());
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1024), 0, s, c->red.get(), nparts, tot);
  }
  PE_CHECK_LAUNCH();
  *total_energy = fetch(c, tot);
  c->have_forces = true;
  PE_API_END(c)
}

}  // extern "C"
