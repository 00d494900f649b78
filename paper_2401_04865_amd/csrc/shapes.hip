// Rigid-body shape types and the dense per-shape products.
//
// Bodies with the same bead count, widths and intra-body distances share
// everything that depends only on those distances: the free-space body
// saddle block of the block-Jacobi preconditioner, and the intra-body part of
// the real-space sum (section "Real-space sum"; for a body smaller than half
// the box every intra-body pair is its own minimum image, so the block does
// not depend on where the body sits or how it is turned).  A shape is
// recognised by the distances of each bead to up to four reference beads,
// chosen non-collinear and non-coplanar, which fix every bead's position up
// to a rigid motion; all bodies are compared with a shape at once on the
// device, so only one body per new shape is ever copied to the host.  Shapes
// are cached across configurations.
//
// A per-shape product Y = A X, with column b of X the bead segment of body b
// (bordered by its dPsi entry for the saddle block), runs as one tiled
// matrix product over all bodies of the shape.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pe_internal.hpp"
#include "precond.hpp"

namespace pe {

namespace {

// Bodies larger than this keep their intra-body pairs in the sparse list.
constexpr int kNearMax = 4096;

// One workgroup per body: does body b match shape `type_id`?  Bodies already
// assigned, or of another bead count, are left alone.
__global__ void __launch_bounds__(256) match_kernel(const double* __restrict__ rel, const double* __restrict__ sig,
                                                    const int64_t* __restrict__ off, int N, int nref,
                                                    const int* __restrict__ refidx, const double* __restrict__ dref,
                                                    const double* __restrict__ dsig, double tol, int type_id,
                                                    int* __restrict__ assigned) {
  const int64_t b = blockIdx.x;
  if (assigned[b] >= 0) return;  // same value for the whole block
  const int64_t o = off[b];
  if (off[b + 1] - o != N) return;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int mine = 0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const double* rj = rel + 3 * (o + j);
    if (!(fabs(sig[o + j] - dsig[j]) <= 1e-12 * fabs(dsig[j]))) mine = 1;
    for (int k = 0; k < nref; ++k) {
      const double* rk = rel + 3 * (o + refidx[k]);
      const double dx = rj[0] - rk[0], dy = rj[1] - rk[1], dz = rj[2] - rk[2];
      const double d = sqrt(dx * dx + dy * dy + dz * dz);
      if (!(fabs(d - dref[(int64_t)j * nref + k]) <= tol)) mine = 1;
    }
  }
  if (mine) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0 && bad == 0) assigned[b] = type_id;
}

// Tiled product for the bodies of one shape: 32 x 32 output tiles (rows of A
// x bodies), K staged through LDS 64 at a time, the next chunk's loads issued
// before the current chunk's products so they are in flight meanwhile.
// Thread (tx, ty) owns rows {ty, ty + 16} and columns {tx, tx + 16}.
constexpr int kGM = 32, kGN = 32, kGK = 64, kGLoads = kGK * kGM / 256;

template <typename T, bool BORDER, bool ACCUM>
__global__ void __launch_bounds__(256) body_gemm_kernel(const T* __restrict__ A, int N,
                                                        const int* __restrict__ bodies, int nbt,
                                                        const int64_t* __restrict__ off, int64_t n_bead,
                                                        const double* __restrict__ x, double* __restrict__ y) {
  const int Np = BORDER ? N + 1 : N;
  __shared__ T As[kGK][kGM + 1];
  __shared__ T Xs[kGK][kGN + 1];
  __shared__ int64_t boff[kGN];
  __shared__ int64_t bpsi[kGN];
  const int row0 = blockIdx.x * kGM;
  const int col0 = blockIdx.y * kGN;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (threadIdx.x < kGN) {
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
  // loader: element e = threadIdx.x + 256 i -> (kk = e % kGK, r = e / kGK)
  T ra[kGLoads], rx[kGLoads];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < kGLoads; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int kk = e % kGK, r = e / kGK;
      const int gr = row0 + r, gk = k0 + kk;
      ra[i] = (gr < Np && gk < Np) ? A[(int64_t)gr * Np + gk] : (T)0;
      T v = 0;
      if (boff[r] >= 0 && gk < Np) v = (T)((!BORDER || gk < N) ? x[boff[r] + gk] : x[bpsi[r]]);
      rx[i] = v;
    }
  };
  T acc[2][2] = {{0, 0}, {0, 0}};
  load(0);
  for (int k0 = 0; k0 < Np; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < kGLoads; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int kk = e % kGK, r = e / kGK;
      As[kk][r] = ra[i];
      Xs[kk][r] = rx[i];
    }
    __syncthreads();
    if (k0 + kGK < Np) load(k0 + kGK);
#pragma unroll 16
    for (int kk = 0; kk < kGK; ++kk) {
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
      const int64_t o = (!BORDER || gr < N) ? boff[cc] + gr : bpsi[cc];
      y[o] = ACCUM ? y[o] + (double)acc[p][q] : (double)acc[p][q];
    }
  }
}

double dist3(const double* a, const double* b) {
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return std::sqrt(dx * dx + dy * dy + dz * dz);
}

// New shape from one body's relative positions and widths: reference beads
// (the first bead, the farthest from it, the farthest from their line, the
// farthest from their plane; the last two only if the body is not collinear
// or planar) and the signature table.
void init_type(pe_context* c, BodyType& t, const double* rel, const double* sig, int N) {
  t.N = N;
  t.ref.assign(rel, rel + 3 * N);
  t.sig.assign(sig, sig + N);
  int r0 = 0, r1 = 0;
  double best = -1;
  for (int j = 0; j < N; ++j) {
    const double d = dist3(&rel[3 * j], &rel[0]);
    if (d > best) { best = d; r1 = j; }
  }
  const double scale = std::max(best, 1e-300);
  t.refidx[0] = r0;
  t.nref = 1;
  if (best > 1e-9 * scale && N > 1) {
    t.refidx[t.nref++] = r1;
    // farthest from the line (r0, r1)
    const double* a = &rel[3 * r0];
    const double* b = &rel[3 * r1];
    const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    int r2 = -1;
    double bl = 0;
    for (int j = 0; j < N; ++j) {
      const double w[3] = {rel[3 * j] - a[0], rel[3 * j + 1] - a[1], rel[3 * j + 2] - a[2]};
      const double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz = u[0] * w[1] - u[1] * w[0];
      const double d = std::sqrt((cx * cx + cy * cy + cz * cz) / uu);
      if (d > bl) { bl = d; r2 = j; }
    }
    if (r2 >= 0 && bl > 1e-6 * scale) {
      t.refidx[t.nref++] = r2;
      const double* cpt = &rel[3 * r2];
      const double v[3] = {cpt[0] - a[0], cpt[1] - a[1], cpt[2] - a[2]};
      double nrm[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
      const double nn = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
      int r3 = -1;
      double bp = 0;
      for (int j = 0; j < N; ++j) {
        const double d = std::fabs((rel[3 * j] - a[0]) * nrm[0] + (rel[3 * j + 1] - a[1]) * nrm[1] +
                                   (rel[3 * j + 2] - a[2]) * nrm[2]) / nn;
        if (d > bp) { bp = d; r3 = j; }
      }
      if (r3 >= 0 && bp > 1e-6 * scale) t.refidx[t.nref++] = r3;
    }
  }
  std::vector<double> dref((size_t)N * t.nref);
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < t.nref; ++k) dref[(size_t)j * t.nref + k] = dist3(&rel[3 * j], &rel[3 * t.refidx[k]]);
  t.scale = scale;
  double cen[3] = {0, 0, 0};
  for (int j = 0; j < N; ++j)
    for (int d = 0; d < 3; ++d) cen[d] += rel[3 * j + d] / N;
  t.extent = 0;
  for (int j = 0; j < N; ++j) t.extent = std::max(t.extent, dist3(&rel[3 * j], cen));
  hipStream_t s = c->stream;
  t.dref.ensure(dref.size());
  t.dsig.ensure(N);
  t.drefidx.ensure(4);
  PE_HIP(hipMemcpyAsync(t.dref.get(), dref.data(), sizeof(double) * dref.size(), hipMemcpyHostToDevice, s));
  PE_HIP(hipMemcpyAsync(t.dsig.get(), sig, sizeof(double) * N, hipMemcpyHostToDevice, s));
  PE_HIP(hipMemcpyAsync(t.drefidx.get(), t.refidx, sizeof(int) * 4, hipMemcpyHostToDevice, s));
  PE_HIP(hipStreamSynchronize(s));
}

void launch_match(pe_context* c, const BodyType& t, int type_id) {
  // distances agree to 1e-11 of the body size for copies of one rigid shape
  // moved and turned in double precision
  const double tol = 1e-11 * t.scale;
  hipLaunchKernelGGL(match_kernel, dim3((unsigned)c->n_body), dim3(256), 0, c->stream, c->rel.get(),
                     c->bead_sig.get(), c->off.get(), t.N, t.nref, t.drefidx.get(), t.dref.get(), t.dsig.get(),
                     tol, type_id, c->pc.assigned.get());
  PE_CHECK_LAUNCH();
}

}  // namespace

void shape_setup(pe_context* c) {
  Precond& pc = c->pc;
  hipStream_t s = c->stream;
  for (auto& t : pc.types) t.bodies.clear();
  const int64_t nbody = c->n_body;
  if (nbody == 0) return;
  pc.assigned.ensure(nbody);
  pc.dense.ensure(nbody);
  PE_HIP(hipMemsetAsync(pc.assigned.get(), 0xFF, sizeof(int) * nbody, s));  // -1: unassigned
  for (size_t ti = 0; ti < pc.types.size(); ++ti) launch_match(c, pc.types[ti], (int)ti);
  std::vector<int> asg(nbody);
  auto fetch_assigned = [&]() {
    PE_HIP(hipMemcpyAsync(asg.data(), pc.assigned.get(), sizeof(int) * nbody, hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
  };
  fetch_assigned();
  for (int64_t first = 0;;) {
    while (first < nbody && asg[first] >= 0) ++first;
    if (first == nbody) break;
    // a new shape from the first unmatched body
    const int64_t o = c->h_off[first];
    const int N = (int)(c->h_off[first + 1] - o);
    std::vector<double> rel(3 * (size_t)N), sig(N);
    PE_HIP(hipMemcpyAsync(rel.data(), c->rel.get() + 3 * o, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, s));
    PE_HIP(hipMemcpyAsync(sig.data(), c->bead_sig.get() + o, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
    pc.types.emplace_back();
    BodyType& t = pc.types.back();
    init_type(c, t, rel.data(), sig.data(), N);
    launch_match(c, t, (int)pc.types.size() - 1);
    fetch_assigned();
    require(asg[first] == (int)pc.types.size() - 1, "a body does not match its own shape");
  }
  for (int64_t b = 0; b < nbody; ++b) pc.types[asg[b]].bodies.push_back((int)b);
  const double Lmin = std::min(c->p.box[0], std::min(c->p.box[1], c->p.box[2]));
  std::vector<unsigned char> dense(nbody, 0);
  for (auto& t : pc.types) {
    if (t.bodies.empty()) continue;
    t.dbodies.ensure(t.bodies.size());
    PE_HIP(hipMemcpyAsync(t.dbodies.get(), t.bodies.data(), sizeof(int) * t.bodies.size(), hipMemcpyHostToDevice, s));
    if (c->p.precond && !t.have_inv) {
      require(t.N <= 16384, "body too large for the block preconditioner (N > 16384)");
      build_type_inverse(c, t);
      t.have_inv = true;
    }
    // every intra-body pair closer than half the box: the dense block is exact
    const bool near_ok = t.N <= kNearMax && 2.0 * t.extent < 0.5 * Lmin * (1.0 - 1e-9);
    if (near_ok && !t.near) {
      t.R64.ensure((size_t)t.N * t.N);
      t.R32.ensure((size_t)t.N * t.N);
      build_near_block(s, t, c->rg, t.R64.get(), t.R32.get());
      t.near = true;
    }
    if (t.near)
      for (int b : t.bodies) dense[b] = 1;
  }
  PE_HIP(hipMemcpyAsync(pc.dense.get(), dense.data(), nbody, hipMemcpyHostToDevice, s));
  PE_HIP(hipStreamSynchronize(s));
}

template <typename T>
void launch_body_gemm(hipStream_t s, const T* A, int N, bool bordered, bool accumulate, const int* bodies,
                      int nbt, const int64_t* off, int64_t n_bead, const double* x, double* y) {
  if (nbt == 0 || N == 0) return;
  const int Np = bordered ? N + 1 : N;
  const dim3 grid((unsigned)((Np + kGM - 1) / kGM), (unsigned)((nbt + kGN - 1) / kGN));
  if (bordered) {
    require(!accumulate, "bordered product overwrites");
    hipLaunchKernelGGL((body_gemm_kernel<T, true, false>), grid, dim3(256), 0, s, A, N, bodies, nbt, off, n_bead,
                       x, y);
  } else if (accumulate) {
    hipLaunchKernelGGL((body_gemm_kernel<T, false, true>), grid, dim3(256), 0, s, A, N, bodies, nbt, off, n_bead,
                       x, y);
  } else {
    hipLaunchKernelGGL((body_gemm_kernel<T, false, false>), grid, dim3(256), 0, s, A, N, bodies, nbt, off, n_bead,
                       x, y);
  }
  PE_CHECK_LAUNCH();
}

template void launch_body_gemm<float>(hipStream_t, const float*, int, bool, bool, const int*, int, const int64_t*,
                                      int64_t, const double*, double*);
template void launch_body_gemm<double>(hipStream_t, const double*, int, bool, bool, const int*, int, const int64_t*,
                                       int64_t, const double*, double*);

}  // namespace pe
