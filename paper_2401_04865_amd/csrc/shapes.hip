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

// Tiled product for the bodies of one shape on the matrix cores (a dense
// contraction: every entry of A meets every body): 64 x 64 output tiles (rows
// of A x bodies) per workgroup, a 32 x 32 quarter per wavefront made of 2 x 2
// MFMA 16 x 16 x 4 blocks (fp32: v_mfma_f32_16x16x4f32, fp64:
// v_mfma_f64_16x16x4f64).  K is staged through LDS 32 at a time; the next
// chunk's global loads are issued before the current chunk's products.
// Operand layout (one wavefront): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; it receives D[4 (l / 16) + i][l % 16] in register i for
// fp32, and D[4 i + l / 16][l % 16] for fp64 (row groups of one), i = 0..3.
constexpr int kGM = 64, kGN = 64, kGK = 32, kGPad = kGM + 1, kGLoads = kGK * kGM / 256;

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<float> {
  using type = f32x4_t;
  static __device__ __forceinline__ type step(float a, float b, type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaAcc<double> {
  using type = f64x4_t;
  static __device__ __forceinline__ type step(double a, double b, type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// K is split over gridDim.z workgroups (enough workgroups to fill the chip
// even for one shape); each writes its partial tile to part[z][row][body],
// summed in a fixed order by body_gemm_reduce_kernel.
template <typename T, bool BORDER>
__global__ void __launch_bounds__(256) body_gemm_kernel(const T* __restrict__ A, int N,
                                                        const int* __restrict__ bodies, int nbt,
                                                        const int64_t* __restrict__ off, int64_t n_bead,
                                                        const double* __restrict__ x, int kspan,
                                                        T* __restrict__ part) {
  using Acc = typename MfmaAcc<T>::type;
  const int Np = BORDER ? N + 1 : N;
  const int kbeg = blockIdx.z * kspan;
  const int kend = min(Np, kbeg + kspan);
  __shared__ T As[kGK][kGPad];   // As[k][row]
  __shared__ T Xs[kGK][kGPad];   // Xs[k][col]
  __shared__ int64_t boff[kGN];
  __shared__ int64_t bpsi[kGN];
  const int row0 = blockIdx.x * kGM;
  const int col0 = blockIdx.y * kGN;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;  // the wavefront's quarter
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
      ra[i] = (gr < Np && gk < kend) ? A[(int64_t)gr * Np + gk] : (T)0;
      T v = 0;
      if (boff[r] >= 0 && gk < kend) v = (T)((!BORDER || gk < N) ? x[boff[r] + gk] : x[bpsi[r]]);
      rx[i] = v;
    }
  };
  Acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Acc{0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
  load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < kGLoads; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int kk = e % kGK, r = e / kGK;
      As[kk][r] = ra[i];
      Xs[kk][r] = rx[i];
    }
    __syncthreads();
    if (k0 + kGK < kend) load(k0 + kGK);
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 4) {
      const T a0 = As[ks + lk][wr + li], a1 = As[ks + lk][wr + 16 + li];
      const T b0 = Xs[ks + lk][wc + li], b1 = Xs[ks + lk][wc + 16 + li];
      acc[0][0] = MfmaAcc<T>::step(a0, b0, acc[0][0]);
      acc[0][1] = MfmaAcc<T>::step(a0, b1, acc[0][1]);
      acc[1][0] = MfmaAcc<T>::step(a1, b0, acc[1][0]);
      acc[1][1] = MfmaAcc<T>::step(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = row0 + wr + 16 * a + (sizeof(T) == 8 ? 4 * i + lk : 4 * lk + i);
        const int cb = col0 + wc + 16 * b + li;
        if (gr >= Np || cb >= nbt) continue;
        part[((int64_t)blockIdx.z * Np + gr) * nbt + cb] = acc[a][b][i];
      }
}

template <typename T, bool BORDER, bool ACCUM>
__global__ void body_gemm_reduce_kernel(const T* __restrict__ part, int nsplit, int N, int nbt,
                                        const int* __restrict__ bodies, const int64_t* __restrict__ off,
                                        int64_t n_bead, double* __restrict__ y) {
  const int Np = BORDER ? N + 1 : N;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)Np * nbt) return;
  const int gr = (int)(e / nbt), cb = (int)(e - (int64_t)gr * nbt);
  double v = 0;
  for (int z = 0; z < nsplit; ++z) v += (double)part[((int64_t)z * Np + gr) * nbt + cb];
  const int body = bodies[cb];
  const int64_t o = (!BORDER || gr < N) ? off[body] + gr : n_bead + body;
  y[o] = ACCUM ? y[o] + v : v;
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

void shape_match_launch(pe_context* c) {
  Precond& pc = c->pc;
  hipStream_t s = c->stream;
  const int64_t nbody = c->n_body;
  if (nbody == 0) return;
  pc.assigned.ensure(nbody);
  pc.dense.ensure(nbody);
  PE_HIP(hipMemsetAsync(pc.assigned.get(), 0xFF, sizeof(int) * nbody, s));  // -1: unassigned
  for (size_t ti = 0; ti < pc.types.size(); ++ti) launch_match(c, pc.types[ti], (int)ti);
  int* asg = pc.h_asg.get<int>(nbody);
  PE_HIP(hipMemcpyAsync(asg, pc.assigned.get(), sizeof(int) * nbody, hipMemcpyDeviceToHost, s));
}

void shape_setup(pe_context* c) {
  Precond& pc = c->pc;
  hipStream_t s = c->stream;
  for (auto& t : pc.types) t.bodies.clear();
  pc.near_beads = 0;
  const int64_t nbody = c->n_body;
  if (nbody == 0) return;
  // the known shapes' matches, launched by shape_match_launch, have reached
  // the host
  int* asg = pc.h_asg.get<int>(nbody);
  auto fetch_assigned = [&]() {
    PE_HIP(hipMemcpyAsync(asg, pc.assigned.get(), sizeof(int) * nbody, hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
  };
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
  pc.near_beads = 0;
  for (auto& t : pc.types)
    if (t.near) pc.near_beads += (int64_t)t.N * (int64_t)t.bodies.size();
  // workspace of the split products (in doubles; float partials use half)
  size_t ws = 1;
  for (auto& t : pc.types)
    if (!t.bodies.empty())
      ws = std::max({ws, body_gemm_workspace(t.N, (int)t.bodies.size(), true),
                     body_gemm_workspace(t.N, (int)t.bodies.size(), false)});
  pc.gemm_ws.ensure(ws);
  // from the kept host copy, which outlives the copy (no wait)
  pc.dense_h = dense;
  PE_HIP(hipMemcpyAsync(pc.dense.get(), pc.dense_h.data(), nbody, hipMemcpyHostToDevice, s));
}

int body_gemm_splits(int N, int nbt, bool bordered) {
  const int Np = bordered ? N + 1 : N;
  const int tiles = ((Np + kGM - 1) / kGM) * ((nbt + kGN - 1) / kGN);
  const int chunks = (Np + kGK - 1) / kGK;
  int z = (1024 + tiles - 1) / tiles;  // aim at about a thousand workgroups
  z = std::min(z, std::max(1, chunks / 2));  // at least two K chunks each
  return std::max(1, std::min(z, 8));
}

size_t body_gemm_workspace(int N, int nbt, bool bordered) {
  const int Np = bordered ? N + 1 : N;
  return (size_t)body_gemm_splits(N, nbt, bordered) * Np * nbt;
}

template <typename T>
void launch_body_gemm(hipStream_t s, const T* A, int N, bool bordered, bool accumulate, const int* bodies,
                      int nbt, const int64_t* off, int64_t n_bead, const double* x, double* y, double* ws) {
  if (nbt == 0 || N == 0) return;
  require(!(bordered && accumulate), "bordered product overwrites");
  const int Np = bordered ? N + 1 : N;
  const int nz = body_gemm_splits(N, nbt, bordered);
  const int chunks = (Np + kGK - 1) / kGK;
  const int kspan = ((chunks + nz - 1) / nz) * kGK;
  T* part = reinterpret_cast<T*>(ws);
  const dim3 grid((unsigned)((Np + kGM - 1) / kGM), (unsigned)((nbt + kGN - 1) / kGN), (unsigned)nz);
  if (bordered)
    hipLaunchKernelGGL((body_gemm_kernel<T, true>), grid, dim3(256), 0, s, A, N, bodies, nbt, off, n_bead, x,
                       kspan, part);
  else
    hipLaunchKernelGGL((body_gemm_kernel<T, false>), grid, dim3(256), 0, s, A, N, bodies, nbt, off, n_bead, x,
                       kspan, part);
  PE_CHECK_LAUNCH();
  const int64_t ne = (int64_t)Np * nbt;
  const dim3 rg((unsigned)((ne + 255) / 256));
  if (bordered)
    hipLaunchKernelGGL((body_gemm_reduce_kernel<T, true, false>), rg, dim3(256), 0, s, part, nz, N, nbt, bodies, off,
                       n_bead, y);
  else if (accumulate)
    hipLaunchKernelGGL((body_gemm_reduce_kernel<T, false, true>), rg, dim3(256), 0, s, part, nz, N, nbt, bodies,
                       off, n_bead, y);
  else
    hipLaunchKernelGGL((body_gemm_reduce_kernel<T, false, false>), rg, dim3(256), 0, s, part, nz, N, nbt, bodies,
                       off, n_bead, y);
  PE_CHECK_LAUNCH();
}

template void launch_body_gemm<float>(hipStream_t, const float*, int, bool, bool, const int*, int, const int64_t*,
                                      int64_t, const double*, double*, double*);
template void launch_body_gemm<double>(hipStream_t, const double*, int, bool, bool, const int*, int, const int64_t*,
                                       int64_t, const double*, double*, double*);

}  // namespace pe
