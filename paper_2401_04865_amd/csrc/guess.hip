// Learned initial guess for the induced bead charges (not in the paper).
//
// Per bead ij the network sees, in the body frame of body i (rotation R_i):
//   f = [R_i^T r_ij (3), R_i^T (E0 + E_ion(x_ij)) (3), one-hot body type (2)]
// and outputs o (4 numbers); the guess is
//   q_hat_ij = o[0:3] . E'_ij + (Q_i / N_i) (1 + o[3]),
// then projected so that each body carries its net charge Q_i.  Layers:
// 8 -> 64 (tanh) -> 64 (tanh) -> 4.  The 64 x 64 layer runs on the matrix
// cores (bf16 operands, fp32 accumulation, v_mfma_f32_16x16x16bf16) in the
// forward pass and in both products of its backward pass; the small first
// and last layers use ordinary FMAs.  Training is full-batch-free minibatch
// Adam on (features, solved charge) pairs recorded from solves of the method
// itself; per-block gradient partials are reduced in a fixed order, so
// training is bitwise reproducible.
//
// MFMA operand layout (16 x 16 x 16, one wavefront): lane l supplies
// A[l % 16][4 (l / 16) + i] and B[4 (l / 16) + i][l % 16], i = 0..3, and
// receives D[4 (l / 16) + i][l % 16].
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "guess.hpp"
#include "pe_internal.hpp"
#include "vector.hpp"

namespace pe {

namespace {

constexpr int kF = 8;      // input features
constexpr int kH = 64;     // hidden width
constexpr int kO = 4;      // outputs
constexpr int kRec = 11;   // recorded floats per bead: f[8], Q_i/N_i, solved q, padding
// parameter offsets
constexpr int oW1 = 0;
constexpr int ob1 = oW1 + kH * kF;
constexpr int oW2 = ob1 + kH;
constexpr int ob2 = oW2 + kH * kH;
constexpr int oW3 = ob2 + kH;
constexpr int ob3 = oW3 + kO * kH;
constexpr int kNPar = ob3 + kO;  // 4996
constexpr int kGroup = 16;       // beads per MFMA group

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Features of every bead: f[8] and Q_i/N_i (9 floats per bead).
__global__ void features_kernel(int64_t n, const double* __restrict__ rel, const double* __restrict__ E_ion,
                                double ex, double ey, double ez, const double* __restrict__ quat,
                                const int* __restrict__ body_of, const int* __restrict__ btype,
                                const double* __restrict__ Q, const int64_t* __restrict__ off,
                                float* __restrict__ feat) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int b = body_of[j];
  const double w = quat[4 * b], x = quat[4 * b + 1], y = quat[4 * b + 2], z = quat[4 * b + 3];
  // R (body -> lab); features use R^T v
  const double R00 = 1 - 2 * (y * y + z * z), R01 = 2 * (x * y - w * z), R02 = 2 * (x * z + w * y);
  const double R10 = 2 * (x * y + w * z), R11 = 1 - 2 * (x * x + z * z), R12 = 2 * (y * z - w * x);
  const double R20 = 2 * (x * z - w * y), R21 = 2 * (y * z + w * x), R22 = 1 - 2 * (x * x + y * y);
  const double rx = rel[3 * j], ry = rel[3 * j + 1], rz = rel[3 * j + 2];
  double Ex = ex, Ey = ey, Ez = ez;
  if (E_ion) {
    Ex += E_ion[3 * j];
    Ey += E_ion[3 * j + 1];
    Ez += E_ion[3 * j + 2];
  }
  float* f = feat + 9 * j;
  f[0] = (float)(R00 * rx + R10 * ry + R20 * rz);
  f[1] = (float)(R01 * rx + R11 * ry + R21 * rz);
  f[2] = (float)(R02 * rx + R12 * ry + R22 * rz);
  f[3] = (float)(R00 * Ex + R10 * Ey + R20 * Ez);
  f[4] = (float)(R01 * Ex + R11 * Ey + R21 * Ez);
  f[5] = (float)(R02 * Ex + R12 * Ey + R22 * Ez);
  const int t = btype ? btype[b] : 0;
  f[6] = t == 0 ? 1.0f : 0.0f;
  f[7] = t == 0 ? 0.0f : 1.0f;
  f[8] = (float)(Q[b] / (double)(off[b + 1] - off[b]));
}

// Forward (and optionally backward) of one group of 16 beads by one
// wavefront.  in: 16 rows of `stride` floats: f[8], qn, target.
// h1 and h2 are overwritten in place by dz1 and dz2 in the backward pass.
struct WaveLDS {
  float h1[kGroup][kH + 1];
  float h2[kGroup][kH + 1];
  float out[kGroup][kO];
  float x[kGroup][kF + 2];
  float dq[kGroup];
};

#define WAVE_SYNC()                                          \
  do {                                                       \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   \
    __builtin_amdgcn_wave_barrier();                         \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");   \
  } while (0)

// layer 1 (FMA), layer 2 (MFMA), layer 3 (FMA); q_hat -> L.dq (temporarily)
__device__ __forceinline__ void forward_group(WaveLDS& L, const float* __restrict__ P, const short* __restrict__ W2b,
                                              int lane) {
  for (int t = lane; t < kGroup * kH; t += 64) {
    const int b = t / kH, o = t % kH;
    float s = P[ob1 + o];
#pragma unroll
    for (int k = 0; k < kF; ++k) s += P[oW1 + o * kF + k] * L.x[b][k];
    L.h1[b][o] = tanhf(s);
  }
  WAVE_SYNC();
  const int r = lane & 15, q4 = (lane >> 4) * 4;
  for (int nt = 0; nt < kH / 16; ++nt) {
    f32x4 acc = {0, 0, 0, 0};
    for (int s = 0; s < kH / 16; ++s) {
      bf16x4 a, b;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = to_bf16(L.h1[r][16 * s + q4 + i]);                  // A[b][k]
        b[i] = W2b[(16 * nt + r) * kH + 16 * s + q4 + i];          // B[k][o] = W2[o][k]
      }
      acc = mfma16(a, b, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 16 * nt + r;
      L.h2[q4 + i][o] = tanhf(acc[i] + P[ob2 + o]);
    }
  }
  WAVE_SYNC();
  {
    const int b = lane >> 2, c = lane & 3;
    float s = P[ob3 + c];
    for (int k = 0; k < kH; ++k) s += P[oW3 + c * kH + k] * L.h2[b][k];
    L.out[b][c] = s;
  }
  WAVE_SYNC();
  if (lane < kGroup) {
    const int b = lane;
    L.dq[b] = L.out[b][0] * L.x[b][3] + L.out[b][1] * L.x[b][4] + L.out[b][2] * L.x[b][5] +
              L.x[b][8] * (1.0f + L.out[b][3]);
  }
  WAVE_SYNC();
}

__global__ void __launch_bounds__(256) predict_kernel(const float* __restrict__ feat, int64_t n,
                                                      const float* __restrict__ P, double* __restrict__ q) {
  __shared__ WaveLDS lds[4];
  __shared__ short W2b[kH * kH];
  for (int t = threadIdx.x; t < kH * kH; t += blockDim.x) W2b[t] = to_bf16(P[oW2 + t]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  WaveLDS& L = lds[wv];
  const int64_t ngroups = (n + kGroup - 1) / kGroup;
  for (int64_t g = (int64_t)blockIdx.x * 4 + wv; g < ngroups; g += (int64_t)gridDim.x * 4) {
    const int64_t g0 = g * kGroup;
    // predict: rows are 9 floats (no target)
    for (int t = lane; t < kGroup * (kF + 2); t += 64) {
      const int b = t / (kF + 2), k = t % (kF + 2);
      const int64_t row = g0 + b;
      L.x[b][k] = (row < n && k < kF + 1) ? feat[row * 9 + k] : 0.0f;
    }
    WAVE_SYNC();
    forward_group(L, P, W2b, lane);
    if (lane < kGroup && g0 + lane < n) q[g0 + lane] = (double)L.dq[lane];
    __builtin_amdgcn_wave_barrier();
  }
}

// One minibatch: rows perm[b0 .. b0+nb) of the dataset.  Every wavefront
// writes its own gradient partial (kNPar floats) and loss partial; they are
// summed in a fixed order by the update kernel.
__global__ void __launch_bounds__(256) train_kernel(const float* __restrict__ data, const int* __restrict__ perm,
                                                    int64_t b0, int64_t nb, const float* __restrict__ P,
                                                    float* __restrict__ gpart, float* __restrict__ lpart) {
  __shared__ WaveLDS lds[4];
  __shared__ short W2b[kH * kH];
  for (int t = threadIdx.x; t < kH * kH; t += blockDim.x) W2b[t] = to_bf16(P[oW2 + t]);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  WaveLDS& L = lds[wv];
  const int r = lane & 15, q4 = (lane >> 4) * 4;
  const int c3 = lane & 3, kq = lane >> 2;   // dW3 ownership: c = lane & 3, k = 4 kq + kk
  f32x4 accW2[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nn = 0; nn < 4; ++nn) accW2[m][nn] = f32x4{0, 0, 0, 0};
  float gW1[kF] = {0, 0, 0, 0, 0, 0, 0, 0};
  float gb1 = 0, gb2 = 0, gb3 = 0;
  float gW3[4] = {0, 0, 0, 0};
  float loss = 0;
  const float inv_nb = 1.0f / (float)nb;
  const int64_t ngroups = (nb + kGroup - 1) / kGroup;
  for (int64_t g = (int64_t)blockIdx.x * 4 + wv; g < ngroups; g += (int64_t)gridDim.x * 4) {
    const int64_t g0 = g * kGroup;
    for (int t = lane; t < kGroup * (kF + 2); t += 64) {
      const int b = t / (kF + 2), k = t % (kF + 2);
      const int64_t row = g0 + b;
      L.x[b][k] = row < nb ? data[(int64_t)perm[b0 + row] * kRec + k] : 0.0f;
    }
    WAVE_SYNC();
    forward_group(L, P, W2b, lane);
    // dq = 2 (q_hat - target) / nb ; rows beyond the batch contribute nothing
    if (lane < kGroup) {
      const int64_t row = g0 + lane;
      float d = 0;
      if (row < nb) {
        const float e = L.dq[lane] - L.x[lane][kF + 1];
        loss += e * e;
        d = 2.0f * e * inv_nb;
      }
      L.dq[lane] = d;
    }
    WAVE_SYNC();
    // d out[b] = dq[b] [E'x, E'y, E'z, qn];  dW3, db3
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = kq * 4 + kk;
      float sacc = 0;
      for (int b = 0; b < kGroup; ++b) sacc += L.dq[b] * (c3 < 3 ? L.x[b][3 + c3] : L.x[b][8]) * L.h2[b][k];
      gW3[kk] += sacc;
    }
    if (lane < kO) {
      float sacc = 0;
      for (int b = 0; b < kGroup; ++b) sacc += L.dq[b] * (lane < 3 ? L.x[b][3 + lane] : L.x[b][8]);
      gb3 += sacc;
    }
    WAVE_SYNC();
    // dz2[b][k] = (sum_c W3[c][k] dout[b][c]) (1 - h2^2), in place of h2
    for (int t = lane; t < kGroup * kH; t += 64) {
      const int b = t / kH, k = t % kH;
      float sacc = 0;
#pragma unroll
      for (int c = 0; c < kO; ++c) sacc += P[oW3 + c * kH + k] * (c < 3 ? L.x[b][3 + c] : L.x[b][8]);
      const float h = L.h2[b][k];
      L.h2[b][k] = L.dq[b] * sacc * (1.0f - h * h);
    }
    WAVE_SYNC();
    {
      float sacc = 0;
      for (int b = 0; b < kGroup; ++b) sacc += L.h2[b][lane];
      gb2 += sacc;
    }
    // dW2 += dz2^T h1 (A = dz2^T: o x b, B = h1: b x k; K = the 16 beads)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      bf16x4 a;
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = to_bf16(L.h2[q4 + i][16 * m + r]);
#pragma unroll
      for (int nn = 0; nn < 4; ++nn) {
        bf16x4 b;
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = to_bf16(L.h1[q4 + i][16 * nn + r]);
        accW2[m][nn] = mfma16(a, b, accW2[m][nn]);
      }
    }
    // dh1 = dz2 W2 (A = dz2: b x o, B = W2: o x k)
    f32x4 dh1[4];
#pragma unroll
    for (int nn = 0; nn < 4; ++nn) {
      dh1[nn] = f32x4{0, 0, 0, 0};
      for (int s = 0; s < kH / 16; ++s) {
        bf16x4 a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = to_bf16(L.h2[r][16 * s + q4 + i]);
          b[i] = W2b[(16 * s + q4 + i) * kH + 16 * nn + r];
        }
        dh1[nn] = mfma16(a, b, dh1[nn]);
      }
    }
    WAVE_SYNC();
    // dz1 = dh1 (1 - h1^2), in place of h1
#pragma unroll
    for (int nn = 0; nn < 4; ++nn)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int b = q4 + i, k = 16 * nn + r;
        const float h = L.h1[b][k];
        L.h1[b][k] = dh1[nn][i] * (1.0f - h * h);
      }
    WAVE_SYNC();
    // dW1[o][k] += sum_b dz1[b][o] x[b][k]; db1[o] += sum_b dz1[b][o]   (o = lane)
    for (int b = 0; b < kGroup; ++b) {
      const float dz = L.h1[b][lane];
      gb1 += dz;
#pragma unroll
      for (int k = 0; k < kF; ++k) gW1[k] += dz * L.x[b][k];
    }
    WAVE_SYNC();
  }
  float* out = gpart + ((int64_t)blockIdx.x * 4 + wv) * kNPar;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nn = 0; nn < 4; ++nn)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[oW2 + (16 * m + q4 + i) * kH + 16 * nn + r] = accW2[m][nn][i];
#pragma unroll
  for (int k = 0; k < kF; ++k) out[oW1 + lane * kF + k] = gW1[k];
  out[ob1 + lane] = gb1;
  out[ob2 + lane] = gb2;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) out[oW3 + c3 * kH + kq * 4 + kk] = gW3[kk];
  if (lane < kO) out[ob3 + lane] = gb3;
  float lsum = loss;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
  if (lane == 0) lpart[blockIdx.x * 4 + wv] = lsum;
}

// g = sum over blocks (fixed order); Adam update of the fp32 master weights.
__global__ void adam_kernel(const float* __restrict__ gpart, int nblk, float* __restrict__ P, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2,
                            float* __restrict__ gout) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNPar) return;
  float g = 0;
  for (int b = 0; b < nblk; ++b) g += gpart[(int64_t)b * kNPar + p];
  if (gout) gout[p] = g;
  if (lr == 0.0f) return;
  const float mm = b1 * m[p] + (1 - b1) * g;
  const float vv = b2 * v[p] + (1 - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void append_kernel(const float* __restrict__ feat, const double* __restrict__ q, int64_t n,
                              float* __restrict__ data, int64_t at) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float* row = data + (at + j) * kRec;
  for (int k = 0; k < 9; ++k) row[k] = feat[9 * j + k];
  row[9] = (float)q[j];
  row[10] = 0.0f;
}

// q += (Q_b - sum_j q_j) / N_b on every bead of body b
__global__ void project_kernel(const int64_t* __restrict__ off, const double* __restrict__ Q,
                               const double* __restrict__ sums, const int* __restrict__ body_of, int64_t n,
                               double* __restrict__ q) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int b = body_of[j];
  q[j] += (Q[b] - sums[b]) / (double)(off[b + 1] - off[b]);
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

struct LearnedGuess {
  DevBuf<float> P, m, v, gpart, lpart, gout;
  DevBuf<float> feat;   // current system, 9 per bead
  DevBuf<float> data;   // recorded rows
  DevBuf<int> perm;
  int64_t n_rec = 0;
  int64_t adam_t = 0;
  bool init = false;
  std::vector<int> types;
};

namespace {

void ensure_data(LearnedGuess* gs, int64_t rows) {
  if ((size_t)rows * kRec <= gs->data.cap) return;
  size_t cap = std::max<size_t>((size_t)rows * kRec, 2 * gs->data.cap);
  DevBuf<float> nd;
  nd.ensure(cap);
  if (gs->n_rec) PE_HIP(hipMemcpy(nd.get(), gs->data.get(), sizeof(float) * gs->n_rec * kRec, hipMemcpyDeviceToDevice));
  nd.swap(gs->data);
}

LearnedGuess* get(pe_context* c) {
  if (!c->guess) c->guess = new LearnedGuess();
  return c->guess;
}

void compute_features(pe_context* c) {
  LearnedGuess* g = get(c);
  const int64_t n = c->n_bead;
  g->feat.ensure(9 * std::max<int64_t>(n, 1));
  if (!c->have_eion) throw Error(PE_ERR_STATE, "ion field at the beads not available (run a solve first)");
  if (!g->types.empty()) {
    require((int64_t)g->types.size() == c->n_body, "body types do not match the system");
    c->body_type.ensure(c->n_body);
    PE_HIP(hipMemcpyAsync(c->body_type.get(), g->types.data(), sizeof(int) * c->n_body, hipMemcpyHostToDevice,
                          c->stream));
  }
  if (n)
    hipLaunchKernelGGL(features_kernel, dim3(nblk(n, 256)), dim3(256), 0, c->stream, n, c->rel.get(),
                       c->n_ion ? c->E_ion.get() : (const double*)nullptr, c->E0[0], c->E0[1], c->E0[2],
                       c->quat.get(), c->body_of.get(), g->types.empty() ? (const int*)nullptr : c->body_type.get(),
                       c->body_Q.get(), c->off.get(), g->feat.get());
  PE_CHECK_LAUNCH();
}

void init_weights(LearnedGuess* g, uint64_t seed, hipStream_t s) {
  std::mt19937_64 rng(seed);
  std::vector<float> P(kNPar, 0.0f);
  auto uni = [&](float a) { return (float)((double)(rng() >> 11) / 9007199254740992.0 * 2.0 - 1.0) * a; };
  const float a1 = std::sqrt(6.0f / (kF + kH)), a2 = std::sqrt(6.0f / (kH + kH)), a3 = 0.1f * std::sqrt(6.0f / (kH + kO));
  for (int i = 0; i < kH * kF; ++i) P[oW1 + i] = uni(a1);
  for (int i = 0; i < kH * kH; ++i) P[oW2 + i] = uni(a2);
  for (int i = 0; i < kO * kH; ++i) P[oW3 + i] = uni(a3);
  g->P.ensure(kNPar);
  g->m.ensure(kNPar);
  g->v.ensure(kNPar);
  PE_HIP(hipMemcpyAsync(g->P.get(), P.data(), sizeof(float) * kNPar, hipMemcpyHostToDevice, s));
  PE_HIP(hipMemsetAsync(g->m.get(), 0, sizeof(float) * kNPar, s));
  PE_HIP(hipMemsetAsync(g->v.get(), 0, sizeof(float) * kNPar, s));
  PE_HIP(hipStreamSynchronize(s));
  g->adam_t = 0;
  g->init = true;
}

}  // namespace

void guess_destroy(pe_context* c) {
  delete c->guess;
  c->guess = nullptr;
}

void guess_on_system(pe_context*) {}

bool guess_ready(const pe_context* c) { return c->guess && c->guess->init; }

void guess_predict(pe_context* c, double* x) {
  LearnedGuess* g = get(c);
  if (!g->init) throw Error(PE_ERR_STATE, "learned guess has no weights (pe_guess_init or pe_guess_load)");
  compute_features(c);
  const int64_t n = c->n_bead;
  if (n == 0) return;
  const int64_t ngroups = (n + kGroup - 1) / kGroup;
  unsigned nb = (unsigned)std::min<int64_t>((ngroups + 3) / 4, 2048);
  hipLaunchKernelGGL(predict_kernel, dim3(nb), dim3(256), 0, c->stream, g->feat.get(), n, g->P.get(), x);
  PE_CHECK_LAUNCH();
  c->sums.ensure(64 + c->n_body);
  double* bs = c->sums.get() + 64;
  launch_seg_sum(c->stream, c->off.get(), c->n_body, x, bs);
  hipLaunchKernelGGL(project_kernel, dim3(nblk(n, 256)), dim3(256), 0, c->stream, c->off.get(), c->body_Q.get(), bs,
                     c->body_of.get(), n, x);
  PE_CHECK_LAUNCH();
}

// Gradient of the minibatch loss (test hook): g[kNPar] for rows 0..nb-1 in order.
void guess_gradient(pe_context* c, int64_t nb, float* host_grad, double* host_loss) {
  LearnedGuess* g = get(c);
  std::vector<int> perm(nb);
  for (int64_t i = 0; i < nb; ++i) perm[i] = (int)i;
  g->perm.ensure(std::max<int64_t>(nb, 1));
  PE_HIP(hipMemcpy(g->perm.get(), perm.data(), sizeof(int) * nb, hipMemcpyHostToDevice));
  const int64_t ngroups = (nb + kGroup - 1) / kGroup;
  const int blocks = (int)std::min<int64_t>((ngroups + 3) / 4, 256);
  g->gpart.ensure((size_t)blocks * 4 * kNPar);
  g->lpart.ensure(blocks * 4);
  g->gout.ensure(kNPar);
  hipLaunchKernelGGL(train_kernel, dim3(blocks), dim3(256), 0, c->stream, g->data.get(), g->perm.get(), (int64_t)0,
                     nb, g->P.get(), g->gpart.get(), g->lpart.get());
  hipLaunchKernelGGL(adam_kernel, dim3((kNPar + 255) / 256), dim3(256), 0, c->stream, g->gpart.get(), blocks * 4,
                     g->P.get(), g->m.get(), g->v.get(), 0.0f, 0.9f, 0.999f, 1e-8f, 1.0f, 1.0f, g->gout.get());
  PE_CHECK_LAUNCH();
  std::vector<float> lp(blocks * 4);
  PE_HIP(hipMemcpy(host_grad, g->gout.get(), sizeof(float) * kNPar, hipMemcpyDeviceToHost));
  PE_HIP(hipMemcpy(lp.data(), g->lpart.get(), sizeof(float) * blocks * 4, hipMemcpyDeviceToHost));
  double L = 0;
  for (float v : lp) L += v;
  *host_loss = L / (double)nb;
}

}  // namespace pe

using namespace pe;

#define PE_API_BEGIN(ctx) ::pe::ArenaScope arena_scope_((ctx) ? &(ctx)->arena : nullptr); try {
#define PE_API_END(ctx)                 \
  }                                     \
  catch (const pe::Error& e) {          \
    (ctx)->err = e.what();              \
    return e.code;                      \
  }                                     \
  catch (const std::exception& e) {     \
    (ctx)->err = e.what();              \
    return PE_ERR_DEVICE;               \
  }                                     \
  return PE_OK;

extern "C" {

pe_status pe_guess_init(pe_context* c, uint64_t seed) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  init_weights(get(c), seed, c->stream);
  PE_API_END(c)
}

pe_status pe_guess_set_types(pe_context* c, const int32_t* body_type) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  if (!c->have_system) throw Error(PE_ERR_STATE, "pe_set_system has not been called");
  LearnedGuess* g = get(c);
  g->types.assign(body_type, body_type + c->n_body);
  for (int t : g->types) require(t == 0 || t == 1, "body types must be 0 or 1");
  PE_API_END(c)
}

pe_status pe_guess_record(pe_context* c, const double* q_solved) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  if (!c->have_solution) throw Error(PE_ERR_STATE, "pe_solve_polarization has not been called");
  require(q_solved != nullptr, "null charges");
  LearnedGuess* g = get(c);
  compute_features(c);
  const int64_t n = c->n_bead;
  ensure_data(g, g->n_rec + n);
  if (n)
    hipLaunchKernelGGL(append_kernel, dim3(nblk(n, 256)), dim3(256), 0, c->stream, g->feat.get(), q_solved, n,
                       g->data.get(), g->n_rec);
  PE_CHECK_LAUNCH();
  PE_HIP(hipStreamSynchronize(c->stream));
  g->n_rec += n;
  PE_API_END(c)
}

pe_status pe_guess_clear(pe_context* c) {
  if (!c) return PE_ERR_ARG;
  if (c->guess) c->guess->n_rec = 0;
  return PE_OK;
}

pe_status pe_guess_train(pe_context* c, int32_t epochs, int32_t batch, double lr, uint64_t seed, double* loss) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  LearnedGuess* g = get(c);
  require(g->init, "pe_guess_init or pe_guess_load first");
  require(g->n_rec > 0, "no recorded samples");
  require(epochs >= 0 && batch >= 16 && lr > 0, "bad training arguments");
  hipStream_t s = c->stream;
  const int64_t N = g->n_rec;
  std::mt19937_64 rng(seed);
  std::vector<int> perm(N);
  g->perm.ensure(N);
  const int64_t ngroups_max = ((int64_t)batch + kGroup - 1) / kGroup;
  const int blocks = (int)std::min<int64_t>((ngroups_max + 3) / 4, 256);
  g->gpart.ensure((size_t)blocks * 4 * kNPar);
  g->lpart.ensure(blocks * 4);
  double last = 0;
  std::vector<float> lp(blocks * 4);
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < N; ++i) perm[i] = (int)i;
    std::shuffle(perm.begin(), perm.end(), rng);
    PE_HIP(hipMemcpyAsync(g->perm.get(), perm.data(), sizeof(int) * N, hipMemcpyHostToDevice, s));
    double ep_loss = 0;
    int64_t ep_rows = 0;
    for (int64_t b0 = 0; b0 < N; b0 += batch) {
      const int64_t nb = std::min<int64_t>(batch, N - b0);
      hipLaunchKernelGGL(train_kernel, dim3(blocks), dim3(256), 0, s, g->data.get(), g->perm.get(), b0, nb,
                         g->P.get(), g->gpart.get(), g->lpart.get());
      g->adam_t += 1;
      const float c1 = 1.0f - (float)std::pow(0.9, (double)g->adam_t);
      const float c2 = 1.0f - (float)std::pow(0.999, (double)g->adam_t);
      hipLaunchKernelGGL(adam_kernel, dim3((kNPar + 255) / 256), dim3(256), 0, s, g->gpart.get(), blocks * 4,
                         g->P.get(), g->m.get(), g->v.get(), (float)lr, 0.9f, 0.999f, 1e-8f, c1, c2,
                         (float*)nullptr);
      PE_CHECK_LAUNCH();
      if (ep == epochs - 1) {
        PE_HIP(hipMemcpyAsync(lp.data(), g->lpart.get(), sizeof(float) * blocks * 4, hipMemcpyDeviceToHost, s));
        PE_HIP(hipStreamSynchronize(s));
        for (float v : lp) ep_loss += v;
        ep_rows += nb;
      }
    }
    if (ep == epochs - 1) last = ep_loss / (double)std::max<int64_t>(ep_rows, 1);
  }
  PE_HIP(hipStreamSynchronize(s));
  if (loss) *loss = last;
  PE_API_END(c)
}

pe_status pe_guess_predict(pe_context* c, double* q_out) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  if (!c->have_system) throw Error(PE_ERR_STATE, "pe_set_system has not been called");
  require(q_out != nullptr, "null output");
  guess_predict(c, q_out);
  PE_HIP(hipStreamSynchronize(c->stream));
  PE_API_END(c)
}

pe_status pe_guess_save(const pe_context* cc, const char* path) {
  pe_context* c = const_cast<pe_context*>(cc);
  if (!c || !path) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  require(c->guess && c->guess->init, "no weights to save");
  std::vector<float> P(kNPar);
  PE_HIP(hipMemcpy(P.data(), c->guess->P.get(), sizeof(float) * kNPar, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  require(f != nullptr, std::string("cannot open ") + path);
  const char magic[8] = {'P', 'E', 'G', 'U', 'E', 'S', 'S', '1'};
  const int32_t hdr[4] = {kF, kH, kO, kNPar};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 4, f) == 4 &&
            std::fwrite(P.data(), sizeof(float), kNPar, f) == (size_t)kNPar;
  std::fclose(f);
  require(ok, "write failed");
  PE_API_END(c)
}

pe_status pe_guess_load(pe_context* c, const char* path) {
  if (!c || !path) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  FILE* f = std::fopen(path, "rb");
  require(f != nullptr, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[4];
  std::vector<float> P(kNPar);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "PEGUESS1", 8) == 0 &&
            std::fread(hdr, sizeof(int32_t), 4, f) == 4 && hdr[0] == kF && hdr[1] == kH && hdr[2] == kO &&
            hdr[3] == kNPar && std::fread(P.data(), sizeof(float), kNPar, f) == (size_t)kNPar;
  std::fclose(f);
  require(ok, "not a learned-guess weight file of this architecture");
  for (float v : P) require(std::isfinite(v), "weight file holds non-finite values");
  LearnedGuess* g = get(c);
  init_weights(g, 0, c->stream);
  PE_HIP(hipMemcpy(g->P.get(), P.data(), sizeof(float) * kNPar, hipMemcpyHostToDevice));
  PE_API_END(c)
}

// Test hook: parameters (host, kNPar floats) in/out and the gradient of the
// mean-squared loss over the first n recorded rows, in row order.
pe_status pe_guess_debug(pe_context* c, float* params_inout, int32_t set_params, int64_t n_rows, float* grad,
                         double* loss) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  LearnedGuess* g = get(c);
  if (!g->init) init_weights(g, 0, c->stream);
  if (set_params) PE_HIP(hipMemcpy(g->P.get(), params_inout, sizeof(float) * kNPar, hipMemcpyHostToDevice));
  else PE_HIP(hipMemcpy(params_inout, g->P.get(), sizeof(float) * kNPar, hipMemcpyDeviceToHost));
  if (n_rows > 0) {
    require(n_rows <= g->n_rec, "not enough recorded rows");
    guess_gradient(c, n_rows, grad, loss);
  }
  PE_API_END(c)
}

pe_status pe_guess_add_rows(pe_context* c, const float* rows, int64_t n_rows) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  require(rows != nullptr && n_rows >= 0, "bad rows");
  LearnedGuess* g = get(c);
  ensure_data(g, g->n_rec + n_rows);
  if (n_rows)
    PE_HIP(hipMemcpy(g->data.get() + g->n_rec * kRec, rows, sizeof(float) * kRec * n_rows, hipMemcpyHostToDevice));
  g->n_rec += n_rows;
  PE_API_END(c)
}

pe_status pe_guess_rows(pe_context* c, float* rows, int64_t n_rows) {
  if (!c) return PE_ERR_ARG;
  PE_API_BEGIN(c)
  LearnedGuess* g = get(c);
  require(n_rows <= g->n_rec, "not enough recorded rows");
  PE_HIP(hipMemcpy(rows, g->data.get(), sizeof(float) * kRec * n_rows, hipMemcpyDeviceToHost));
  PE_API_END(c)
}

}  // extern "C"
