// Hand-written 3-D FFT with the Green's-function scaling fused in (section
// "Spectral Ewald implementation", steps 3-5).
//
// Layout: real grids [Nx][Ny][Nz] (z fastest); the half spectrum
// [Nx][Ny][Nzs], Nzc = Nz/2 + 1 values used per row and the row stride Nzs
// rounded up to a multiple of 16, so the strided passes read every group of
// 16 lines as whole 128-byte segments (with Nzc odd, rows of Nzc values would
// start at every alignment and each group would touch two segments).  Five
// passes, each one read and one write of the grid through LDS:
//   1. z, real -> complex: two real lines packed into one complex line, one
//      complex FFT, then split (X_a = (Z_k + conj Z_{N-k})/2,
//      X_b = (Z_k - conj Z_{N-k})/2i).
//   2. y, complex, forward.
//   3. x forward, multiply by G_k / (Nx Ny Nz), x inverse: the whole x line
//      stays in LDS, so scaling and both x transforms cost one pass.
//   4. y, complex, inverse.
//   5. z, complex -> real (mirror of 1).
// Each 1-D transform is a Stockham autosort FFT in LDS (ping-pong buffers)
// with radices 8, 4, 2, 3, 5 and a twiddle table computed on the host in
// double.  A block transforms several lines at once; lines of the strided
// passes are taken along the contiguous kz / (y,kz) index so global loads
// and stores are coalesced.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pe_internal.hpp"

namespace pe {

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };

namespace {

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return {a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return {a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// multiply by -i*s (s = +1 forward: -i; s = -1 inverse: +i)
template <typename C>
__device__ __forceinline__ C mul_mi(C a, int s) { return s > 0 ? C{a.y, -a.x} : C{-a.y, a.x}; }

// In-register DFT of size R; fwd = +1 for exp(-2 pi i ...), -1 for inverse.
template <typename T, typename C>
__device__ __forceinline__ void dft2(C& a, C& b) {
  C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <typename T, typename C>
__device__ __forceinline__ void dft4(C& v0, C& v1, C& v2, C& v3, int fwd) {
  C t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_mi(csub(v1, v3), fwd);
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}

// In-register DFT of compile-time size R.
template <typename T, typename C, int R>
__device__ __forceinline__ void butterfly(C (&v)[R], int fwd) {
  const T r2 = (T)0.70710678118654752440;
  if constexpr (R == 2) {
    dft2<T, C>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<T, C>(v[0], v[1], v[2], v[3], fwd);
  } else if constexpr (R == 8) {
    // even / odd halves, then combine with W8^k
    dft4<T, C>(v[0], v[2], v[4], v[6], fwd);
    dft4<T, C>(v[1], v[3], v[5], v[7], fwd);
    // W8^1 = (1 - i fwd)/sqrt2, W8^2 = -i fwd, W8^3 = (-1 - i fwd)/sqrt2
    C o1 = v[3], o2 = v[5], o3 = v[7];
    C w1 = {r2, -r2 * (T)fwd};
    C w3 = {-r2, -r2 * (T)fwd};
    o1 = cmul(o1, w1);
    o2 = mul_mi(o2, fwd);
    o3 = cmul(o3, w3);
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
  } else if constexpr (R == 3) {
    const T s3 = (T)0.86602540378443864676 * (T)fwd;
    C t = cadd(v[1], v[2]);
    C u = csub(v[1], v[2]);
    C a = {v[0].x - (T)0.5 * t.x, v[0].y - (T)0.5 * t.y};
    // X1 = a - i s3 u, X2 = a + i s3 u
    C iu = {-s3 * u.y, s3 * u.x};  // i*s3*u
    v[0] = cadd(v[0], t);
    v[1] = csub(a, iu);
    v[2] = cadd(a, iu);
  } else if constexpr (R == 5) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212 * (T)fwd, s2 = (T)0.58778525229247312917 * (T)fwd;
    C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    C x0 = cadd(v[0], cadd(a1, a2));
    C p1 = {v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    C p2 = {v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    // -i * (s1 b1 + s2 b2) and -i * (s2 b1 - s1 b2)
    C q1 = {s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
    C q2 = {s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
    C mq1 = {q1.y, -q1.x}, mq2 = {q2.y, -q2.x};
    v[0] = x0;
    v[1] = cadd(p1, mq1);
    v[4] = csub(p1, mq1);
    v[2] = cadd(p2, mq2);
    v[3] = csub(p2, mq2);
  }
}

// Position of element j of line `line` in an LDS buffer: lines `ls` apart,
// and the low bits of j XORed with the line number (a bijection within each
// line when n is a multiple of smask + 1), so that reading one element of
// many lines at once, as the strided passes do, hits different banks even
// without padding the lines.
struct LdsLayout {
  int ls;
  int smask;
  __device__ __forceinline__ int at(int line, int j) const { return line * ls + (j ^ (line & smask)); }
};

// One Stockham stage of radix R over nl lines of length n.  When n is a
// power of two (so are nb = n / R and Ns), the index splits use shifts and
// masks instead of integer division.
template <typename T, typename C, int R>
__device__ __forceinline__ void stockham_stage(const C* __restrict__ in, C* __restrict__ out, int n, int nl,
                                               LdsLayout L, int Ns, const C* __restrict__ tw, int fwd) {
  const int nb = n / R;
  const int tws = n / (Ns * R);
  const bool pow2 = (n & (n - 1)) == 0;
  const int lnb = pow2 ? __builtin_ctz(nb) : 0;
  const int lns = pow2 ? __builtin_ctz(Ns) : 0;
  for (int t = threadIdx.x; t < nl * nb; t += blockDim.x) {
    int line, j, k, jq;
    if (pow2) {
      line = t >> lnb;
      j = t & (nb - 1);
      k = j & (Ns - 1);
      jq = j >> lns;
    } else {
      line = t / nb;
      j = t - line * nb;
      jq = j / Ns;
      k = j - jq * Ns;
    }
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[L.at(line, j + r * nb)];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tw[r * k * tws];
        if (fwd < 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    butterfly<T, C, R>(v, fwd);
    const int base = jq * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[L.at(line, base + r * Ns)] = v[r];
  }
}

// Transform `nl` lines of length n held in LDS (`in`, layout L).
// Returns the buffer that holds the result (in or out).
template <typename T, typename C>
__device__ C* lds_fft(C* in, C* out, int n, int nl, LdsLayout ls, const FFTPlan1D& plan,
                      const C* __restrict__ tw, int fwd) {
  int Ns = 1;
  for (int s = 0; s < plan.nstage; ++s) {
    const int R = plan.radix[s];
    switch (R) {
      case 8: stockham_stage<T, C, 8>(in, out, n, nl, ls, Ns, tw, fwd); break;
      case 4: stockham_stage<T, C, 4>(in, out, n, nl, ls, Ns, tw, fwd); break;
      case 2: stockham_stage<T, C, 2>(in, out, n, nl, ls, Ns, tw, fwd); break;
      case 3: stockham_stage<T, C, 3>(in, out, n, nl, ls, Ns, tw, fwd); break;
      default: stockham_stage<T, C, 5>(in, out, n, nl, ls, Ns, tw, fwd); break;
    }
    __syncthreads();
    C* tmp = in;
    in = out;
    out = tmp;
    Ns *= R;
  }
  return in;
}

// Green's function of the wave-space part, with the inverse-DFT
// normalization, in separable form: G = ex[x] ey[y] ez[z] / (kx^2 + ky^2 + kz^2)
// with e_d = exp(-(1 - eta) k_d^2 / (4 xi^2)) tabulated per axis on the host.
struct ScaleArgs {
  int Nx, Ny, Nz, Nzc, Nzs;
  const double* ex;   // Nx
  const double* ey;   // Ny
  const double* ez;   // Nzc
  const double* kx2;  // Nx
  const double* ky2;  // Ny
  const double* kz2;  // Nzc
  double norm;        // 1 / (Nx Ny Nz)
  double shell_a;     // > 0: the Green's function also carries j0^2(|k| a) (the paper's shell split)
};

// j0(|k| a)^2 from k^2 (the paper's split puts the shells' form factor in the
// wave space too); below |k| a = 1e-3 the series 1 - x^2/3.
template <typename T>
__device__ __forceinline__ T j0_squared(T k2, T a) {
  const T x = sqrt(k2) * a;
  if (x < (T)1e-3) return (T)1 - x * x / (T)3;
  const T j = sin(x) / x;
  return j * j;
}

// Lines along a strided axis: line L (0..nlines-1), element j at
// base(L) + j*stride, base(L) = (L / inner) * outer + (L % inner); a line
// with L % vmod >= vlim is row padding and is skipped.
template <typename T, bool SCALE>
__global__ void __launch_bounds__(512) fft_lines_kernel(typename C2<T>::type* __restrict__ data, int n,
                                                        int64_t nlines, int64_t inner, int64_t outer,
                                                        int64_t stride, int vmod, int vlim, int lpb,
                                                        FFTPlan1D plan,
                                                        const typename C2<T>::type* __restrict__ tw,
                                                        int fwd, ScaleArgs sa) {
  using C = typename C2<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int64_t lbase[64];
  __shared__ T lfac[64], lksq[64];
  C* b0 = reinterpret_cast<C*>(smem_raw);
  const LdsLayout ll{n, (n % 16 == 0) ? 15 : ((n % 8 == 0) ? 7 : ((n % 4 == 0) ? 3 : ((n % 2 == 0) ? 1 : 0)))};
  C* b1 = b0 + lpb * n;
  const int64_t L0 = (int64_t)blockIdx.x * lpb;
  if ((int)threadIdx.x < lpb) {
    const int64_t L = L0 + threadIdx.x;
    const bool valid = L < nlines && (int)(L % vmod) < vlim;
    lbase[threadIdx.x] = valid ? (L / inner) * outer + (L % inner) : -1;
    if (SCALE && valid) {
      // x lines: L = y * Nzs + kz
      const int y = (int)(L / sa.Nzs);
      const int kz = (int)(L - (int64_t)y * sa.Nzs);
      lfac[threadIdx.x] = (T)(sa.ey[y] * sa.ez[kz] * sa.norm);
      lksq[threadIdx.x] = (T)(sa.ky2[y] + sa.kz2[kz]);
    }
  }
  __syncthreads();
  const int llpb = __builtin_ctz(lpb);  // lpb is a power of two
  for (int t = threadIdx.x; t < n * lpb; t += blockDim.x) {
    const int j = t >> llpb;
    const int c = t & (lpb - 1);
    C v = {0, 0};
    const int64_t lb = lbase[c];
    if (lb >= 0) v = data[lb + (int64_t)j * stride];
    b0[ll.at(c, j)] = v;
  }
  __syncthreads();
  C* res = lds_fft<T, C>(b0, b1, n, lpb, ll, plan, tw, fwd);
  if (SCALE) {
    for (int t = threadIdx.x; t < n * lpb; t += blockDim.x) {
      const int c = t / n;
      const int j = t - c * n;
      if (lbase[c] < 0) continue;
      const T k2 = (T)sa.kx2[j] + lksq[c];
      T gk = k2 > (T)0 ? (T)sa.ex[j] * lfac[c] / k2 : (T)0;
      if (sa.shell_a > 0.0) gk *= j0_squared<T>(k2, (T)sa.shell_a);
      C v = res[ll.at(c, j)];
      res[ll.at(c, j)] = {v.x * gk, v.y * gk};
    }
    __syncthreads();
    C* other = (res == b0) ? b1 : b0;
    res = lds_fft<T, C>(res, other, n, lpb, ll, plan, tw, -fwd);
  }
  for (int t = threadIdx.x; t < n * lpb; t += blockDim.x) {
    const int j = t >> llpb;
    const int c = t & (lpb - 1);
    const int64_t lb = lbase[c];
    if (lb >= 0) data[lb + (int64_t)j * stride] = res[ll.at(c, j)];
  }
}

// ------------------------------------------------------- 256-point lines
//
// Strided passes of length 256 as two 16-point stages (256 = 16 x 16, the
// four-step form of the DFT): with j = 16 j1 + j2 and k = k1 + 16 k2,
//   X[k1 + 16 k2] = sum_j2 W16^(j2 k2) W256^(j2 k1) sum_j1 x[16 j1 + j2] W16^(j1 k1).
// A block takes 16 lines; thread (c, g) = (t mod 16, t / 16) loads the 16
// values x[16 j1 + g] of line c straight from HBM (16 neighbouring lines per
// 128-byte segment), does the inner 16-point DFT and the twiddle in
// registers, and writes through LDS once; then thread (c, g) reads the 16
// values of k1 = g and does the outer DFT, and stores X[g + 16 k2].  The
// 16-point DFT is itself 4 x 4 in registers.  One LDS exchange and one
// barrier per transform, against one per radix stage in the Stockham form.
// With SCALE the x pass scales X in registers and runs the inverse the same
// way (inner DFT over k2 in registers, exchange, outer over k1).

constexpr int kF16Lines = 16;
constexpr int kF16Ld = 260;  // LDS values per k1 row (256 + 4: successive rows start in other banks)

template <typename T>
__device__ __forceinline__ T cos16(int m) {
  constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                            -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                            0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  return (T)c[m & 15];
}
template <typename T>
__device__ __forceinline__ T sin16(int m) { return cos16<T>(m + 12); }  // sin(x) = cos(x - pi/2)

// v <- 16-point DFT of v (natural order in and out), sign fwd.
template <typename T, typename C>
__device__ __forceinline__ void dft16(C (&v)[16], int fwd) {
  C u[16];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    C t[4] = {v[b], v[4 + b], v[8 + b], v[12 + b]};
    dft4<T, C>(t[0], t[1], t[2], t[3], fwd);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int m = b * c;
      if (m == 0) {
        u[4 * b + c] = t[c];
      } else {
        const C w = {cos16<T>(m), -(T)fwd * sin16<T>(m)};
        u[4 * b + c] = cmul(t[c], w);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    C t[4] = {u[c], u[4 + c], u[8 + c], u[12 + c]};
    dft4<T, C>(t[0], t[1], t[2], t[3], fwd);
    v[c] = t[0];
    v[c + 4] = t[1];
    v[c + 8] = t[2];
    v[c + 12] = t[3];
  }
}

template <typename T, bool SCALE>
__global__ void __launch_bounds__(256) fft256_lines_kernel(typename C2<T>::type* __restrict__ data, int64_t nlines,
                                                           int64_t inner, int64_t outer, int64_t stride, int vmod,
                                                           int vlim, const typename C2<T>::type* __restrict__ tw,
                                                           int fwd, ScaleArgs sa) {
  using C = typename C2<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* X = reinterpret_cast<C*>(smem_raw);  // [16 rows][kF16Ld]
  C* twl = X + 16 * kF16Ld;               // 256 twiddles exp(-2 pi i m / 256)
  __shared__ int64_t lbase[kF16Lines];
  __shared__ T lfac[kF16Lines], lksq[kF16Lines];
  // scaling: the x factors e_x and k_x^2 of the 256 points, staged once per
  // block (read from LDS in the middle of the transform, not from memory)
  __shared__ T xfac[SCALE ? 256 : 1], xksq[SCALE ? 256 : 1];
  const int64_t L0 = (int64_t)blockIdx.x * kF16Lines;
  if ((int)threadIdx.x < kF16Lines) {
    const int64_t L = L0 + threadIdx.x;
    const bool valid = L < nlines && (int)(L % vmod) < vlim;
    lbase[threadIdx.x] = valid ? (L / inner) * outer + (L % inner) : -1;
    if (SCALE && valid) {
      const int y = (int)(L / sa.Nzs);
      const int kz = (int)(L - (int64_t)y * sa.Nzs);
      lfac[threadIdx.x] = (T)(sa.ey[y] * sa.ez[kz] * sa.norm);
      lksq[threadIdx.x] = (T)(sa.ky2[y] + sa.kz2[kz]);
    }
  }
  twl[threadIdx.x] = tw[threadIdx.x];
  if (SCALE) {
    xfac[threadIdx.x] = (T)sa.ex[threadIdx.x];
    xksq[threadIdx.x] = (T)sa.kx2[threadIdx.x];
  }
  __syncthreads();
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t lb = lbase[c];
  auto twiddle = [&](int m, int sgn) {  // W256^m for the transform of sign sgn
    C w = twl[m & 255];
    if (sgn < 0) w.y = -w.y;
    return w;
  };
  C v[16];
  // inner DFT over j1 of x[16 j1 + g], twiddle W256^(g k1), exchange
#pragma unroll
  for (int j1 = 0; j1 < 16; ++j1) v[j1] = lb >= 0 ? data[lb + (int64_t)(16 * j1 + g) * stride] : C{0, 0};
  dft16<T, C>(v, fwd);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], twiddle(g * k1, fwd));
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) X[k1 * kF16Ld + g * 16 + c] = v[k1];
  __syncthreads();
  // outer DFT over j2 for k1 = g
#pragma unroll
  for (int j2 = 0; j2 < 16; ++j2) v[j2] = X[g * kF16Ld + j2 * 16 + c];
  dft16<T, C>(v, fwd);
  if (SCALE) {
    // v[k2] = X[g + 16 k2]: scale by the Green's function, then the inverse
    // with k = k1 + 16 k2 (k1 = g held here): inner DFT over k2 in registers,
    // twiddle W256^-(g j1), exchange, outer DFT over k1
    if (lb >= 0) {
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) {
        const int kx = g + 16 * k2;
        const T k2s = xksq[kx] + lksq[c];
        // single precision: the hardware reciprocal (1 ulp) instead of the
        // correctly rounded division sequence
        T inv;
        if constexpr (sizeof(T) == 4) inv = __builtin_amdgcn_rcpf(k2s);
        else inv = (T)1 / k2s;
        T gk = k2s > (T)0 ? xfac[kx] * lfac[c] * inv : (T)0;
        if (sa.shell_a > 0.0) gk *= j0_squared<T>(k2s, (T)sa.shell_a);
        v[k2] = {v[k2].x * gk, v[k2].y * gk};
      }
    }
    dft16<T, C>(v, -fwd);
#pragma unroll
    for (int j1 = 1; j1 < 16; ++j1) v[j1] = cmul(v[j1], twiddle(g * j1, -fwd));
    __syncthreads();  // every read of the first exchange is done
#pragma unroll
    for (int j1 = 0; j1 < 16; ++j1) X[j1 * kF16Ld + g * 16 + c] = v[j1];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) v[k1] = X[g * kF16Ld + k1 * 16 + c];
    dft16<T, C>(v, -fwd);
  }
  // v[m] is element g + 16 m of line c
  if (lb >= 0) {
#pragma unroll
    for (int m = 0; m < 16; ++m) data[lb + (int64_t)(g + 16 * m) * stride] = v[m];
  }
}

// z passes of 256 points, two real lines per complex line, in the same
// two-stage form.  Thread (c, g) = (t / 16, t mod 16) works on complex line c
// of the block (16 per block), so the 16 lanes of a line read or write 16
// neighbouring values.  The exchange between the stages goes through LDS
// with the value index XORed by the row (k1 or j2), which keeps both the
// writes of one row and the column reads of the other stage free of bank
// conflicts.  r2c: Z_{N-k}, needed to split the packed transform, sits in
// lane (c, 16 - g) of the same wavefront (register 15 - k2), or for g = 0 in
// the lane itself (register 16 - k2): a lane shuffle, no second exchange.
template <typename T>
__global__ void __launch_bounds__(256) fft256_z_r2c_kernel(const T* __restrict__ real,
                                                           typename C2<T>::type* __restrict__ cplx, int Nzs,
                                                           int64_t nlines, const typename C2<T>::type* __restrict__ tw) {
  using C = typename C2<T>::type;
  constexpr int Nz = 256;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* X = reinterpret_cast<C*>(smem_raw);  // [16 lines][kF16Ld]
  C* twl = X + 16 * kF16Ld;
  twl[threadIdx.x] = tw[threadIdx.x];
  const int c = threadIdx.x >> 4, g = threadIdx.x & 15;
  const int64_t la = 2 * ((int64_t)blockIdx.x * 16 + c), lb = la + 1;
  const bool va = la < nlines, vb = lb < nlines;
  C v[16];
#pragma unroll
  for (int j1 = 0; j1 < 16; ++j1) {
    const int j = 16 * j1 + g;
    v[j1] = {va ? real[la * Nz + j] : (T)0, vb ? real[lb * Nz + j] : (T)0};
  }
  __syncthreads();  // twiddles
  dft16<T, C>(v, 1);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) {
    const C w = twl[(g * k1) & 255];
    v[k1] = cmul(v[k1], w);
  }
  C* Xl = X + c * kF16Ld;
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) Xl[k1 * 16 + (g ^ k1)] = v[k1];
  __syncthreads();
#pragma unroll
  for (int j2 = 0; j2 < 16; ++j2) v[j2] = Xl[g * 16 + (j2 ^ g)];
  dft16<T, C>(v, 1);
  // v[k2] = Z_k, k = g + 16 k2
  const int lane = threadIdx.x & 63;
  const int partner = (lane & 48) | ((16 - g) & 15);
#pragma unroll
  for (int k2 = 0; k2 <= 8; ++k2) {
    C p;
    p.x = __shfl(v[15 - k2].x, partner, 64);
    p.y = __shfl(v[15 - k2].y, partner, 64);
    if (g == 0) p = v[(16 - k2) & 15];
    const int k = g + 16 * k2;
    if (k > Nz / 2) continue;
    const C z = v[k2];
    const C A = {(T)0.5 * (z.x + p.x), (T)0.5 * (z.y - p.y)};
    const C Bv = {(T)0.5 * (z.y + p.y), (T)-0.5 * (z.x - p.x)};
    if (va) cplx[la * Nzs + k] = A;
    if (vb) cplx[lb * Nzs + k] = Bv;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) fft256_z_c2r_kernel(const typename C2<T>::type* __restrict__ cplx,
                                                           T* __restrict__ real, int Nzs, int64_t nlines,
                                                           const typename C2<T>::type* __restrict__ tw) {
  using C = typename C2<T>::type;
  constexpr int Nz = 256;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* X = reinterpret_cast<C*>(smem_raw);
  C* twl = X + 16 * kF16Ld;
  twl[threadIdx.x] = tw[threadIdx.x];
  const int c = threadIdx.x >> 4, g = threadIdx.x & 15;
  const int64_t la = 2 * ((int64_t)blockIdx.x * 16 + c), lb = la + 1;
  const bool va = la < nlines, vb = lb < nlines;
  C v[16];
  // z_k = A_k + i B_k over the full spectrum.  Only k <= N/2 is read (j1 <= 8);
  // above it z_k = conj(A_{N-k}) + i conj(B_{N-k}), and N - k = g' + 16 j1'
  // sits in lane (c, 16 - g) at j1' = 15 - j1, or for g = 0 in the lane itself
  // at j1' = 16 - j1: that lane forms the mirrored value and a shuffle brings it.
  C m[9];
#pragma unroll
  for (int j1 = 0; j1 <= 8; ++j1) {
    const int k = 16 * j1 + g;
    C A = {0, 0}, Bv = {0, 0};
    if (k <= Nz / 2) {
      if (va) A = cplx[la * Nzs + k];
      if (vb) Bv = cplx[lb * Nzs + k];
    }
    v[j1] = {A.x - Bv.y, A.y + Bv.x};
    m[j1] = {A.x + Bv.y, Bv.x - A.y};
  }
  {
    const int lane = threadIdx.x & 63;
    const int partner = (lane & 48) | ((16 - g) & 15);
#pragma unroll
    for (int j1 = 8; j1 < 16; ++j1) {
      C p;
      p.x = __shfl(m[15 - j1].x, partner, 64);
      p.y = __shfl(m[15 - j1].y, partner, 64);
      if (g == 0) p = m[(16 - j1) & 15];
      // k = 16 j1 + g is above N/2 except k = N/2 itself (j1 = 8, g = 0)
      if (j1 > 8 || g > 0) v[j1] = p;
    }
  }
  __syncthreads();  // twiddles
  dft16<T, C>(v, -1);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) {
    C w = twl[(g * k1) & 255];
    w.y = -w.y;
    v[k1] = cmul(v[k1], w);
  }
  C* Xl = X + c * kF16Ld;
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) Xl[k1 * 16 + (g ^ k1)] = v[k1];
  __syncthreads();
#pragma unroll
  for (int j2 = 0; j2 < 16; ++j2) v[j2] = Xl[g * 16 + (j2 ^ g)];
  dft16<T, C>(v, -1);
  // v[k2] = x_j, j = g + 16 k2: real line a in x, b in y
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    const int j = g + 16 * k2;
    if (va) real[la * Nz + j] = v[k2].x;
    if (vb) real[lb * Nz + j] = v[k2].y;
  }
}

// z pass, real -> half complex, two real lines per complex transform.
template <typename T>
__global__ void __launch_bounds__(256) fft_z_r2c_kernel(const T* __restrict__ real,
                                                        typename C2<T>::type* __restrict__ cplx,
                                                        int Nz, int Nzs, int64_t nlines, int ppb, FFTPlan1D plan,
                                                        const typename C2<T>::type* __restrict__ tw) {
  using C = typename C2<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* b0 = reinterpret_cast<C*>(smem_raw);
  const int ls = Nz + 1;
  C* b1 = b0 + ppb * ls;
  const int Nzc = Nz / 2 + 1;
  const int64_t p0 = (int64_t)blockIdx.x * ppb;
  for (int t = threadIdx.x; t < Nz * ppb; t += blockDim.x) {
    const int c = t / Nz;
    const int j = t - c * Nz;
    const int64_t la = 2 * (p0 + c), lb = la + 1;
    T a = 0, b = 0;
    if (la < nlines) a = real[la * Nz + j];
    if (lb < nlines) b = real[lb * Nz + j];
    b0[c * ls + j] = {a, b};
  }
  __syncthreads();
  C* res = lds_fft<T, C>(b0, b1, Nz, ppb, LdsLayout{ls, 0}, plan, tw, 1);
  for (int t = threadIdx.x; t < Nzc * ppb; t += blockDim.x) {
    const int c = t / Nzc;
    const int k = t - c * Nzc;
    const int64_t la = 2 * (p0 + c), lb = la + 1;
    const C zk = res[c * ls + k];
    const C zn = res[c * ls + ((Nz - k) % Nz)];
    // A = (Z_k + conj Z_{N-k}) / 2 ; B = (Z_k - conj Z_{N-k}) / (2i)
    const C A = {(T)0.5 * (zk.x + zn.x), (T)0.5 * (zk.y - zn.y)};
    const T dr = zk.x - zn.x, di = zk.y + zn.y;
    const C Bv = {(T)0.5 * di, (T)-0.5 * dr};
    if (la < nlines) cplx[la * Nzs + k] = A;
    if (lb < nlines) cplx[lb * Nzs + k] = Bv;
  }
}

// z pass, half complex -> real (unnormalized inverse), two lines at once.
template <typename T>
__global__ void __launch_bounds__(256) fft_z_c2r_kernel(const typename C2<T>::type* __restrict__ cplx,
                                                        T* __restrict__ real, int Nz, int Nzs, int64_t nlines,
                                                        int ppb, FFTPlan1D plan,
                                                        const typename C2<T>::type* __restrict__ tw) {
  using C = typename C2<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* b0 = reinterpret_cast<C*>(smem_raw);
  const int ls = Nz + 1;
  C* b1 = b0 + ppb * ls;
  const int Nzc = Nz / 2 + 1;
  const int64_t p0 = (int64_t)blockIdx.x * ppb;
  for (int t = threadIdx.x; t < Nz * ppb; t += blockDim.x) {
    const int c = t / Nz;
    const int k = t - c * Nz;
    const int64_t la = 2 * (p0 + c), lb = la + 1;
    C A = {0, 0}, Bv = {0, 0};
    if (k < Nzc) {
      if (la < nlines) A = cplx[la * Nzs + k];
      if (lb < nlines) Bv = cplx[lb * Nzs + k];
    } else {
      if (la < nlines) { A = cplx[la * Nzs + (Nz - k)]; A.y = -A.y; }
      if (lb < nlines) { Bv = cplx[lb * Nzs + (Nz - k)]; Bv.y = -Bv.y; }
    }
    b0[c * ls + k] = {A.x - Bv.y, A.y + Bv.x};  // A + i B
  }
  __syncthreads();
  C* res = lds_fft<T, C>(b0, b1, Nz, ppb, LdsLayout{ls, 0}, plan, tw, -1);
  for (int t = threadIdx.x; t < Nz * ppb; t += blockDim.x) {
    const int c = t / Nz;
    const int j = t - c * Nz;
    const int64_t la = 2 * (p0 + c), lb = la + 1;
    const C z = res[c * ls + j];
    if (la < nlines) real[la * Nz + j] = z.x;
    if (lb < nlines) real[lb * Nz + j] = z.y;
  }
}

// About 2048 complex values per block (8 per thread) so a pass launches
// many blocks; two ping-pong LDS buffers of (n+1) values per line must fit
// the budget.
// Strided passes: up to 4096 values per block, as many lines as fit (a power
// of two, so the contiguous index is read in aligned runs of 128 bytes or
// more); two unpadded LDS buffers must fit the budget.
inline int strided_lines_per_block(int n, size_t elem, size_t lds_budget) {
  int cap = 4096 / n;
  const int lds_cap = (int)(lds_budget / (2 * (size_t)n * elem));
  if (lds_cap < cap) cap = lds_cap;
  int l = 1;
  while (2 * l <= cap && 2 * l <= 64) l *= 2;
  return l;
}

inline int lines_per_block(int n, size_t elem, size_t lds_budget) {
  int l = 2048 / n;
  const int cap = (int)(lds_budget / (2 * (size_t)(n + 1) * elem));
  if (l > cap) l = cap;
  if (l < 1) l = 1;
  if (l > 64) l = 64;
  return l;
}

}  // namespace

void build_green_tables(pe_context* c) {
  const int Nx = c->p.mesh[0], Ny = c->p.mesh[1], Nz = c->p.mesh[2], Nzc = Nz / 2 + 1;
  const int ns[3] = {Nx, Ny, Nzc};
  const double gexp = (1.0 - c->eta) / (4.0 * c->xi * c->xi);
  std::vector<double> e, k2;
  for (int d = 0; d < 3; ++d) {
    const int N = c->p.mesh[d];
    for (int m = 0; m < ns[d]; ++m) {
      const int sm = (d < 2 && m >= (N + 1) / 2) ? m - N : m;
      const double k = 2.0 * M_PI * sm / c->p.box[d];
      e.push_back(std::exp(-gexp * k * k));
      k2.push_back(k * k);
    }
  }
  e.insert(e.end(), k2.begin(), k2.end());
  c->gtab.ensure(e.size());
  PE_HIP(hipMemcpy(c->gtab.get(), e.data(), sizeof(double) * e.size(), hipMemcpyHostToDevice));
}

void make_fft_plan(int n, FFTPlan1D& plan) {
  require(n >= 1 && n <= 1024, "FFT length must be in [1, 1024]");
  plan.n = n;
  plan.nstage = 0;
  int m = n;
  while (m > 1) {
    int r;
    if (m % 8 == 0) r = 8;
    else if (m % 4 == 0) r = 4;
    else if (m % 2 == 0) r = 2;
    else if (m % 3 == 0) r = 3;
    else if (m % 5 == 0) r = 5;
    else throw Error(PE_ERR_ARG, "mesh size " + std::to_string(n) + " has a prime factor other than 2, 3, 5");
    require(plan.nstage < 16, "FFT length has too many factors");
    plan.radix[plan.nstage++] = r;
    m /= r;
  }
}

template <typename T>
void launch_wave_pipeline(hipStream_t s, pe_context* c, T* gA, T* gB, void* gCv) {
  using C = typename C2<T>::type;
  C* gC = reinterpret_cast<C*>(gCv);
  const GridGeom& g = c->gg;
  const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2], Nzc = g.Nzc, Nzs = g.Nzs;
  const C* twx;
  const C* twy;
  const C* twz;
  if constexpr (sizeof(T) == 8) {
    twx = c->tw64[0].get(); twy = c->tw64[1].get(); twz = c->tw64[2].get();
  } else {
    twx = c->tw32[0].get(); twy = c->tw32[1].get(); twz = c->tw32[2].get();
  }
  const size_t budget = 64 * 1024;
  // strided passes: what the device allows per workgroup, less the static
  // per-line tables (64-line maximum)
  const size_t sbudget = std::min<size_t>((size_t)c->lds_per_block, 80 * 1024) - 2048;
  // 256-point strided lines: the two-stage kernel, where its LDS fits
  const size_t sh256 = (16 * (size_t)kF16Ld + 256) * sizeof(C);
  auto use256 = [&](int n) { return n == 256 && sh256 + 1024 <= (size_t)c->lds_per_block; };
  // 1. z, r2c
  {
    ProfScope ps(c->prof, s, PE_PROF_FFT_Z_R2C, sizeof(T) == 8, 1.0);
    const int64_t nlines = (int64_t)Nx * Ny;
    const int64_t npairs = (nlines + 1) / 2;
    if (use256(Nz)) {
      hipLaunchKernelGGL(fft256_z_r2c_kernel<T>, dim3((unsigned)((npairs + 15) / 16)), dim3(256), sh256, s, gA, gC,
                         Nzs, nlines, twz);
      PE_CHECK_LAUNCH();
    } else {
    const int ppb = lines_per_block(Nz, sizeof(C), budget);
    const unsigned nb = (unsigned)((npairs + ppb - 1) / ppb);
    const size_t sh = 2 * (size_t)ppb * (Nz + 1) * sizeof(C);
    hipLaunchKernelGGL(fft_z_r2c_kernel<T>, dim3(nb), dim3(256), sh, s, gA, gC, Nz, Nzs, nlines, ppb,
                       c->plan[2], twz);
    PE_CHECK_LAUNCH();
    }
  }
  ScaleArgs sa{};
  sa.Nx = Nx; sa.Ny = Ny; sa.Nz = Nz; sa.Nzc = Nzc; sa.Nzs = Nzs;
  const double* gt = c->gtab.get();
  sa.ex = gt;
  sa.ey = gt + Nx;
  sa.ez = gt + Nx + Ny;
  sa.kx2 = gt + Nx + Ny + Nzc;
  sa.ky2 = sa.kx2 + Nx;
  sa.kz2 = sa.ky2 + Ny;
  sa.norm = 1.0 / ((double)Nx * Ny * Nz);
  sa.shell_a = c->p.reg == PE_REG_SHELL_PAPER ? c->p.shell_radius : 0.0;
  // 2. y forward: lines (x, kz), element y
  auto ypass = [&](int fwd) {
    ProfScope ps(c->prof, s, fwd > 0 ? PE_PROF_FFT_Y_FWD : PE_PROF_FFT_Y_INV, sizeof(T) == 8, 1.0);
    const int64_t nlines = (int64_t)Nx * Nzs;
    if (use256(Ny)) {
      hipLaunchKernelGGL((fft256_lines_kernel<T, false>), dim3((unsigned)((nlines + 15) / 16)), dim3(256), sh256, s,
                         gC, nlines, (int64_t)Nzs, (int64_t)Ny * Nzs, (int64_t)Nzs, Nzs, Nzc, twy, fwd, sa);
      PE_CHECK_LAUNCH();
      return;
    }
    const int lpb = strided_lines_per_block(Ny, sizeof(C), sbudget);
    const unsigned nb = (unsigned)((nlines + lpb - 1) / lpb);
    const size_t sh = 2 * (size_t)lpb * Ny * sizeof(C);
    hipLaunchKernelGGL((fft_lines_kernel<T, false>), dim3(nb), dim3(lpb * Ny >= 4096 ? 512 : 256), sh, s, gC, Ny, nlines,
                       (int64_t)Nzs, (int64_t)Ny * Nzs, (int64_t)Nzs, Nzs, Nzc, lpb, c->plan[1], twy, fwd, sa);
    PE_CHECK_LAUNCH();
  };
  ypass(1);
  // 3. x forward + scale + x inverse: lines (y, kz), element x
  {
    ProfScope ps(c->prof, s, PE_PROF_FFT_X_SCALE, sizeof(T) == 8, 1.0);
    const int64_t nlines = (int64_t)Ny * Nzs;
    if (use256(Nx)) {
      hipLaunchKernelGGL((fft256_lines_kernel<T, true>), dim3((unsigned)((nlines + 15) / 16)), dim3(256), sh256, s,
                         gC, nlines, nlines, (int64_t)0, (int64_t)Ny * Nzs, Nzs, Nzc, twx, 1, sa);
      PE_CHECK_LAUNCH();
    } else {
    const int lpb = strided_lines_per_block(Nx, sizeof(C), sbudget);
    const unsigned nb = (unsigned)((nlines + lpb - 1) / lpb);
    const size_t sh = 2 * (size_t)lpb * Nx * sizeof(C);
    hipLaunchKernelGGL((fft_lines_kernel<T, true>), dim3(nb), dim3(lpb * Nx >= 4096 ? 512 : 256), sh, s, gC, Nx, nlines,
                       nlines, (int64_t)0, (int64_t)Ny * Nzs, Nzs, Nzc, lpb, c->plan[0], twx, 1, sa);
    PE_CHECK_LAUNCH();
    }
  }
  // 4. y inverse
  ypass(-1);
  // 5. z, c2r into grid B
  {
    ProfScope ps(c->prof, s, PE_PROF_FFT_Z_C2R, sizeof(T) == 8, 1.0);
    const int64_t nlines = (int64_t)Nx * Ny;
    const int64_t npairs = (nlines + 1) / 2;
    if (use256(Nz)) {
      hipLaunchKernelGGL(fft256_z_c2r_kernel<T>, dim3((unsigned)((npairs + 15) / 16)), dim3(256), sh256, s, gC, gB,
                         Nzs, nlines, twz);
      PE_CHECK_LAUNCH();
    } else {
    const int ppb = lines_per_block(Nz, sizeof(C), budget);
    const unsigned nb = (unsigned)((npairs + ppb - 1) / ppb);
    const size_t sh = 2 * (size_t)ppb * (Nz + 1) * sizeof(C);
    hipLaunchKernelGGL(fft_z_c2r_kernel<T>, dim3(nb), dim3(256), sh, s, gC, gB, Nz, Nzs, nlines, ppb,
                       c->plan[2], twz);
    PE_CHECK_LAUNCH();
    }
  }
}

template void launch_wave_pipeline<float>(hipStream_t, pe_context*, float*, float*, void*);
template void launch_wave_pipeline<double>(hipStream_t, pe_context*, double*, double*, void*);

}  // namespace pe
