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
// digits to cancellation; erfc(b r) is dropped once b r is so large that it
// is below the rounding of the other term.
//
// Pair traversal (one kernel for every pass): a wavefront takes up to 64
// targets of one cell, one per lane, so every lane scans the same candidate
// sources.  The wavefront loads 64 candidates at a time (one per lane) and
// broadcasts them lane by lane; each lane tests the distance in single
// precision against a slightly enlarged cutoff and, on a hit, appends the
// source to its own queue in LDS.  Whenever every lane has work queued (or
// a queue runs close to full) the wavefront pops one entry per lane and
// evaluates the pair kernel with all lanes busy, redoing the distance in
// double with the exact cutoff.  So the expensive error-function evaluations
// run at full width instead of once per candidate for any hit in the
// wavefront, and each lane still sums its own pairs in a fixed order.
//
// Positions are fixed during a solve, so the bead-bead block is evaluated once
// per configuration and stored as a CSR matrix (rows in cell order, entries
// in traversal order).  Every Krylov iteration then applies it as a sparse
// matrix-vector product.  One-off passes (ion -> bead for the right-hand
// side, all pairs with fields for the forces) are evaluated on the fly.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <type_traits>

#include "pe_internal.hpp"
#include "vector.hpp"

namespace pe {

namespace {

constexpr int kWaves = 4;  // wavefronts per 256-thread block
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

// b r beyond which erfc(b r) is dropped: erfc(6.5) = 3.8e-20, erfc(5) = 1.5e-12.
template <typename T>
__device__ __forceinline__ T erfc_drop() { return sizeof(T) == 8 ? (T)6.5 : (T)5.0; }

template <typename T>
__device__ __forceinline__ T erf_diff(T b, T xi, T r) {
  // erf(b r) - erf(xi r)
  const T br = b * r;
  if (br < (T)1.0) return erf(br) - erf(xi * r);
  if (br > erfc_drop<T>()) return erfc(xi * r);
  return erfc(xi * r) - erfc(br);
}

// The paper's split for shells of radius a (j0^2(ka) in both parts): the
// real-space kernel is the inverse transform of (1 - h(k)) j0^2(ka) / k^2,
// whose printed closed form (its Heaviside term read as
// -(1/(4 pi r) - (4a - r)/(16 pi a^2)) H(2a - r)) regroups as a second
// difference,
//   R(r) = [g(r + 2a) + g(r - 2a) - 2 g(r)] / (a^2 r) - Heaviside term,
//   g(s) = (2 xi^2 s^2 + 1) erfc(xi s) / (64 pi xi^2) - s exp(-xi^2 s^2) / (32 pi^1.5 xi),
//   g'(s) = (s erfc(xi s) - exp(-xi^2 s^2) / (sqrt(pi) xi)) / (16 pi).
// The difference cancels about (a xi)^-2 of the leading digits, so it is
// formed in double whatever the caller's precision.
__device__ __forceinline__ void shell_paper_g(double s, double xi, double& gv, double& g1) {
  const double ec = erfc(xi * s), ex = exp(-xi * xi * s * s);
  gv = (2.0 * xi * xi * s * s + 1.0) * ec * (1.0 / (64.0 * kPi)) / (xi * xi) - s * ex / (32.0 * kPi * sqrt(kPi) * xi);
  g1 = (s * ec - ex / (sqrt(kPi) * xi)) * (1.0 / (16.0 * kPi));
}

__device__ __forceinline__ void shell_paper_kernel(double r, const RealGeom& g, double& R, double& dR) {
  const double a = g.a, xi = g.xi, c = 1.0 / g.eps;
  double gp, g1p, gm, g1m, g0, g10;
  shell_paper_g(r + 2.0 * a, xi, gp, g1p);
  shell_paper_g(r - 2.0 * a, xi, gm, g1m);
  shell_paper_g(r, xi, g0, g10);
  const double G = gp + gm - 2.0 * g0, G1 = g1p + g1m - 2.0 * g10;
  const double ia2 = 1.0 / (a * a);
  double v = G * ia2 / r, d = G1 * ia2 / r - G * ia2 / (r * r);
  if (r < 2.0 * a) {
    v -= kInv4Pi / r - (4.0 * a - r) * ia2 * (1.0 / (16.0 * kPi));
    d -= -kInv4Pi / (r * r) + ia2 * (1.0 / (16.0 * kPi));
  }
  R = c * v;
  dR = c * d;
}

// R(r) and dR/dr for one pair (r > 0).
template <typename T>
__device__ __forceinline__ void pair_kernel(T r, T s2, const RealGeom& g, T& R, T& dR, bool want_d) {
  const T xi = (T)g.xi;
  const T c = (T)(kInv4Pi / g.eps);
  const T inv_r = (T)1 / r;
  if (g.reg == PE_REG_SHELL_PAPER) {
    double Rd, dRd;
    shell_paper_kernel((double)r, g, Rd, dRd);
    R = (T)Rd;
    if (want_d) dR = (T)dRd;
    return;
  }
  if (g.reg == PE_REG_GAUSSIAN) {
    const T b = rsqrt((T)2 * s2);
    const T D = erf_diff<T>(b, xi, r);
    R = c * D * inv_r;
    if (want_d) {
      // d/dr [D/r] = (D' r - D)/r^2, D' = (2/sqrt pi)(b e^{-b^2 r^2} - xi e^{-xi^2 r^2})
      const T eb = b * r > erfc_drop<T>() ? (T)0 : b * exp(-b * b * r * r);
      const T Dp = (T)kTwoOverSqrtPi * (eb - xi * exp(-xi * xi * r * r));
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
  if (g.reg == PE_REG_SHELL_PAPER) {
    // the printed self term of the paper's split (the kernel's r -> 0 limit)
    const double a = g.a, xi = g.xi;
    return (T)(((1.0 - exp(-4.0 * a * a * xi * xi)) / (8.0 * kPi * sqrt(kPi) * a * a * xi) +
                erfc(2.0 * a * xi) * kInv4Pi / a) / g.eps);
  }
  return c * ((T)1 / (T)g.a - (T)2 * (T)g.xi / (T)sqrt(kPi));
}

// Single-precision Gaussian pair kernel with no data-dependent branch but a
// rarely taken one for tiny distances.  erfc(x) = exp(-x^2) erfcx(x), erfcx
// from the piecewise Taylor table (float relative error about 1e-7), and the
// two Gaussians exp(-x^2) serve the derivative as well.  Where both arguments
// are below 1/2 the difference of error functions comes from the Maclaurin
// series of erf instead, which keeps its relative accuracy as r -> 0.
//   R = c D / r,   F = -R'(r) / r = c (D - D' r) / r^3,
//   D = erf(b r) - erf(xi r),  D' = (2/sqrt pi)(b e^{-b^2 r^2} - xi e^{-xi^2 r^2}).
// Beyond the table's range the last piece is held (erfc(6) = 2e-17, so the
// product is far below the rounding of every other term).
__device__ __forceinline__ float erfcx_lookup(const float4* __restrict__ tab, float x) {
  const float xc = fminf(x, (float)kErfcxPieces / kErfcxInvWidth);
  const int k = min((int)(xc * kErfcxInvWidth), kErfcxPieces - 1);
  const float s = xc - ((float)k + 0.5f) * (1.0f / kErfcxInvWidth);
  static_assert(kErfcxDeg == 7, "two float4 per piece");
  const float4 lo = tab[2 * k], hi = tab[2 * k + 1];
  float v = fmaf(hi.w, s, hi.z);
  v = fmaf(v, s, hi.y);
  v = fmaf(v, s, hi.x);
  v = fmaf(v, s, lo.w);
  v = fmaf(v, s, lo.z);
  v = fmaf(v, s, lo.y);
  return fmaf(v, s, lo.x);
}

// erf(x) = (2/sqrt pi) sum_n (-1)^n x^(2n+1) / (n! (2n+1)), n <= 7: below
// 1e-9 relative for x < 1/2.
__device__ __forceinline__ float erf_series(float x) {
  const float z = x * x;
  float v = -1.0f / 75600.0f;
  v = fmaf(v, z, 1.0f / 9360.0f);
  v = fmaf(v, z, -1.0f / 1320.0f);
  v = fmaf(v, z, 1.0f / 216.0f);
  v = fmaf(v, z, -1.0f / 42.0f);
  v = fmaf(v, z, 1.0f / 10.0f);
  v = fmaf(v, z, -1.0f / 3.0f);
  v = fmaf(v, z, 1.0f);
  return (float)kTwoOverSqrtPi * x * v;
}

__device__ __forceinline__ void pair_kernel_fast(float r2, float s2, float xi, float c,
                                                 const float4* __restrict__ tab, float& R, float& F) {
  const float inv_r = __builtin_amdgcn_rsqf(r2);
  const float r = r2 * inv_r;
  const float b = __builtin_amdgcn_rsqf(2.0f * s2);
  const float x1 = xi * r, x2 = b * r;
  constexpr float kLog2e = 1.44269504088896341f;
  const float e1 = __builtin_amdgcn_exp2f(-(x1 * x1) * kLog2e);
  const float e2 = __builtin_amdgcn_exp2f(-(x2 * x2) * kLog2e);
  float D;
  if (fmaxf(x1, x2) < 0.5f) D = erf_series(x2) - erf_series(x1);
  else D = e1 * erfcx_lookup(tab, x1) - e2 * erfcx_lookup(tab, x2);
  const float Dp = (float)kTwoOverSqrtPi * (b * e2 - xi * e1);
  R = c * D * inv_r;
  F = c * (D - Dp * r) * (inv_r * inv_r * inv_r);
}

// ---------------------------------------------------------------- cell list

// Order within a cell: by the particle's z slab (kZSlabs per cell), then by
// caller index, packed in one sort key (slab << kSlabShift | index) while the
// set has fewer than 2^kSlabShift particles (larger sets sort by index
// only).  A traversal unit, a run of consecutive particles of one (x, y)
// column, then spans a short stretch of z instead of whole cells, so its
// bounding box, and the candidates it tests, shrink.
constexpr int kSlabShift = 24;
constexpr int kZSlabs = 128;

__global__ void assign_cells_kernel(const double* __restrict__ pos, const double* __restrict__ sig,
                                    double sig_const, int64_t n, RealGeom g, double4* __restrict__ tmp,
                                    int* __restrict__ cell_of, int* __restrict__ zsub, int* __restrict__ count,
                                    unsigned long long* __restrict__ sig_check) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // uniform widths: sig_check[1] = the first width; a wavefront that sees
  // another value sets sig_check[0] (a plain store of 1, no atomics, so the
  // common uniform case costs nothing)
  const double s_ref = sig ? sig[0] : sig_const;
  bool differs = false;
  if (i < n) {
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
    const double fz = z * g.cell_inv[2] - cz;  // position within the cell along z, [0, 1)
    zsub[i] = min(max((int)(fz * kZSlabs), 0), kZSlabs - 1);
    atomicAdd(&count[c], 1);
    differs = !(s == s_ref);
  }
  if (i == 0) sig_check[1] = (unsigned long long)__double_as_longlong(s_ref);
  if (__ballot(differs) != 0ull && (threadIdx.x & 63) == 0) sig_check[0] = 1ull;
}

// idx receives sort keys (see kSlabShift); gather_sorted_kernel strips them.
__global__ void scatter_cells_kernel(const int* __restrict__ cell_of, const int* __restrict__ zsub, int64_t n,
                                     int slabs, int* __restrict__ cursor, int* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int slot = atomicAdd(&cursor[cell_of[i]], 1);
  idx[slot] = slabs ? (int)i | zsub[i] << kSlabShift : (int)i;
}

__global__ void gather_sorted_kernel(const double4* __restrict__ tmp, int* __restrict__ idx,
                                     const int* __restrict__ owner, int64_t n, int slabs, RealGeom g,
                                     double4* __restrict__ pos, float4* __restrict__ posf, uint4* __restrict__ posx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = slabs ? idx[i] & ((1 << kSlabShift) - 1) : idx[i];
  idx[i] = k;
  const double4 p = tmp[k];
  pos[i] = p;
  // single-precision copy: x and y relative to the origin of the particle's
  // cell, z as is (cells of one (x, y) column are read as one run)
  const double ax = g.L[0] / g.nc[0], ay = g.L[1] / g.nc[1];
  const int cx = cell_coord(p.x, g.cell_inv[0], g.nc[0]);
  const int cy = cell_coord(p.y, g.cell_inv[1], g.nc[1]);
  const int tag = owner ? owner[k] : -1;
  posf[i] = make_float4((float)(p.x - cx * ax), (float)(p.y - cy * ay), (float)p.z, __int_as_float(tag));
  // fixed point: the box maps onto 2^32 units per axis, so the 32-bit
  // difference of two records is exact and already the minimum image
  auto fix = [](double x, double inv_L) { return (unsigned)(long long)rint(x * inv_L * 4294967296.0); };
  posx[i] = make_uint4(fix(p.x, g.inv_L[0]), fix(p.y, g.inv_L[1]), fix(p.z, g.inv_L[2]), __float_as_uint((float)p.w));
}

// Charges of a set in its sorted (cell) order, so the pair kernels read them
// without the index indirection.
__global__ void sort_charges_kernel(const int* __restrict__ idx, const double* __restrict__ q, int64_t n,
                                    double* __restrict__ qs, float* __restrict__ qsf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double v = q[idx[i]];
    qs[i] = v;
    qsf[i] = (float)v;
  }
}

// ------------------------------------------------------------ pair traversal

// One source set of a traversal.
struct SrcSet {
  const double4* pos;   // sorted by cell: wrapped x, y, z, sigma
  const float4* posf;   // single precision: x, y relative to the cell origin, z; w: owner tag
  const uint4* posx;    // fixed point (2^32 units per box length): x, y, z; w: sigma as float bits
  const int* idx;       // sorted slot -> caller index
  const int* start;     // cell_start
  const double* q;      // charges in sorted order (potential passes)
  const float* qf;      // the same in single precision
  const float4* tab;    // pair table of the class (targets, this set), or null
};

// Outputs of a traversal; which ones are used depends on the mode.
struct PairOut {
  double* phi;          // potential, caller order of the targets (added to)
  double* E;            // field (3 per target) or null
  int* cnt;             // per sorted target: pairs within r_c (count mode)
  const int64_t* row_ptr;
  int* col;             // CSR of the bead block (fill mode)
  double* v64;
  float* v32;
  const int* body_of;          // count / fill: body of each bead (caller order)
  const unsigned char* dense;  // count / fill: per body, intra-body pairs held by a dense block
  unsigned long long* npairs;  // if set: pairs inside the cutoff evaluated are added here
};

enum { MODE_COUNT = 0, MODE_FILL = 1, MODE_POT = 2, MODE_FIELD = 3 };

constexpr int kQ = 16;          // queue entries per lane
constexpr int kQFlush = 8;      // candidates between flushes (kQ - kQFlush entries stay free)
constexpr int kSetBit = 30;     // queue entry: sorted source index | set << kSetBit
constexpr int kMaxRuns = 36;    // stencil runs: 2 source sets x 9 columns x 2 runs
// single-precision passes: staged candidates stay in an LDS ring of
// kRegions batches of 64 and the queues hold ring slots (slot | set <<
// kRingSetShift); one more slot, kRing, is a placeholder (at the origin,
// charge zero) that a lane with no queued pair evaluates
constexpr int kRegions = 2;
constexpr int kRing = 64 * kRegions;
constexpr int kRingSetShift = 11;  // the set's offset in the class tables in LDS, in bytes
static_assert(kRing < 256 && (kRegions & (kRegions - 1)) == 0, "ring slots are 8 bits, regions a power of two");
static_assert(2 * kPairTabPieces * 16 == 1 << kRingSetShift, "one set's class table: two float4 per piece");


// EV selects the pair evaluation: EV_GENERAL (any precision and
// regularization), EV_ERFCX (single precision, Gaussian: erfc from the
// scaled-erfc table, per-pair widths) or EV_TABLE (single precision,
// Gaussian, uniform widths per set: R and R' from the class tables).
enum { EV_GENERAL = 0, EV_ERFCX = 1, EV_TABLE = 2 };

template <int MODE, typename T, typename TF, int EV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(EV == EV_TABLE ? 6 : 1))) pair_queue_kernel(
    const double4* __restrict__ tpos, const uint4* __restrict__ tposx, const int* __restrict__ tidx,
    const int* __restrict__ tstart, const int4* __restrict__ chunks, int nchunk, SrcSet s0, SrcSet s1, int nsrc,
    RealGeom g, float rc2f, PairOut out) {
  static_assert(EV == EV_GENERAL || (sizeof(T) == 4 && sizeof(TF) == 4 && (MODE == MODE_POT || MODE == MODE_FIELD)),
                "table evaluations are single-precision potential / field passes");
  constexpr bool kOwn = MODE == MODE_COUNT || MODE == MODE_FILL;
  constexpr int kTabF4 = EV == EV_TABLE ? 4 * kPairTabPieces : (EV == EV_ERFCX ? 2 * kErfcxPieces : 1);
  // Single-precision passes keep every staged candidate (position in the
  // target frame, charge, width) in an LDS ring and queue ring slots, so a
  // pair's evaluation reads LDS only; the general pass queues source indices
  // and reads the double records from global memory.
  constexpr bool kRingQ = EV != EV_GENERAL;
  using QE = typename std::conditional<kRingQ, unsigned short, int>::type;
  __shared__ QE qbuf[kWaves][kQ][64];
  __shared__ float4 cbuf[kWaves][kRingQ ? kRing + 1 : 64];  // ring: -2 x, -2 y, -2 z, |c|^2; else x, y, z, entry
  __shared__ float cq[kRingQ ? kWaves : 1][kRingQ ? kRing + 1 : 1];                // ring: charge
  __shared__ float cw[EV == EV_ERFCX ? kWaves : 1][EV == EV_ERFCX ? kRing + 1 : 1];  // ring: width
  __shared__ float4 etab[kTabF4];
  __shared__ int cownb[kOwn ? kWaves : 1][64];  // owner tags of the staged candidates (count / fill)
  __shared__ int rstart[kWaves][kMaxRuns + 1];
  __shared__ int rbase[kWaves][kMaxRuns];
  __shared__ int rcode[kWaves][kMaxRuns];    // per run: set | (ox+1) << 1 | (oy+1) << 3 | z image << 5
  if constexpr (EV == EV_ERFCX) {
    if (threadIdx.x < 2 * kErfcxPieces) etab[threadIdx.x] = reinterpret_cast<const float4*>(g.erfcx)[threadIdx.x];
    __syncthreads();  // before any wavefront leaves
  } else if constexpr (EV == EV_TABLE) {
    // the class tables of source sets 0 and 1 (2 float4 per piece)
    for (int i = threadIdx.x; i < 4 * kPairTabPieces; i += blockDim.x)
      etab[i] = i < 2 * kPairTabPieces ? s0.tab[i] : s1.tab[i - 2 * kPairTabPieces];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int w = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wv;
  if (w >= nchunk) return;  // whole wavefront; no block barrier follows
  // chunk: sorted targets [begin, end) in the cells cell .. cell + nz - 1 of
  // one (x, y) column
  const int4 ch = chunks[w];
  const int begin = __builtin_amdgcn_readfirstlane(ch.x);
  const int end = __builtin_amdgcn_readfirstlane(ch.y);
  const int cell = __builtin_amdgcn_readfirstlane(ch.z);
  const int nz = __builtin_amdgcn_readfirstlane(ch.w);
  const int t = begin + lane;
  const bool active = t < end;
  const double4 p = tpos[active ? t : begin];
  const int nc0 = g.nc[0], nc1 = g.nc[1], nc2 = g.nc[2];
  const int cz = cell % nc2, cy = (cell / nc2) % nc1, cx = cell / (nc1 * nc2);
  const bool per_pair_image = nc0 < 3 || nc1 < 3 || nc2 < 3;
  const int rx = nc0 >= 3 ? 1 : 0, ry = nc1 >= 3 ? 1 : 0, rz = nc2 >= 3 ? 1 : 0;
  const float Lf0 = (float)g.L[0], Lf1 = (float)g.L[1], Lf2 = (float)g.L[2];
  const double a0 = g.L[0] / nc0, a1 = g.L[1] / nc1;
  QE (*qb)[64] = qbuf[wv];
  int pushed = 0, popped = 0;

  // per-target results
  T acc = 0;
  TF ex = 0, ey = 0, ez = 0;
  int cnt = 0;
  int nev = 0;  // pairs inside the cutoff this lane evaluated
  int64_t o = 0, o_end = 0;
  if (MODE == MODE_FILL && active) {
    o = out.row_ptr[t];
    o_end = out.row_ptr[t + 1];
  }
  // count / fill: pairs inside a body with a dense intra-body block are left out
  int own_body = -1;
  if ((MODE == MODE_COUNT || MODE == MODE_FILL) && out.dense) {
    const int b = out.body_of[tidx[active ? t : begin]];
    if (out.dense[b]) own_body = b;
  }

  auto evaluate = [&](int e) {
    const int set = e >> kSetBit;
    const int sidx = e & ((1 << kSetBit) - 1);
    const double4 qp = set ? s1.pos[sidx] : s0.pos[sidx];
    double dx = p.x - qp.x, dy = p.y - qp.y, dz = p.z - qp.z;
    dx -= g.L[0] * rint(dx * g.inv_L[0]);
    dy -= g.L[1] * rint(dy * g.inv_L[1]);
    dz -= g.L[2] * rint(dz * g.inv_L[2]);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < g.rc2)) return;
    ++nev;
    if constexpr (MODE == MODE_COUNT) {
      ++cnt;
      return;
    }
    const double s2 = p.w * p.w + qp.w * qp.w;
    if constexpr (MODE == MODE_FILL) {
      // the row was sized by the count pass; never write past it
      if (o < o_end) {
        out.col[o] = s0.idx[sidx];
        if (out.v64) {  // values here, or later from the structure
          double R;
          if (r2 == 0.0) {
            R = self_value<double>(s2, g);
          } else {
            double dR;
            pair_kernel<double>(sqrt(r2), s2, g, R, dR, false);
          }
          out.v64[o] = R;
          if (out.v32) out.v32[o] = (float)R;
        }
        ++o;
      }
      return;
    }
    const double qd = set ? s1.q[sidx] : s0.q[sidx];
    // the self pair (r = 0) has R(0) and no field; one accumulation site for
    // both cases keeps the sums in registers
    T R = 0;
    TF F = 0;  // -R'(r) / r
    if (r2 == 0.0) {
      R = self_value<T>((T)s2, g);
    } else {
      T dR = 0;
      const T r = (T)sqrt(r2);
      constexpr bool same = sizeof(T) == sizeof(TF);
      pair_kernel<T>(r, (T)s2, g, R, dR, MODE == MODE_FIELD && same);
      if constexpr (MODE == MODE_FIELD) {
        TF dRf;
        if constexpr (same) {
          dRf = (TF)dR;
        } else {
          TF Rf;
          pair_kernel<TF>((TF)r, (TF)s2, g, Rf, dRf, true);
        }
        F = -dRf / (TF)r;
      }
    }
    acc += R * (T)qd;
    if constexpr (MODE == MODE_FIELD) {
      const TF f = F * (TF)qd;  // E = -grad_t R q = -R'(r) d/r q
      ex += f * (TF)dx;
      ey += f * (TF)dy;
      ez += f * (TF)dz;
    }
  };

  // Single-precision evaluations: the candidate's position was staged in the
  // target frame (differences formed in double once per candidate, so the
  // float coordinates stay within about two cells of the origin), and a
  // lane's queued pair is evaluated from the ring alone.
  const float pw2 = (float)p.w * (float)p.w;
  const float rc2e = (float)g.rc2;
  const float xif = (float)g.xi, cf = (float)(kInv4Pi / g.eps);
  const float iL0 = (float)g.inv_L[0], iL1 = (float)g.inv_L[1], iL2 = (float)g.inv_L[2];
  auto evaluate_fast = [&](float dx, float dy, float dz, float qf, float sw) {
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (!(r2 < rc2e)) return;
    ++nev;
    const float s2 = fmaf(sw, sw, pw2);
    float R, F = 0.0f;
    if (r2 == 0.0f) R = self_value<float>(s2, g);
    else pair_kernel_fast(r2, s2, xif, cf, etab, R, F);
    acc += R * qf;
    if constexpr (MODE == MODE_FIELD) {
      const float fq = F * qf;
      ex += fq * dx;
      ey += fq * dy;
      ez += fq * dz;
    }
  };

  // Class tables: piece k = floor(w) of w = r / h (h = r_c / kPairTabPieces)
  // at t = 2 frac(w) - 1, so t stays in [-1, 1) and the polynomial finite.
  // Branch- and select-free: a lane with no queued pair evaluates the ring's
  // placeholder slot (charge zero) and adds exact zeros; w is clamped to the
  // last piece, which keeps the placeholder's (and a NaN difference's) table
  // read in range.  The self pair (r = 0) reads R(0) at the first piece's
  // first point; its field term vanishes with dx = dy = dz = 0.  The field
  // sums collect d u q x with u = 1 / (h r); -R'(r) / r = -2 d u, and the
  // factor -2 is applied once per target.
  const float tab_w = (float)(kPairTabPieces / sqrt(g.rc2));  // 1 / h
  const float tab_top = (float)kPairTabPieces - 0.0625f;
  auto evaluate_tab = [&](float dx, float dy, float dz, float q, int e) {
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float u = __builtin_amdgcn_rsqf(fmaxf(r2, 1e-30f)) * tab_w;
    const float w = fminf(r2 * u, tab_top);
    const float t = fmaf(2.0f, __builtin_amdgcn_fractf(w), -1.0f);
    const float4* tb =
        reinterpret_cast<const float4*>(reinterpret_cast<const char*>(etab) + (e & (1 << kRingSetShift))) +
        2 * (int)w;
    const float4 lo = tb[0], hi = tb[1];
    // degree 6: value v and slope d = dv/dt in one Horner pass
    float v = hi.z, d = hi.z;
    v = fmaf(v, t, hi.y);
    d = fmaf(d, t, v);
    v = fmaf(v, t, hi.x);
    d = fmaf(d, t, v);
    v = fmaf(v, t, lo.w);
    d = fmaf(d, t, v);
    v = fmaf(v, t, lo.z);
    d = fmaf(d, t, v);
    v = fmaf(v, t, lo.y);
    d = fmaf(d, t, v);
    v = fmaf(v, t, lo.x);
    acc = fmaf(v, q, acc);
    if constexpr (MODE == MODE_FIELD) {
      const float fq = d * u * q;
      ex = fmaf(fq, dx, ex);
      ey = fmaf(fq, dy, ey);
      ez = fmaf(fq, dz, ez);
    }
  };

  // The candidate stream.  The stencil is a list of runs: for each source
  // set and each (x, y) column, the cells along z (contiguous in the sorted
  // order; a second run holds the cell reached through the periodic wrap in
  // z).  Lane r describes run r; the runs are concatenated into one list of
  // M candidates that is visited in the order pos_j = j S mod M, with S
  // coprime to M near M times the golden ratio, so every stretch of the
  // stream samples all stencil cells evenly: each target then finds its
  // pairs at a steady rate and the queues of all lanes fill alike (a
  // cell-by-cell order feeds the targets near one face first and leaves the
  // others idle).  Candidates are staged 64 at a time in LDS, in the
  // frame of the target chunk, and tested in unrolled groups of kQFlush (the
  // batch is padded with NaN points, which never hit).  After every group
  // the queues are drained: as many rounds as keep every lane busy, and at
  // least enough that kQFlush more pushes cannot overflow any queue; after
  // the last group, everything left.  (One drain site, so the pair
  // evaluation is emitted once.)  Single-precision passes stage each batch
  // into the next of the ring's kRegions regions; before a region is staged
  // again, the drain also empties every queue entry that points into it.
  float4* cb = cbuf[wv];
  int* cown = cownb[kOwn ? wv : 0];
  int* rs = rstart[wv];
  int* rb = rbase[wv];
  int* rc = rcode[wv];
  const int sx = 2 * rx + 1, sy = 2 * ry + 1;
  const int n_open = nsrc * sx * sy * 2;  // <= kMaxRuns
  int rlen = 0;
  if (lane < n_open) {
    const int set = lane / (sx * sy * 2);
    const int rem = lane - set * (sx * sy * 2);
    const int ox = rem / (sy * 2) - rx, oy = (rem >> 1) % sy - ry, run = rem & 1;
    const SrcSet& S = set ? s1 : s0;
    int x = cx + ox, y = cy + oy;
    if (x < 0) x += nc0;
    if (x >= nc0) x -= nc0;
    if (y < 0) y += nc1;
    if (y >= nc1) y -= nc1;
    int zimg = 0;  // 1: image at z - L, 2: at z + L
    int z0 = 0, z1 = 0;
    if (rz == 0) {
      if (run == 0) { z0 = cz; z1 = cz + 1; }
    } else if (run == 0) {
      z0 = max(cz - 1, 0);
      z1 = min(cz + nz + 1, nc2);
    } else if (cz == 0) {
      z0 = nc2 - 1; z1 = nc2; zimg = 1;
    } else if (cz + nz == nc2) {
      z0 = 0; z1 = 1; zimg = 2;
    }
    const int c0 = (x * nc1 + y) * nc2;
    const int b0 = S.start[c0 + z0];
    rlen = z1 > z0 ? S.start[c0 + z1] - b0 : 0;
    rb[lane] = b0;
    rc[lane] = set | (ox + 1) << 1 | (oy + 1) << 3 | zimg << 5;
  }
  int incl = rlen;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane < n_open) rs[lane + 1] = incl;
  if (lane == 0) rs[0] = 0;
  if constexpr (kRingQ) {
    if (lane == 0) {  // the placeholder slot
      cb[kRing] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      cq[wv][kRing] = 0.0f;
    }
  }
  const int M = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
  // stride: near M / golden ratio, coprime to M (a permutation of 0 .. M-1)
  int stride = 1;
  if (M > 2) {
    stride = max(1, (int)(0.6180339887 * M + 0.5));
    for (;;) {
      int ga = stride, gb = M;
      while (gb) { const int tmp = ga % gb; ga = gb; gb = tmp; }
      if (ga == 1) break;
      ++stride;
    }
  }
  stride = __builtin_amdgcn_readfirstlane(stride);
  const int lane_pos = M > 0 ? (int)(((long long)lane * stride) % M) : 0;
  const int step64 = M > 0 ? __builtin_amdgcn_readfirstlane((int)((64LL * stride) % M)) : 0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // The target frame.  General passes: x, y relative to the target
  // column's origin, z as is (a source's float x, y are relative to its own
  // column's origin, which lies ox a0, oy a1 from the target column's origin
  // in the target's image).  Single-precision passes: relative to the centre
  // of the chunk's cells, from the fixed-point records: the 32-bit
  // difference to the centre is exact and the minimum image, rounded to
  // float once and scaled (the same operations for a target and a source,
  // so the self pair has r = 0 exactly).  With the stencil's cells distinct
  // (three columns per axis, a unit at most nc_z - 2 cells long) every
  // source within r_c of a target is that image; boxes of one cell along an
  // axis take the per-pair minimum image as well.
  const double a2 = g.L[2] / nc2;
  const double fx0 = cx * a0, fy0 = cy * a1;
  const double sfix = 4294967296.0;
  const unsigned fcx = (unsigned)(long long)rint((cx + 0.5) * a0 * g.inv_L[0] * sfix);
  const unsigned fcy = (unsigned)(long long)rint((cy + 0.5) * a1 * g.inv_L[1] * sfix);
  const unsigned fcz = (unsigned)(long long)rint((cz + 0.5 * nz) * a2 * g.inv_L[2] * sfix);
  const float fsc0 = (float)(g.L[0] / sfix), fsc1 = (float)(g.L[1] / sfix), fsc2 = (float)(g.L[2] / sfix);
  auto fix_off = [](unsigned a, unsigned c, float sc) { return (float)(int)(a - c) * sc; };
  float px, py, pz;
  if constexpr (kRingQ) {
    const uint4 tp = tposx[active ? t : begin];
    px = fix_off(tp.x, fcx, fsc0);
    py = fix_off(tp.y, fcy, fsc1);
    pz = fix_off(tp.z, fcz, fsc2);
  } else {
    px = (float)(p.x - fx0);
    py = (float)(p.y - fy0);
    pz = (float)p.z;
  }
  const float a0f = (float)a0, a1f = (float)a1, Lz = Lf2;
  // bounding box of the wavefront's targets (same frame as the candidates)
  float bx0 = active ? px : INFINITY, bx1 = active ? px : -INFINITY;
  float by0 = active ? py : INFINITY, by1 = active ? py : -INFINITY;
  float bz0 = active ? pz : INFINITY, bz1 = active ? pz : -INFINITY;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    bx0 = fminf(bx0, __shfl_xor(bx0, off, 64));
    bx1 = fmaxf(bx1, __shfl_xor(bx1, off, 64));
    by0 = fminf(by0, __shfl_xor(by0, off, 64));
    by1 = fmaxf(by1, __shfl_xor(by1, off, 64));
    bz0 = fminf(bz0, __shfl_xor(bz0, off, 64));
    bz1 = fmaxf(bz1, __shfl_xor(bz1, off, 64));
  }
  // uniform after the reduction: scalar registers
  auto uniform_f = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
  bx0 = uniform_f(bx0);
  bx1 = uniform_f(bx1);
  by0 = uniform_f(by0);
  by1 = uniform_f(by1);
  bz0 = uniform_f(bz0);
  bz1 = uniform_f(bz1);
  const float nanf_ = __int_as_float(0x7fc00000);
  if (kRingQ && !active) px = py = pz = nanf_;  // no candidate test hits
  // single-precision candidate test: |t - c|^2 < r_c^2 as
  // |c|^2 - 2 t.c < r_c^2 - |t|^2, three multiply-adds on the staged
  // (-2c, |c|^2) (rounding moves the test by about 1e-6 of r_c^2, where the
  // pair's value is at the split's tolerance; a queued pair just beyond r_c
  // is evaluated on the last piece of the table)
  const float thr = rc2e - fmaf(px, px, fmaf(py, py, pz * pz));
  int next = 0, pbase = 0;  // next stream position to stage and (next S) mod M
  int nbat = 0, k0 = 0;
  int batch = 0;  // batches staged
  const float4* cnd_base = cb;  // the batch under test
  int creg = 0, cn0 = 0;        // its ring region and its number of set-0 candidates (set 1 follows)
  // ring: pushed at the end of each of the last kRegions - 1 batches, newest first
  int ends[kRegions > 1 ? kRegions - 1 : 1] = {};
  for (;;) {
    bool finished = false;
    if (k0 >= nbat) {
      if (next < M) {
        float4 v = make_float4(nanf_, nanf_, nanf_, nanf_);
        float vq = 0.0f, vw = 0.0f;  // ring: charge and width
        int own = -1;
        bool keep = false;
        if (next + lane < M) {
          int pos = pbase + lane_pos;
          if (pos >= M) pos -= M;
          int lo = 0, hi = n_open;  // rs[lo] <= pos < rs[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rs[mid] <= pos) lo = mid;
            else hi = mid;
          }
          const int code = rc[lo];
          const int set = code & 1;
          const int sidx = rb[lo] + (pos - rs[lo]);
          if constexpr (kRingQ) {
            const uint4 sp = (set ? s1.posx : s0.posx)[sidx];
            v = make_float4(fix_off(sp.x, fcx, fsc0), fix_off(sp.y, fcy, fsc1), fix_off(sp.z, fcz, fsc2),
                            __int_as_float(set << kRingSetShift));
            vq = (set ? s1.qf : s0.qf)[sidx];
            vw = __uint_as_float(sp.w);
          } else {
            // the run's column and z image
            const float ofx = (float)(((code >> 1) & 3) - 1) * a0f;
            const float ofy = (float)(((code >> 3) & 3) - 1) * a1f;
            const int zimg = code >> 5;
            const float ofz = zimg == 1 ? -Lz : (zimg == 2 ? Lz : 0.0f);
            const float4 sp = (set ? s1.posf : s0.posf)[sidx];
            v = make_float4(sp.x + ofx, sp.y + ofy, sp.z + ofz, __int_as_float(sidx | set << kSetBit));
            own = __float_as_int(sp.w);
          }
          keep = true;
          if (!per_pair_image) {
            // farther than the cutoff from the targets' bounding box: no lane can hit it
            const float ex = fmaxf(fmaxf(bx0 - v.x, v.x - bx1), 0.0f);
            const float ey = fmaxf(fmaxf(by0 - v.y, v.y - by1), 0.0f);
            const float ez = fmaxf(fmaxf(bz0 - v.z, v.z - bz1), 0.0f);
            keep = ex * ex + ey * ey + ez * ez < rc2f;
          }
        }
        // the kept candidates first, in stream order (single-precision
        // passes: those of set 0, then those of set 1); NaN points after them
        const unsigned long long lt = (1ull << lane) - 1ull;
        const unsigned long long km = __ballot(keep);
        const int nkeep = __popcll(km);
        const int region = kRingQ ? (batch & (kRegions - 1)) * 64 : 0;
        float4* dst = cb + region;
        int n0 = nkeep;
        if constexpr (kRingQ) {
          const unsigned long long k1 = __ballot(keep && (__float_as_int(v.w) >> kRingSetShift) != 0);
          n0 = nkeep - __popcll(k1);
          if (keep) {
            const int slot = (k1 >> lane) & 1ull ? n0 + __popcll(k1 & lt) : __popcll(km & ~k1 & lt);
            cq[wv][region + slot] = vq;
            if constexpr (EV == EV_ERFCX) cw[wv][region + slot] = vw;
            dst[slot] = make_float4(-2.0f * v.x, -2.0f * v.y, -2.0f * v.z, fmaf(v.x, v.x, fmaf(v.y, v.y, v.z * v.z)));
          }
        } else if (keep) {
          const int slot = __popcll(km & lt);
          dst[slot] = v;
          if constexpr (MODE == MODE_COUNT || MODE == MODE_FILL) cown[slot] = own;
        }
        if (lane >= nkeep) dst[lane] = make_float4(nanf_, nanf_, nanf_, nanf_);  // slots past the kept ones
        cnd_base = dst;
        creg = __builtin_amdgcn_readfirstlane(region);
        cn0 = __builtin_amdgcn_readfirstlane(n0);
        ++batch;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        nbat = nkeep;
        next += min(64, M - next);
        pbase += step64;
        if (pbase >= M) pbase -= M;
        k0 = 0;
      } else {
        finished = true;
      }
    }
    if (!finished && kRingQ) {
      // (the per-pair minimum image is a separate copy of the loop)
      auto test_group = [&](auto img) {
#pragma unroll
        for (int kk = 0; kk < kQFlush; ++kk) {
          const float4 cnd = cnd_base[k0 + kk];
          bool hit;
          if constexpr (decltype(img)::value) {  // the differences as the evaluation forms them
            float dx = fmaf(0.5f, cnd.x, px), dy = fmaf(0.5f, cnd.y, py), dz = fmaf(0.5f, cnd.z, pz);
            dx -= Lf0 * rintf(dx * iL0);
            dy -= Lf1 * rintf(dy * iL1);
            dz -= Lf2 * rintf(dz * iL2);
            hit = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < rc2e;
          } else {
            hit = fmaf(px, cnd.x, fmaf(py, cnd.y, fmaf(pz, cnd.z, cnd.w))) < thr;
          }
          // the slot at pushed is free (at most kQ - 1 entries pending)
          const int kc = k0 + kk;
          qb[pushed & (kQ - 1)][lane] = (QE)((creg + kc) | (kc >= cn0 ? 1 << kRingSetShift : 0));
          pushed += hit ? 1 : 0;
        }
      };
      if (per_pair_image) test_group(std::true_type{});
      else test_group(std::false_type{});
      k0 += kQFlush;
    } else if (!finished) {
#pragma unroll
      for (int kk = 0; kk < kQFlush; ++kk) {
        const float4 cnd = cnd_base[k0 + kk];
        float dx = px - cnd.x;
        float dy = py - cnd.y;
        float dz = pz - cnd.z;
        if (per_pair_image) {
          dx -= Lf0 * rintf(dx / Lf0);
          dy -= Lf1 * rintf(dy / Lf1);
          dz -= Lf2 * rintf(dz / Lf2);
        }
        bool hit = active && dx * dx + dy * dy + dz * dz < rc2f;
        if constexpr (MODE == MODE_COUNT || MODE == MODE_FILL) {
          // pairs inside a body with a dense intra-body block are not listed
          hit = hit && (own_body < 0 || cown[k0 + kk] != own_body);
        }
        // the slot at pushed is free (at most kQ - 1 entries pending)
        qb[pushed & (kQ - 1)][lane] = (QE)__float_as_int(cnd.w);
        pushed += hit ? 1 : 0;
      }
      k0 += kQFlush;
    }
    if constexpr (EV == EV_GENERAL) {
      const int pend = pushed - popped;
      int mn = active ? pend : 1 << 30, mx = pend;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        mn = min(mn, __shfl_xor(mn, off, 64));
        mx = max(mx, __shfl_xor(mx, off, 64));
      }
      const int rounds = finished ? mx : max(mn, mx - (kQ - kQFlush));
      for (int r = 0; r < rounds; ++r) {
        if (popped < pushed) {
          const int e = qb[popped & (kQ - 1)][lane];
          ++popped;
          evaluate(e);
        }
      }
    } else {
      // The same drain policy decided by ballots pass by pass: another round
      // while some queue holds more than kQ - kQFlush entries, or every
      // active lane has one, or (the batch's last group) some entry points
      // into the region the next staging reuses, that of batch
      // (this - kRegions + 1), whose entries are the first ends[last]; after
      // the last group, while any entry is left.
      const bool batch_end = !finished && k0 >= nbat;
      const int old_end = kRegions > 1 ? ends[kRegions > 1 ? kRegions - 2 : 0] : pushed;
      if (batch_end) {
#pragma unroll
        for (int i = kRegions - 2; i > 0; --i) ends[i] = ends[i - 1];
        ends[0] = pushed;
      }
      // rounds per drain pass: with more, the lanes whose queues hold fewer
      // entries than the pass takes evaluate the placeholder
      constexpr int kPass = 1;
      auto rounds_wanted = [&]() {  // 0 .. kPass (or more) rounds still due
        const int pend = pushed - popped;
        auto due = [&](int r) {  // at least r more rounds
          if (finished) return __ballot(pend >= r) != 0ull;
          // (every active lane holding r entries: the chunk's first lane is active)
          bool d = __ballot(pend > kQ - kQFlush + r - 1) != 0ull ||
                   (__ballot(active && pend < r) == 0ull && __ballot(pend >= r) != 0ull);
          if (batch_end) d = d || __ballot(old_end - popped >= r) != 0ull;
          return d;
        };
#pragma unroll
        for (int r = kPass; r > 0; --r)
          if (due(r)) return r;
        return 0;
      };
      // kPass rounds per pass, all ring entries read first (a lane without an
      // entry reads the placeholder slot); the per-pair minimum image (boxes
      // of one cell along an axis) is a separate copy of the loop
      const float4* ring = cb;
      auto drain = [&](auto img) {
        constexpr bool kImg = decltype(img)::value;
        auto diff = [&](float d, float Lf, float iL) { return kImg ? d - Lf * rintf(d * iL) : d; };
        for (;;) {
          const int rw = rounds_wanted();
          if (rw == 0) break;
          const int avail = min(pushed - popped, rw);
          int e[kPass];
          float4 cv[kPass];
          float qv[kPass];
#pragma unroll
          for (int i = 0; i < kPass; ++i) e[i] = avail > i ? (int)qb[(popped + i) & (kQ - 1)][lane] : kRing;
#pragma unroll
          for (int i = 0; i < kPass; ++i) {
            cv[i] = ring[e[i] & 255];
            qv[i] = cq[wv][e[i] & 255];
          }
          popped += avail;
#pragma unroll
          for (int i = 0; i < kPass; ++i) {
            // (the ring holds -2c: t - c = t + c' / 2, exact as a subtraction)
            const float dx = diff(fmaf(0.5f, cv[i].x, px), Lf0, iL0), dy = diff(fmaf(0.5f, cv[i].y, py), Lf1, iL1),
                        dz = diff(fmaf(0.5f, cv[i].z, pz), Lf2, iL2);
            if constexpr (EV == EV_TABLE) evaluate_tab(dx, dy, dz, qv[i], e[i]);
            else if (avail > i) evaluate_fast(dx, dy, dz, qv[i], cw[wv][e[i] & 255]);
          }
        }
      };
      if (per_pair_image) drain(std::true_type{});
      else drain(std::false_type{});
    }
    if (finished) break;
  }
  if (out.npairs) {
    // (table passes evaluate every queued entry, each inside the cutoff)
    unsigned long long v = (unsigned long long)(EV == EV_TABLE ? pushed : nev);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) atomicAdd(out.npairs, v);
  }
  if (!active) return;
  if (MODE == MODE_COUNT) {
    out.cnt[t] = cnt;
  } else if (MODE == MODE_FILL) {
    // a pair counted but not found again (rounding at the cutoff) adds
    // nothing: column -1 - own index, value zero
    for (; o < o_end; ++o) {
      out.col[o] = -1 - tidx[t];
      if (out.v64) {
        out.v64[o] = 0.0;
        if (out.v32) out.v32[o] = 0.0f;
      }
    }
  } else if (MODE == MODE_POT || MODE == MODE_FIELD) {
    const int oi = tidx[t];
    out.phi[oi] += (double)acc;
    if (MODE == MODE_FIELD) {
      const TF fs = EV == EV_TABLE ? (TF)-2 : (TF)1;  // see evaluate_tab
      out.E[3 * oi] += (double)(fs * ex);
      out.E[3 * oi + 1] += (double)(fs * ey);
      out.E[3 * oi + 2] += (double)(fs * ez);
    }
  }
}

// phi_real[b] += sum_j R_bj q_j over the stored inter-body pairs of bead b
// (which then holds the whole real-space part).  CSR rows in cell order;
// kSpmvLanes lanes per row read the row's entries contiguously and reduce
// with lane shuffles.  Rows hold about ten entries, so a lane takes one or
// two: each lane loads its first two entries and the bead's own term before
// using any of them, which overlaps the chains of dependent loads.
constexpr int kSpmvLanes = 8;

template <typename T>
__global__ void __launch_bounds__(256) spmv_add_kernel(const int64_t* __restrict__ row_ptr,
                                                       const int* __restrict__ col, const T* __restrict__ val,
                                                       const int* __restrict__ row_bead, int64_t n,
                                                       const double* __restrict__ q, double* __restrict__ phi_real) {
  constexpr int L = kSpmvLanes;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int sub = threadIdx.x % L;
  T acc = 0;
  int b = 0;
  double pn = 0.0;
  if (i < n) {
    const int64_t o0 = row_ptr[i] + sub, e = row_ptr[i + 1];
    b = row_bead[i];
    int j0 = 0, j1 = 0;  // a negative column is a zero entry
    T v0 = 0, v1 = 0;
    if (o0 < e) {
      j0 = col[o0];
      v0 = val[o0];
    }
    if (o0 + L < e) {
      j1 = col[o0 + L];
      v1 = val[o0 + L];
    }
    if (sub == 0) pn = phi_real[b];
    if (o0 < e) acc = v0 * (T)q[j0 < 0 ? -1 - j0 : j0];
    if (o0 + L < e) acc += v1 * (T)q[j1 < 0 ? -1 - j1 : j1];
    for (int64_t o = o0 + 2 * L; o < e; o += L) {
      const int jj = col[o];
      acc += val[o] * (T)q[jj < 0 ? -1 - jj : jj];
    }
  }
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, L);
  if (i < n && sub == 0) phi_real[b] = (double)acc + pn;
}

// y_top[b] = -(phi_wave[b] + phi_real[b] - ck0_b) + dpsi[body(b)]
__global__ void __launch_bounds__(256) assemble_kernel(int64_t n, const double* __restrict__ phi_wave,
                                                       const double* __restrict__ phi_real,
                                                       const double* __restrict__ sig, const double* __restrict__ ck,
                                                       const double* __restrict__ dpsi, const int* __restrict__ body_of,
                                                       double* __restrict__ y) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const double sg = sig[b];
  const double phi = phi_wave[b] + phi_real[b] - (ck[0] - ck[1] * sg * sg);
  y[b] = -phi + (dpsi ? dpsi[body_of[b]] : 0.0);
}

// Values of the stored bead-bead pairs from the current positions (caller
// order, minimum image) with the exact cutoff: R(r) inside r_c, the self
// value at r = 0, zero outside r_c and for the zero entries (negative
// column).  16 lanes per row, each taking every 16th entry.
__global__ void __launch_bounds__(256) csr_refresh_kernel(const int64_t* __restrict__ row_ptr,
                                                          const int* __restrict__ col,
                                                          const int* __restrict__ row_bead, int64_t n,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ sig, RealGeom g,
                                                          double* __restrict__ v64, float* __restrict__ v32) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int sub = threadIdx.x & 15;
  if (i >= n) return;
  const int b = row_bead[i];
  const double xb = x[3 * b], yb = x[3 * b + 1], zb = x[3 * b + 2], sb = sig[b];
  for (int64_t o = row_ptr[i] + sub; o < row_ptr[i + 1]; o += 16) {
    const int j = col[o];
    double R = 0.0;
    if (j >= 0) {
      const double dx = min_img(xb - x[3 * j], g.L[0], g.inv_L[0]);
      const double dy = min_img(yb - x[3 * j + 1], g.L[1], g.inv_L[1]);
      const double dz = min_img(zb - x[3 * j + 2], g.L[2], g.inv_L[2]);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double s2 = sb * sb + sig[j] * sig[j];
      if (r2 == 0.0) {
        R = self_value<double>(s2, g);
      } else if (r2 < g.rc2) {
        double dR;
        pair_kernel<double>(sqrt(r2), s2, g, R, dR, false);
      }
    }
    v64[o] = R;
    if (v32) v32[o] = (float)R;
  }
}

// Per-block maximum of |x - x0|^2 over the beads (caller order, unwrapped).
__global__ void __launch_bounds__(256) max_disp_kernel(const double* __restrict__ x, const double* __restrict__ x0,
                                                       int64_t n, double* __restrict__ part) {
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double dx = x[3 * i] - x0[3 * i], dy = x[3 * i + 1] - x0[3 * i + 1], dz = x[3 * i + 2] - x0[3 * i + 2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    m = d2 > m || d2 != d2 ? d2 : m;  // a NaN wins, so it forces a rebuild
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double v = __shfl_xor(m, o, 64);
    m = v > m || v != v ? v : m;
  }
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int w = 1; w < 4; ++w) t = sh[w] > t || sh[w] != sh[w] ? sh[w] : t;
    part[blockIdx.x] = t;
  }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// Cutoff of the single-precision candidate test: r_c enlarged by more than
// the rounding of the float coordinates (at most a box length in size), so
// no pair inside r_c is missed; the exact test is redone in double.
float candidate_rc2(const RealGeom& g) {
  double lmax = 0;
  for (int d = 0; d < 3; ++d) lmax = std::max(lmax, g.L[d]);
  const double rc = std::sqrt(g.rc2);
  const double rcf = rc * (1.0 + 1e-5) + 16.0 * lmax * std::ldexp(1.0, -24);
  return (float)(rcf * rcf);
}

void cells_count(hipStream_t s, ParticleSet& ps, const double* pos_caller, const double* sig_caller,
                 double sig_const, int64_t n, const RealGeom& rg) {
  ps.n = n;
  ps.wfac_valid = false;
  const int ncell = rg.nc[0] * rg.nc[1] * rg.nc[2];
  ps.pos.ensure(n);
  ps.posf.ensure(n);
  ps.posx.ensure(n);
  ps.idx.ensure(n);
  ps.tmp.ensure(n);
  ps.cell_of.ensure(n);
  ps.zsub.ensure(n);
  ps.cell_start.ensure(ncell + 1);
  ps.cell_count.ensure(ncell);
  PE_HIP(hipMemsetAsync(ps.cell_count.get(), 0, sizeof(int) * ncell, s));
  ps.sig_check.ensure(2);
  PE_HIP(hipMemsetAsync(ps.sig_check.get(), 0, sizeof(unsigned long long), s));
  if (n > 0) {
    hipLaunchKernelGGL(assign_cells_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, pos_caller, sig_caller,
                       sig_const, n, rg, ps.tmp.get(), ps.cell_of.get(), ps.zsub.get(), ps.cell_count.get(),
                       ps.sig_check.get());
    PE_CHECK_LAUNCH();
  }
  // counts and, 8-byte aligned after them, the width check in one
  // page-locked buffer
  const size_t sig_at = ((size_t)ncell + 1) & ~(size_t)1;  // ints
  int* cnt = ps.h_ccnt.get<int>(sig_at + 4);
  unsigned long long* sig = reinterpret_cast<unsigned long long*>(cnt + sig_at);
  PE_HIP(hipMemcpyAsync(cnt, ps.cell_count.get(), sizeof(int) * ncell, hipMemcpyDeviceToHost, s));
  if (n > 0) PE_HIP(hipMemcpyAsync(sig, ps.sig_check.get(), 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
}

void cells_finish(hipStream_t s, ParticleSet& ps, const int* owner, const RealGeom& rg) {
  const int64_t n = ps.n;
  const int ncell = rg.nc[0] * rg.nc[1] * rg.nc[2];
  const size_t sig_at = ((size_t)ncell + 1) & ~(size_t)1;  // ints
  const int* cnt = ps.h_ccnt.get<int>(sig_at + 4);
  const unsigned long long* sig = reinterpret_cast<const unsigned long long*>(cnt + sig_at);
  int* start_pinned = ps.h_cstart.get<int>((size_t)ncell + 1);
  {
    double w = 0;
    if (n > 0) std::memcpy(&w, &sig[1], sizeof(double));
    ps.sig_uniform = n > 0 && sig[0] == 0 && w > 0 && w < INFINITY ? w : 0.0;
  }
  // offsets in ordinary host memory (the walk below reads them many times;
  // the page-locked copy only carries the upload), the counts read once
  std::vector<int>& start_v = ps.h_start;
  start_v.resize((size_t)ncell + 1);
  int cmax = 0;
  start_v[0] = 0;
  for (int c = 0; c < ncell; ++c) {
    const int k = cnt[c];
    start_v[c + 1] = start_v[c] + k;
    cmax = std::max(cmax, k);
  }
  const int* start = start_v.data();
  // traversal work units: runs of up to 64 consecutive particles of one
  // (x, y) column, so a wavefront's lanes are all busy however the cells are
  // filled; a unit spans at most nz_max cells along z (the stencil reaches
  // one cell beyond each end, and with nz <= nc_z - 2 the cell reached
  // through the periodic wrap is never also a cell of the run)
  const int nc0 = rg.nc[0], nc1 = rg.nc[1], nc2 = rg.nc[2];
  const int nz_max = nc2 >= 3 ? std::min(nc2 - 2, 2) : 1;
  const int ncol = nc0 * nc1;
  // work order: bricks of kBrick^3 cells, so the units in flight on one XCD
  // (a contiguous range, see xcd_remap) read their sources from a compact
  // region that its L2 can hold, rather than from a slab of whole planes.
  // One pass: the bricks in order, and in each the columns' units that start
  // in the brick, every column walked on from where its previous brick left
  // it (per column the next particle and its cell).
  constexpr int kBrick = 8;
  // at most n/64 full units, and per column one unit per nz_max cells ended
  // by the z limit and one ended by the column's end
  const int64_t bound = n / 64 + 1 + (int64_t)ncol * ((nc2 + nz_max - 1) / nz_max + 1);
  int4* chunks = ps.h_chunks.get<int4>((size_t)bound);
  std::vector<int>& ccur = ps.h_colcur;
  std::vector<int>& cz = ps.h_colz;
  ccur.resize(ncol);
  cz.assign(ncol, 0);
  for (int col = 0; col < ncol; ++col) ccur[col] = start[col * nc2];
  int nch = 0;
  for (int bx = 0; bx < nc0; bx += kBrick)
    for (int by = 0; by < nc1; by += kBrick)
      for (int bz = 0; bz < nc2; bz += kBrick) {
        const int zb = std::min(bz + kBrick, nc2);
        for (int x = bx; x < std::min(bx + kBrick, nc0); ++x)
          for (int y = by; y < std::min(by + kBrick, nc1); ++y) {
            const int col = x * nc1 + y, c0 = col * nc2;
            const int* st = start + c0;
            int cur = ccur[col], z = cz[col];
            const int col_end = st[nc2];
            while (cur < col_end) {
              while (st[z + 1] <= cur) ++z;  // cell of the unit's first particle
              if (z >= zb) break;            // the unit starts in a later brick
              int end = std::min(cur + 64, col_end);
              end = std::min(end, st[std::min(z + nz_max, nc2)]);
              int zl = z;
              while (st[zl + 1] < end) ++zl;  // cell of the unit's last particle
              require(nch < bound, "traversal work units exceed their bound");
              chunks[nch++] = make_int4(cur, end, c0 + z, zl - z + 1);
              cur = end;
            }
            ccur[col] = cur;
            cz[col] = z;
          }
      }
  ps.n_chunks = nch;
  ps.chunks.ensure(std::max<int64_t>(ps.n_chunks, 1));
  if (ps.n_chunks)
    PE_HIP(hipMemcpyAsync(ps.chunks.get(), chunks, sizeof(int4) * ps.n_chunks, hipMemcpyHostToDevice, s));
  std::memcpy(start_pinned, start, sizeof(int) * ((size_t)ncell + 1));
  PE_HIP(hipMemcpyAsync(ps.cell_start.get(), start_pinned, sizeof(int) * (ncell + 1), hipMemcpyHostToDevice, s));
  // cursor = start (reuse cell_count)
  PE_HIP(hipMemcpyAsync(ps.cell_count.get(), start_pinned, sizeof(int) * ncell, hipMemcpyHostToDevice, s));
  if (n > 0) {
    const int slabs = n < ((int64_t)1 << kSlabShift) ? 1 : 0;
    hipLaunchKernelGGL(scatter_cells_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, ps.cell_of.get(), ps.zsub.get(), n,
                       slabs, ps.cell_count.get(), ps.idx.get());
    PE_CHECK_LAUNCH();
    // sort each cell's slice by z slab and caller index, so the order (and
    // every sum over it) is the same on every run
    launch_segment_sort(s, ps.cell_start.get(), ncell, ps.idx.get(), cmax);
    hipLaunchKernelGGL(gather_sorted_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, ps.tmp.get(),
                       ps.idx.get(), owner, n, slabs, rg, ps.pos.get(), ps.posf.get(), ps.posx.get());
    PE_CHECK_LAUNCH();
  }
  // the host arrays live in the set: no wait here
}

void build_cells(hipStream_t s, ParticleSet& ps, const double* pos_caller, const double* sig_caller,
                 double sig_const, const int* owner, int64_t n, const RealGeom& rg) {
  cells_count(s, ps, pos_caller, sig_caller, sig_const, n, rg);
  PE_HIP(hipStreamSynchronize(s));
  cells_finish(s, ps, owner, rg);
}

namespace {

SrcSet src_of(const ParticleSet& ps, const double* qsorted, const float* qsortedf = nullptr,
              const float4* tab = nullptr) {
  return SrcSet{ps.pos.get(), ps.posf.get(), ps.posx.get(), ps.idx.get(), ps.cell_start.get(), qsorted, qsortedf, tab};
}

template <int MODE, typename T, typename TF, int EV>
void launch_queue_ev(hipStream_t s, const ParticleSet& tgt, const SrcSet& s0, const SrcSet& s1, int nsrc,
                     const RealGeom& rg, const PairOut& out) {
  hipLaunchKernelGGL((pair_queue_kernel<MODE, T, TF, EV>), dim3(nblk(tgt.n_chunks, kWaves)), dim3(64 * kWaves), 0,
                     s, tgt.pos.get(), tgt.posx.get(), tgt.idx.get(), tgt.cell_start.get(), tgt.chunks.get(),
                     tgt.n_chunks, s0, s1,
                     nsrc, rg, candidate_rc2(rg), out);
  PE_CHECK_LAUNCH();
}

// Single-precision Gaussian passes take the class tables when every source
// set has one, else the scaled-erfc kernel; everything else the general one.
template <int MODE, typename T, typename TF>
void launch_queue(hipStream_t s, const ParticleSet& tgt, const SrcSet& s0, const SrcSet& s1, int nsrc,
                  const RealGeom& rg, const PairOut& out) {
  if (tgt.n_chunks == 0) return;
  if constexpr (sizeof(T) == 4 && sizeof(TF) == 4 && (MODE == MODE_POT || MODE == MODE_FIELD)) {
    if (rg.reg == PE_REG_GAUSSIAN && s0.tab && s1.tab)
      return launch_queue_ev<MODE, T, TF, EV_TABLE>(s, tgt, s0, s1, nsrc, rg, out);
    if (rg.reg == PE_REG_GAUSSIAN && rg.erfcx)
      return launch_queue_ev<MODE, T, TF, EV_ERFCX>(s, tgt, s0, s1, nsrc, rg, out);
  }
  launch_queue_ev<MODE, T, TF, EV_GENERAL>(s, tgt, s0, s1, nsrc, rg, out);
}

}  // namespace

void launch_max_disp_early(pe_context* c) {
  c->disp_pending = false;
  const int64_t n = c->n_bead;
  if (!(c->csr_valid && n > 0 && c->csr_off == c->h_off)) return;
  const unsigned nbk = std::min<unsigned>(256, nblk(n, 256));
  c->csr_part.ensure(256);
  hipLaunchKernelGGL(max_disp_kernel, dim3(nbk), dim3(256), 0, c->stream, c->bead_x.get(), c->csr_x0.get(), n,
                     c->csr_part.get());
  PE_CHECK_LAUNCH();
  PE_HIP(hipMemcpyAsync(c->h_disp.get<double>(256), c->csr_part.get(), sizeof(double) * nbk, hipMemcpyDeviceToHost,
                        c->stream));
  c->disp_pending = true;
  c->disp_nbk = nbk;
}

void build_bead_matrix(pe_context* c) {
  hipStream_t s = c->stream;
  const int64_t n = c->n_bead;
  ParticleSet& B = c->B;
  require(n < (int64_t(1) << kSetBit), "too many particles in one set for the pair traversal");
  c->have_val32 = c->p.precision == PE_MIXED;
  // skin: what the cells allow beyond r_c (the 27-cell stencil must still
  // hold every pair within r_c + skin), at most r_c / 10; none when an axis
  // has fewer than three cells
  const double rc = std::sqrt(c->rg.rc2);
  double skin = 0.1 * rc;
  for (int d = 0; d < 3; ++d) {
    if (c->rg.nc[d] < 3) skin = 0.0;
    else skin = std::min(skin, c->rg.L[d] / c->rg.nc[d] - rc);
  }
  if (skin < 1e-3 * rc) skin = 0.0;
  bool rebuild = !(c->csr_valid && skin > 0 && c->csr_skin == skin && c->csr_rc == rc && c->csr_off == c->h_off &&
                   c->csr_dense == c->pc.dense_h);
  if (!rebuild && n > 0) {
    const double* part;
    unsigned nbk;
    if (c->disp_pending) {
      // launched by launch_max_disp_early; the stream has been waited on since
      part = c->h_disp.get<double>(256);
      nbk = c->disp_nbk;
    } else {
      nbk = std::min<unsigned>(256, nblk(n, 256));
      c->csr_part.ensure(256);
      hipLaunchKernelGGL(max_disp_kernel, dim3(nbk), dim3(256), 0, s, c->bead_x.get(), c->csr_x0.get(), n,
                         c->csr_part.get());
      PE_CHECK_LAUNCH();
      PE_HIP(hipMemcpyAsync(c->pinned, c->csr_part.get(), sizeof(double) * nbk, hipMemcpyDeviceToHost, s));
      PE_HIP(hipStreamSynchronize(s));
      part = c->pinned;
    }
    double mx = 0;
    for (unsigned k = 0; k < nbk; ++k) mx = (part[k] > mx || part[k] != part[k]) ? part[k] : mx;
    rebuild = !(mx <= 0.25 * skin * skin);
  }
  c->disp_pending = false;
  if (rebuild) {
    c->cnt.ensure(n);
    RealGeom rgb = c->rg;
    rgb.rc2 = (rc + skin) * (rc + skin);
    const SrcSet sb = src_of(B, nullptr);
    PairOut out{};
    out.cnt = c->cnt.get();
    if (c->n_body > 0) {
      out.body_of = c->body_of.get();
      out.dense = c->pc.dense.get();
    }
    if (n > 0) launch_queue<MODE_COUNT, double, double>(s, B, sb, sb, 1, rgb, out);
    // row offsets on the device; only the total comes back to size the arrays
    c->row_ptr.ensure(n + 1);
    c->scan_tmp.ensure((size_t)scan_workspace(n));
    launch_exclusive_scan(s, c->cnt.get(), n, c->row_ptr.get(), c->scan_tmp.get());
    PE_HIP(hipMemcpyAsync(c->pinned, c->row_ptr.get() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
    int64_t nnz;
    std::memcpy(&nnz, c->pinned, sizeof(int64_t));
    c->nnz = nnz;
    c->col.ensure(c->nnz);
    c->val64.ensure(c->nnz);
    if (c->have_val32) c->val32.ensure(c->nnz);
    out.row_ptr = c->row_ptr.get();
    out.col = c->col.get();
    // with a skin the values come from the refresh below (exact cutoff)
    out.v64 = skin > 0 ? nullptr : c->val64.get();
    out.v32 = skin > 0 || !c->have_val32 ? nullptr : c->val32.get();
    if (n > 0) launch_queue<MODE_FILL, double, double>(s, B, sb, sb, 1, rgb, out);
    c->csr_row.ensure((size_t)std::max<int64_t>(n, 1));
    if (n > 0) PE_HIP(hipMemcpyAsync(c->csr_row.get(), B.idx.get(), sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    c->csr_valid = skin > 0;
    c->csr_skin = skin;
    c->csr_rc = rc;
    c->csr_off = c->h_off;
    c->csr_dense = c->pc.dense_h;
    if (skin > 0) {
      c->csr_x0.ensure(3 * (size_t)std::max<int64_t>(n, 1));
      if (n > 0)
        PE_HIP(hipMemcpyAsync(c->csr_x0.get(), c->bead_x.get(), sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
    }
  }
  if (skin > 0 && n > 0) {
    hipLaunchKernelGGL(csr_refresh_kernel, dim3(nblk(16 * n, 256)), dim3(256), 0, s, c->row_ptr.get(), c->col.get(),
                       c->csr_row.get(), n, c->bead_x.get(), c->bead_sig.get(), c->rg, c->val64.get(),
                       c->have_val32 ? c->val32.get() : nullptr);
    PE_CHECK_LAUNCH();
  }
}

namespace {

// Dense intra-body block of one shape: every pair of the reference geometry
// (all closer than half the box, so each is its own minimum image), the
// diagonal by the self value.
__global__ void near_block_kernel(const double* __restrict__ ref, const double* __restrict__ sig, int N, RealGeom g,
                                  double* __restrict__ R64, float* __restrict__ R32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * N) return;
  const int i = (int)(e / N), j = (int)(e - (int64_t)i * N);
  const double dx = ref[3 * i] - ref[3 * j], dy = ref[3 * i + 1] - ref[3 * j + 1], dz = ref[3 * i + 2] - ref[3 * j + 2];
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double s2 = sig[i] * sig[i] + sig[j] * sig[j];
  double R;
  if (r2 == 0.0) {
    R = self_value<double>(s2, g);
  } else {
    double dR;
    pair_kernel<double>(sqrt(r2), s2, g, R, dR, false);
  }
  R64[e] = R;
  R32[e] = (float)R;
}

}  // namespace

void build_near_block(hipStream_t s, const BodyType& t, const RealGeom& rg, double* R64, float* R32) {
  const int N = t.N;
  DevBuf<double> dref, dsig;
  dref.ensure(3 * (size_t)N);
  dsig.ensure(N);
  PE_HIP(hipMemcpyAsync(dref.get(), t.ref.data(), sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
  PE_HIP(hipMemcpyAsync(dsig.get(), t.sig.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
  const int64_t NN = (int64_t)N * N;
  hipLaunchKernelGGL(near_block_kernel, dim3(nblk(NN, 256)), dim3(256), 0, s, dref.get(), dsig.get(), N, rg, R64,
                     R32);
  PE_CHECK_LAUNCH();
  PE_HIP(hipStreamSynchronize(s));
}

template <typename T>
void launch_spmv_add(hipStream_t s, pe_context* c, const double* q, double* phi_real) {
  const int64_t n = c->n_bead;
  if (n == 0) return;
  const T* val;
  if constexpr (sizeof(T) == 8) val = c->val64.get();
  else {
    require(c->have_val32, "float real-space operator not built (precision is PE_FP64)");
    val = c->val32.get();
  }
  hipLaunchKernelGGL(spmv_add_kernel<T>, dim3(nblk(kSpmvLanes * n, 256)), dim3(256), 0, s, c->row_ptr.get(),
                     c->col.get(), val, c->csr_row.get(), n, q, phi_real);
  PE_CHECK_LAUNCH();
}

void launch_assemble(hipStream_t s, pe_context* c, const double* dpsi, const double* phi_wave,
                     const double* phi_real, const double* ck0, double* y_top) {
  const int64_t n = c->n_bead;
  if (n == 0) return;
  hipLaunchKernelGGL(assemble_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, n, phi_wave, phi_real,
                     c->bead_sig.get(), ck0, dpsi, c->body_of.get(), y_top);
  PE_CHECK_LAUNCH();
}

template <typename T>
void launch_pair_onfly(hipStream_t s, const ParticleSet& tgt, const ParticleSet* src0, const double* q0,
                       const ParticleSet* src1, const double* q1, const RealGeom& rg, double* phi, double* E,
                       bool field_single, unsigned long long* npairs, const float4* tab0, const float4* tab1) {
  if (tgt.n == 0) return;
  if (src1 && src1->n == 0) src1 = nullptr;
  if (src0 && src0->n == 0) {
    src0 = src1;
    q0 = q1;
    tab0 = tab1;
    src1 = nullptr;
  }
  if (!src0) return;
  require(src0->n < (int64_t(1) << kSetBit) && (!src1 || src1->n < (int64_t(1) << kSetBit)),
          "too many particles in one set for the pair traversal");
  auto sorted_q = [&](const ParticleSet& ps, const double* q, const float4* tab) {
    ParticleSet& m = const_cast<ParticleSet&>(ps);
    m.qsorted.ensure(std::max<int64_t>(ps.n, 1));
    m.qsortedf.ensure(std::max<int64_t>(ps.n, 1));
    hipLaunchKernelGGL(sort_charges_kernel, dim3(nblk(ps.n, 256)), dim3(256), 0, s, ps.idx.get(), q, ps.n,
                       m.qsorted.get(), m.qsortedf.get());
    PE_CHECK_LAUNCH();
    return src_of(ps, m.qsorted.get(), m.qsortedf.get(), tab);
  };
  const SrcSet a = sorted_q(*src0, q0, tab0);
  const SrcSet b = src1 ? sorted_q(*src1, q1, tab1) : a;
  const int nsrc = src1 ? 2 : 1;
  PairOut out{};
  out.phi = phi;
  out.E = E;
  out.npairs = npairs;
  if (!E)
    launch_queue<MODE_POT, T, T>(s, tgt, a, b, nsrc, rg, out);
  else if (field_single)
    launch_queue<MODE_FIELD, T, float>(s, tgt, a, b, nsrc, rg, out);
  else
    launch_queue<MODE_FIELD, T, T>(s, tgt, a, b, nsrc, rg, out);
}

// erfcx = exp(x^2) erfc(x) satisfies y' = 2 x y - 2/sqrt(pi); differentiating
// n times gives y^(n+1) = 2 x y^(n) + 2 n y^(n-1), so the Taylor coefficients
// e_n = y^(n)(x0)/n! about a midpoint x0 follow from erfcx(x0) by
//   e_1 = 2 x0 e_0 - 2/sqrt(pi),  (n+1) e_(n+1) = 2 x0 e_n + 2 e_(n-1).
// Degree 7 over half-widths of 1/8 leaves a truncation below 2e-9.
void build_erfcx_table(hipStream_t s, DevBuf<float>& tab) {
  constexpr int per = kErfcxDeg + 1;
  std::vector<float> h((size_t)kErfcxPieces * per);
  for (int k = 0; k < kErfcxPieces; ++k) {
    const double x0 = (k + 0.5) / (double)kErfcxInvWidth;
    double e[per];
    e[0] = std::exp(x0 * x0) * std::erfc(x0);
    e[1] = 2.0 * x0 * e[0] - kTwoOverSqrtPi;
    for (int n = 1; n + 1 < per; ++n) e[n + 1] = (2.0 * x0 * e[n] + 2.0 * e[n - 1]) / (n + 1);
    for (int n = 0; n < per; ++n) h[(size_t)k * per + n] = (float)e[n];
  }
  tab.ensure(h.size());
  PE_HIP(hipMemcpyAsync(tab.get(), h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, s));
  PE_HIP(hipStreamSynchronize(s));
}

namespace {

// R(r) and dR/dr of the Gaussian-regularized split, in double (r >= 0;
// R(0) is the limit c (2/sqrt pi)(b - xi), where the slope is zero).
void gauss_pair(double r, double b, double xi, double c, double& R, double& dR) {
  if (r < 1e-300) {
    R = c * kTwoOverSqrtPi * (b - xi);
    dR = 0.0;
    return;
  }
  const double D = std::erf(b * r) - std::erf(xi * r);
  const double Dp = kTwoOverSqrtPi * (b * std::exp(-b * b * r * r) - xi * std::exp(-xi * xi * r * r));
  R = c * D / r;
  dR = c * (Dp * r - D) / (r * r);
}

}  // namespace

bool build_pair_table(const RealGeom& rg, double s2, float* out) {
  if (rg.reg != PE_REG_GAUSSIAN || !(s2 > 0.0) || !(rg.rc2 > 0.0)) return false;
  constexpr int K = kPairTabPieces, N = 7;  // N coefficients of 8 stored
  const double rc = std::sqrt(rg.rc2), h = rc / K;
  const double b = 1.0 / std::sqrt(2.0 * s2), xi = rg.xi, c = kInv4Pi / rg.eps;
  double err_v = 0.0, err_d = 0.0, max_v = 0.0, max_d = 0.0;
  for (int k = 0; k < K; ++k) {
    const double mid = (k + 0.5) * h;
    // interpolation at the N Chebyshev points of the piece: Chebyshev
    // coefficients, then the same polynomial in powers of t
    double f[N], cc[N], mono[N] = {};
    for (int i = 0; i < N; ++i) {
      double dR;
      gauss_pair(mid + 0.5 * h * std::cos(kPi * (i + 0.5) / N), b, xi, c, f[i], dR);
    }
    for (int m = 0; m < N; ++m) {
      double a = 0.0;
      for (int i = 0; i < N; ++i) a += f[i] * std::cos(kPi * m * (i + 0.5) / N);
      cc[m] = a * (m == 0 ? 1.0 : 2.0) / N;
    }
    // T_0 = 1, T_1 = t, T_(m+1) = 2 t T_m - T_(m-1), as coefficient vectors
    double Tp[N] = {}, Tc[N] = {}, Tn[N];
    Tp[0] = 1.0;
    Tc[1] = 1.0;
    for (int j = 0; j < N; ++j) mono[j] = cc[0] * Tp[j] + cc[1] * Tc[j];
    for (int m = 2; m < N; ++m) {
      for (int j = 0; j < N; ++j) Tn[j] = (j > 0 ? 2.0 * Tc[j - 1] : 0.0) - Tp[j];
      for (int j = 0; j < N; ++j) {
        mono[j] += cc[m] * Tn[j];
        Tp[j] = Tc[j];
        Tc[j] = Tn[j];
      }
    }
    float* o = out + (size_t)8 * k;
    for (int j = 0; j < 8; ++j) o[j] = j < N ? (float)mono[j] : 0.0f;
    // the rounded coefficients against the closed form, ends of the piece included
    for (int i = 0; i <= 17; ++i) {
      const double t = -1.0 + 2.0 * i / 17.0;
      double v = o[N - 1], d = 0.0;
      for (int j = N - 2; j >= 0; --j) {
        d = d * t + v;
        v = v * t + o[j];
      }
      double R, dR;
      gauss_pair(mid + 0.5 * h * t, b, xi, c, R, dR);
      err_v = std::max(err_v, std::fabs(v - R));
      err_d = std::max(err_d, std::fabs(d * 2.0 / h - dR));
      max_v = std::max(max_v, std::fabs(R));
      max_d = std::max(max_d, std::fabs(dR));
    }
  }
  return err_v <= 1e-7 * max_v && err_d <= 1e-7 * max_d;
}

void update_pair_tables(hipStream_t s, PairTables& pt, const RealGeom& rg, const ParticleSet& beads,
                        const ParticleSet& ions) {
  const double key[6] = {rg.xi, rg.eps, rg.rc2, (double)rg.reg, beads.sig_uniform, ions.sig_uniform};
  if (pt.built && std::equal(key, key + 6, pt.key)) return;
  std::copy(key, key + 6, pt.key);
  pt.built = true;
  const double sg[2] = {beads.sig_uniform, ions.sig_uniform};
  std::vector<float> h;
  std::vector<double> s2_of;  // per slot
  for (int t = 0; t < 2; ++t)
    for (int u = 0; u < 2; ++u) {
      pt.slot[t][u] = -1;
      if (!(sg[t] > 0.0 && sg[u] > 0.0)) continue;
      const double s2 = sg[t] * sg[t] + sg[u] * sg[u];
      const auto it = std::find(s2_of.begin(), s2_of.end(), s2);
      if (it != s2_of.end()) {
        pt.slot[t][u] = (int)(it - s2_of.begin());
        continue;
      }
      h.resize(h.size() + kPairTabFloats);
      if (build_pair_table(rg, s2, h.data() + h.size() - kPairTabFloats)) {
        pt.slot[t][u] = (int)s2_of.size();
        s2_of.push_back(s2);
      } else {
        h.resize(h.size() - kPairTabFloats);
      }
    }
  if (h.empty()) return;
  pt.buf.ensure(h.size());
  PE_HIP(hipMemcpyAsync(pt.buf.get(), h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, s));
  PE_HIP(hipStreamSynchronize(s));
}

template void launch_spmv_add<float>(hipStream_t, pe_context*, const double*, double*);
template void launch_spmv_add<double>(hipStream_t, pe_context*, const double*, double*);
template void launch_pair_onfly<float>(hipStream_t, const ParticleSet&, const ParticleSet*, const double*,
                                       const ParticleSet*, const double*, const RealGeom&, double*, double*, bool,
                                       unsigned long long*, const float4*, const float4*);
template void launch_pair_onfly<double>(hipStream_t, const ParticleSet&, const ParticleSet*, const double*,
                                        const ParticleSet*, const double*, const RealGeom&, double*, double*, bool,
                                        unsigned long long*, const float4*, const float4*);

}  // namespace pe
