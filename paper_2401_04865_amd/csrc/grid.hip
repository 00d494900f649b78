// Gaussian spreading and contraction (section "Spectral Ewald
// implementation", steps 2 and 6; window of section "Wave-space sum").
//
// Contraction (single precision): per home tile (the tile holding a
// particle's first support point), the reachable grid region is staged in LDS
// once and contracted by groups of 16 lanes, one particle each.  In double,
// or where that region does not fit in LDS, one 64-lane wavefront per
// particle: lanes 0..3P-1
// first evaluate the separable window factors w_x[j], w_y[j], w_z[j] (3P
// exponentials per particle instead of P^3) and the wrapped grid indices into
// LDS; then the wavefront sweeps the P x P (y,z) lines of the support, lane t
// owning line (t / P, t % P) and looping over the P x-points, and reduces
// across lanes.
//
// Support (the P closest grid points per axis): even P takes
// m0-P/2+1 .. m0+P/2 with m0 = floor(x/h); odd P is centred on rint(x/h).
// Index and displacement are computed in double for both precisions, so
// the float and double paths use the same support.
#include <algorithm>
#include <climits>
#include <vector>

#include "pe_internal.hpp"
#include "vector.hpp"

namespace pe {

namespace {

constexpr int kWaves = 4;      // particles per 256-thread block
constexpr int kMaxP = 16;

// Support start m0 (unwrapped; positions are already wrapped into the box, so
// m0 lies in [1 - P, N)) and its offset delta = m0 - x / h on one axis.  The
// displacement of support point j is d_j = (j + delta) h.
__device__ __forceinline__ int support_start(double x, double inv_h, int P, double& delta) {
  const double u = x * inv_h;
  const double m0 = (P & 1) ? rint(u) - (double)((P - 1) / 2) : floor(u) - (double)(P / 2 - 1);
  delta = m0 - u;
  return (int)m0;
}

// The value of axis ax (per lane) among three uniform ones, by selects: an
// index into the by-value geometry struct would read the kernel arguments
// from memory at every use.
template <typename V>
__device__ __forceinline__ V sel3(int ax, V a, V b, V c) {
  return ax == 0 ? a : (ax == 1 ? b : c);
}

// m in [-N, 2N) -> [0, N)
__device__ __forceinline__ int wrap_idx(int m, int N) {
  m = m < 0 ? m + N : m;
  return m >= N ? m - N : m;
}

// Window factor w(d_j) = wnorm exp(-wexp d_j^2) of support point j.
template <typename T>
__device__ __forceinline__ T window(const GridGeom& g, int ax, int j, double delta) {
  const double dj = ((double)j + delta) * sel3(ax, g.h[0], g.h[1], g.h[2]);
  return (T)g.wnorm * exp((T)(-g.wexp * dj * dj));
}

template <typename T>
__device__ __forceinline__ void window_setup(const double4 p, const GridGeom& g, int lane,
                                             T* w_s, int* i_s, T* d_s) {
  const int P = g.P;
  if (lane < 3 * P) {
    const int ax = lane / P;
    const int j = lane - ax * P;
    const double x = ax == 0 ? p.x : (ax == 1 ? p.y : p.z);
    double delta;
    const int m0 = support_start(x, sel3(ax, g.inv_h[0], g.inv_h[1], g.inv_h[2]), P, delta);
    w_s[lane] = window<T>(g, ax, j, delta);
    i_s[lane] = wrap_idx(m0 + j, sel3(ax, g.N[0], g.N[1], g.N[2]));
    if (d_s) d_s[lane] = (T)(((double)j + delta) * sel3(ax, g.h[0], g.h[1], g.h[2]));
  }
}

// ------------------------------------------------------------------ spread
//
// Tile-binned spreading.  The grid is cut into tiles of kTile^3 points; for
// every tile, set_system lists the particles whose support overlaps it (a
// particle overlaps about 8 tiles at P = 8).  The tile is written to HBM
// once, with no atomics; every tile is written (empty ones with zeros), so
// the grid needs no clearing between products.  Requires mesh >= P + 8 per
// axis, so a support never reaches the same tile from both sides.

constexpr int kTile = 8;
constexpr int kTile3 = kTile * kTile * kTile;

// Distinct tiles (per axis) touched by the support of a particle; returns count (<= 4).
__device__ __forceinline__ int axis_tiles(int m0, int P, int N, int* t) {
  int n = 0;
  int last = -1;
  for (int j = 0; j < P; ++j) {
    const int tile = wrap_idx(m0 + j, N) / kTile;
    if (tile != last) {
      bool seen = false;
      for (int k = 0; k < n; ++k) seen |= (t[k] == tile);
      if (!seen && n < 4) t[n++] = tile;
      last = tile;
    }
  }
  return n;
}

__device__ __forceinline__ int axis_start(double x, double inv_h, int P) {
  double delta;
  return support_start(x, inv_h, P, delta);
}

// Tiles a particle's support overlaps, per axis, in ascending order.
__device__ __forceinline__ int sorted_axis_tiles(double x, double inv_h, int P, int N, int* t) {
  const int n = axis_tiles(axis_start(x, inv_h, P), P, N, t);
  for (int a = 1; a < n; ++a)
    for (int b = a; b > 0 && t[b - 1] > t[b]; --b) {
      const int u = t[b];
      t[b] = t[b - 1];
      t[b - 1] = u;
    }
  return n;
}

// Tile lists with one atomic per distinct tile of a wavefront: every lane
// walks its tiles (x, y, z tile products) in ascending order and, round by
// round, the lanes whose next tile is the wavefront's smallest pending tile
// join one atomic (the particles of a wavefront are neighbours in the cell
// order, so they share most of their tiles).  FILL: each joining lane takes
// the slot base + its rank among the joining lanes.
template <bool FILL>
__global__ void __launch_bounds__(256) tile_list_kernel(const double4* __restrict__ pos, int64_t n, GridGeom g,
                                                        int* __restrict__ cursor, int* __restrict__ entries) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int tx[4], ty[4], tz[4];
  int nx = 0, ny = 0, nz = 0;
  if (i < n) {
    const double4 p = pos[i];
    nx = sorted_axis_tiles(p.x, g.inv_h[0], g.P, g.N[0], tx);
    ny = sorted_axis_tiles(p.y, g.inv_h[1], g.P, g.N[1], ty);
    nz = sorted_axis_tiles(p.z, g.inv_h[2], g.P, g.N[2], tz);
  }
  int a = 0, b = 0, c = 0;  // next (x, y, z) tile of this lane; done when a == nx
  for (;;) {
    const int mine = a < nx ? (tx[a] * g.ntile[1] + ty[b]) * g.ntile[2] + tz[c] : INT_MAX;
    int key = mine;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) key = min(key, __shfl_xor(key, o, 64));
    if (key == INT_MAX) break;
    const bool join = mine == key;
    const unsigned long long m = __ballot(join);
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&cursor[key], __popcll(m));
    if (FILL) {
      base = __shfl(base, leader, 64);
      if (join) entries[base + __popcll(m & ((1ull << lane) - 1ull))] = (int)i;
    }
    if (join) {
      if (++c == nz) {
        c = 0;
        if (++b == ny) {
          b = 0;
          ++a;
        }
      }
    }
  }
}

// Home tile of a particle: the tile that holds its first support point.
__device__ __forceinline__ int home_tile(const double4 p, const GridGeom& g) {
  const int hx = wrap_idx(axis_start(p.x, g.inv_h[0], g.P), g.N[0]) / kTile;
  const int hy = wrap_idx(axis_start(p.y, g.inv_h[1], g.P), g.N[1]) / kTile;
  const int hz = wrap_idx(axis_start(p.z, g.inv_h[2], g.P), g.N[2]) / kTile;
  return (hx * g.ntile[1] + hy) * g.ntile[2] + hz;
}

__global__ void home_count_kernel(const double4* __restrict__ pos, int64_t n, GridGeom g, int* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicAdd(&count[home_tile(pos[i], g)], 1);
}

__global__ void home_fill_kernel(const double4* __restrict__ pos, int64_t n, GridGeom g, int* __restrict__ cursor,
                                 int* __restrict__ entries) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  entries[atomicAdd(&cursor[home_tile(pos[i], g)], 1)] = (int)i;
}

// Charges in the particle set's sorted order (one load per staged particle
// instead of two dependent ones).
__global__ void sorted_charges_kernel(const int* __restrict__ idx, const double* __restrict__ q, int64_t n,
                                      double* __restrict__ qs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) qs[i] = q[idx[i]];
}

// One workgroup per column of four tiles along z; wavefront w owns tile
// (ux, uy, 4 bz + w) and walks that tile's particle list on its own, 21
// particles at a time: lanes 0..62, one per (particle, axis), stage the eight
// tile-local window factors (f_x[a] q, f_y[b], f_z[c], zero where the support
// misses the tile) in the wavefront's LDS slice; then lane (a, b) adds
// q f_x[a] f_y[b] f_z[c] into the z-pencil (a, b, 0..7) it holds in
// registers.  No workgroup barrier inside the loop.  At the end the four
// tiles meet in LDS and the column is written once, 32 values of z per row
// (whole 128-byte lines in single precision, 16-byte stores where the mesh
// allows), with no atomics; every tile is written (empty ones with zeros), so
// the grid needs no clearing between products.  The lists are sorted, so the
// result is the same bit for bit on every run.
constexpr int kWaveChunk = 21;

// Single-precision window factors of a particle set, once per configuration
// (positions fixed, charges not), for supports of at most 8 points on meshes
// of whole tiles (every N a multiple of 8).  Such a support covers a tile
// from slot m mod 8 on (m: wrapped index of support point 0, the home tile)
// and, when it does not start on slot 0, the next tile up to slot m mod 8
// (exclusive).  Both are the eight factors rotated by m mod 8,
// rot[loc] = f[(loc - m) mod 8], masked: so rot is stored, per particle
// (sorted order) and axis, with m.  f[j] = wnorm exp(-wexp ((j + delta) h)^2)
// for j < P (zero up to 8), in the float arithmetic the spreading kernel
// applies.  Planar layout: wf[(2 ax + h) n + i] holds slots 4h..4h+3 of
// particle i, so consecutive threads store consecutive vectors.
__global__ void __launch_bounds__(256) window_factors_kernel(const double4* __restrict__ pos, int64_t n, GridGeom g,
                                                             float4* __restrict__ wf, int4* __restrict__ ws) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 p = pos[i];
  const float we = (float)g.wexp, wn = (float)g.wnorm;
  int m[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const double x = ax == 0 ? p.x : (ax == 1 ? p.y : p.z);
    double delta;
    m[ax] = wrap_idx(support_start(x, g.inv_h[ax], g.P, delta), g.N[ax]);
    const float hf = (float)g.h[ax], df = (float)delta;
    float f[kTile];
#pragma unroll
    for (int loc = 0; loc < kTile; ++loc) {
      const int j = (loc - m[ax]) & (kTile - 1);
      const float d = ((float)j + df) * hf;
      f[loc] = j < g.P ? wn * __expf(-we * d * d) : 0.0f;
    }
    wf[(2 * ax) * n + i] = make_float4(f[0], f[1], f[2], f[3]);
    wf[(2 * ax + 1) * n + i] = make_float4(f[4], f[5], f[6], f[7]);
  }
  ws[i] = make_int4(m[0], m[1], m[2], 0);
}

template <typename T> struct Vec16;
template <> struct Vec16<float> {
  using type = float4;
  static __device__ __forceinline__ type add(type a, type b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
  }
};
template <> struct Vec16<double> {
  using type = double2;
  static __device__ __forceinline__ type add(type a, type b) { return make_double2(a.x + b.x, a.y + b.y); }
};

// HOME: the particle list of a tile is the concatenation of the sorted home
// lists of the tiles (ux - dx, uy - dy, uz - dz), d in {0, 1}^3 (tile_start /
// entries are then the home lists); particles whose support misses the tile
// get zero factors.  Eight wavefronts per SIMD (at most 64 VGPRs, no spills;
// at most 16 KB of LDS per workgroup leaves room for eight workgroups per CU): the
// loop waits on its list and position loads, and more resident wavefronts hide
// them (bead spread 198 -> 189 us on the 256^3 mesh).
// PRE (single precision, P <= 8, N a multiple of 8 on every axis; nset
// particles in the set): the factors come rotated from window_factors_kernel; a staging lane keeps slot
// loc where loc >= s0 in the home tile (s0 >= 0, the tile-local position of
// support point 0) or loc < s0 + 8 in the next one, times the charge (x
// axis): eight selects instead of eight exponentials (staging drops from
// about 120 vector instructions per round to about 30).  Its rows are 12
// floats, which spreads the row stores of a wavefront over more LDS banks.
// Double precision (used for the ions' home lists when a double pass spreads
// them) takes the window factors in double and holds four wavefronts per
// SIMD (the z-pencil is twice as wide in registers).
template <typename T, bool HOME, bool PRE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4))) spread_tile_kernel(const double4* __restrict__ pos,
                                                          const double* __restrict__ qs,
                                                          const int* __restrict__ tile_start,
                                                          const int* __restrict__ entries,
                                                          const float4* __restrict__ wfac,
                                                          const int* __restrict__ wsta, int64_t nset,
                                                          T* __restrict__ grid, GridGeom g, int accumulate) {
  static_assert(!PRE || sizeof(T) == 4, "precomputed factors are single precision");
  constexpr int kRow = PRE ? 12 : kTile;  // LDS slots per staged (particle, axis)
  constexpr int kSlice = kWaveChunk * 3 * kRow;
  constexpr int kStage = kWaves * kSlice;
  constexpr int kColLen = kWaves * kTile;                  // z values of the column
  constexpr int kCol = kTile * kTile * kColLen;
  // staged rows during the loop, the column (a, b, z) after it
  __shared__ __align__(16) T smem[kStage > kCol ? kStage : kCol];
  const int nbz = (g.ntile[2] + kWaves - 1) / kWaves;
  const int bz = blockIdx.x % nbz;
  const int uy = (blockIdx.x / nbz) % g.ntile[1];
  const int ux = blockIdx.x / (nbz * g.ntile[1]);
  const int P = g.P;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int uz = kWaves * bz + wv;
  const int pa = lane >> 3, pb = lane & 7;
  T acc[kTile];
#pragma unroll
  for (int c = 0; c < kTile; ++c) acc[c] = 0;
  if (uz < g.ntile[2]) {
    int e0, e1;
    // HOME: segment d of the virtual list starts at my_b in the home lists
    // and at my_p in the list on lane d < 8; every lane keeps the list
    // offsets hp[d] to find a position's segment
    int hp[9];
    int my_b = 0, my_p = 0;
    if constexpr (HOME) {
      int my_n = 0;
      if (lane < 8) {
        const int dx = lane >> 2, dy = (lane >> 1) & 1, dz = lane & 1;
        // a neighbour index that wraps onto the tile itself is not a second source
        const bool dup = (dx && g.ntile[0] < 2) || (dy && g.ntile[1] < 2) || (dz && g.ntile[2] < 2);
        if (!dup) {
          const int tx = ux - dx < 0 ? ux - dx + g.ntile[0] : ux - dx;
          const int ty = uy - dy < 0 ? uy - dy + g.ntile[1] : uy - dy;
          const int tz = uz - dz < 0 ? uz - dz + g.ntile[2] : uz - dz;
          const int t = (tx * g.ntile[1] + ty) * g.ntile[2] + tz;
          my_b = tile_start[t];
          my_n = tile_start[t + 1] - my_b;
        }
      }
      hp[0] = 0;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        hp[d + 1] = hp[d] + __shfl(my_n, d, 64);
        if (lane == d) my_p = hp[d];
      }
      e0 = 0;
      e1 = hp[8];
    } else {
      const int tid = (ux * g.ntile[1] + uy) * g.ntile[2] + uz;
      e0 = tile_start[tid];
      e1 = tile_start[tid + 1];
    }
    T* fw = smem + wv * kSlice;  // row (c, ax) at fw + (3 c + ax) kRow
    // staging lane: particle c3 of the round, axis ax3.  Loads run ahead of
    // use: the entries two rounds ahead, the coordinate (or the factors) and
    // charge one round ahead, so their latency overlaps the current round's
    // work.
    const int c3 = lane / 3, ax3 = lane - 3 * (lane / 3);
    const bool stager = lane < 3 * kWaveChunk;
    const int N = sel3(ax3, g.N[0], g.N[1], g.N[2]);
    const double ih3 = sel3(ax3, g.inv_h[0], g.inv_h[1], g.inv_h[2]);
    const double h3 = sel3(ax3, g.h[0], g.h[1], g.h[2]);
    const int u = ax3 == 0 ? ux : (ax3 == 1 ? uy : uz);
    T* const srow = fw + (3 * c3 + ax3) * kRow;
    // (called with every lane of the wavefront active)
    auto entry_at = [&](int c0) {
      const int k = c0 + c3;
      if constexpr (HOME) {
        int d = 0;
#pragma unroll
        for (int m = 1; m < 8; ++m) d += k >= hp[m] ? 1 : 0;
        const int b = __shfl(my_b, d, 64), p0 = __shfl(my_p, d, 64);
        if (!stager || k >= e1) return -1;
        return entries[b + (k - p0)];
      } else {
        if (!stager || k >= e1) return -1;
        return entries[k];
      }
    };
    // what a staging lane reads per round
    struct Stage {
      double x = 0, q = 1;                        // coordinate, charge
      float4 fa = {0, 0, 0, 0}, fb = {0, 0, 0, 0};  // PRE: factors 0..7
      int mw = 0;                                 // PRE: wrapped index of support point 0
    };
    auto fetch = [&](int i, Stage& st) {
      if (i < 0) return;
      if constexpr (PRE) {
        st.fa = wfac[(2 * ax3) * nset + i];
        st.fb = wfac[(2 * ax3 + 1) * nset + i];
        st.mw = wsta[4 * i + ax3];
      } else {
        st.x = reinterpret_cast<const double*>(pos + i)[ax3];
      }
      if (ax3 == 0) st.q = qs[i];
    };
    int i1 = entry_at(e0), i2 = entry_at(e0 + kWaveChunk);
    Stage st1;
    fetch(i1, st1);
    for (int c0 = e0; c0 < e1; c0 += kWaveChunk) {
      const int nc = min(kWaveChunk, e1 - c0);
      const int i3 = entry_at(c0 + 2 * kWaveChunk);
      Stage st2;
      fetch(i2, st2);
      if (i1 >= 0) {
        if constexpr (PRE) {
          int s0 = st1.mw - kTile * u;
          if (s0 > kTile - 1) s0 -= N;
          if (s0 < 1 - P) s0 += N;
          // s0 outside [1 - P, 7]: a neighbour's home particle whose support
          // stops short of this tile (all zero)
          const bool seen = s0 >= 1 - P && s0 <= kTile - 1;
          const int mr = s0 & (kTile - 1);
          const bool home = s0 >= 0;
          const float qf = seen ? (float)st1.q : 0.0f;
          const float f[kTile] = {st1.fa.x, st1.fa.y, st1.fa.z, st1.fa.w, st1.fb.x, st1.fb.y, st1.fb.z, st1.fb.w};
#pragma unroll
          for (int loc = 0; loc < kTile; ++loc) srow[loc] = (loc >= mr) == home ? f[loc] * qf : 0.0f;
        } else {
          double delta;
          const int m0 = support_start(st1.x, ih3, P, delta);
          // tile-local position of support point 0, taken in [1 - P, kTile - 1]
          int s0 = wrap_idx(m0, N) - kTile * u;
          if (s0 > kTile - 1) s0 -= N;
          if (s0 < 1 - P) s0 += N;
          if constexpr (sizeof(T) == 4) {
            // single precision once the support is placed: the displacement
            // (j + delta) h is below P h, so float keeps it to rounding and the
            // exponential to a few ulp
            const float hf = (float)h3, df = (float)delta, we = (float)g.wexp;
            const float wn = (float)g.wnorm * (float)st1.q;
#pragma unroll
            for (int loc = 0; loc < kTile; ++loc) {
              const int j = loc - s0;
              const float d = ((float)j + df) * hf;
              srow[loc] = (j >= 0 && j < P) ? (T)(wn * __expf(-we * d * d)) : (T)0;
            }
          } else {
            const double wn = g.wnorm * st1.q;
#pragma unroll
            for (int loc = 0; loc < kTile; ++loc) {
              const int j = loc - s0;
              const double d = ((double)j + delta) * h3;
              srow[loc] = (j >= 0 && j < P) ? (T)(wn * exp(-g.wexp * d * d)) : (T)0;
            }
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int c = 0; c < nc; ++c) {
        const T* r = fw + 3 * c * kRow;
        const T coef = r[pa] * r[kRow + pb];
#pragma unroll
        for (int z = 0; z < kTile; ++z) acc[z] += coef * r[2 * kRow + z];
      }
      // the slice is restaged next round
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      i1 = i2;
      i2 = i3;
      st1 = st2;
    }
  }
  __syncthreads();  // every wavefront is done with its staged rows
  T* col = smem;    // (a, b, z of the column)
#pragma unroll
  for (int z = 0; z < kTile; ++z) col[(pa * kTile + pb) * kColLen + kTile * wv + z] = acc[z];
  __syncthreads();
  const int zlen = min(kColLen, g.N[2] - kColLen * bz);
  constexpr int kV = 16 / (int)sizeof(T);
  if (g.N[2] % kV == 0) {
    // rows (a, b) of up to 32 z values in 16-byte vectors (zlen and every
    // offset are multiples of kV)
    using V = typename Vec16<T>::type;
    for (int k = threadIdx.x; k < kCol / kV; k += blockDim.x) {
      const int zz = (k % (kColLen / kV)) * kV;
      const int row = k / (kColLen / kV);
      const int a = row / kTile, b = row % kTile;
      const int gx = kTile * ux + a, gy = kTile * uy + b, gz = kColLen * bz + zz;
      if (gx < g.N[0] && gy < g.N[1] && zz < zlen) {
        const int64_t o = ((int64_t)gx * g.N[1] + gy) * g.N[2] + gz;
        V v = *reinterpret_cast<const V*>(col + row * kColLen + zz);
        V* dst = reinterpret_cast<V*>(grid + o);
        if (accumulate) v = Vec16<T>::add(*dst, v);
        *dst = v;
      }
    }
  } else {
    // rows (a, b) of up to 32 z values: 8 threads per row, 4 values each
    for (int k = threadIdx.x; k < kCol; k += blockDim.x) {
      const int zz = k % kColLen;
      const int row = k / kColLen;
      const int a = row / kTile, b = row % kTile;
      const int gx = kTile * ux + a, gy = kTile * uy + b, gz = kColLen * bz + zz;
      if (gx < g.N[0] && gy < g.N[1] && zz < zlen) {
        const int64_t o = ((int64_t)gx * g.N[1] + gy) * g.N[2] + gz;
        const T v = col[row * kColLen + zz];
        grid[o] = accumulate ? grid[o] + v : v;
      }
    }
  }
}

// Double precision: one workgroup (four wavefronts) per tile.  The tile's
// particle list is
// processed in chunks of kChunk: one thread per (particle, axis) stages the
// eight tile-local window factors (f_x[a] q, f_y[b], f_z[c], zero where the
// support misses the tile) in LDS.  Lane (a, b) of a wavefront owns the
// z-pencil (a, b, 0..7) of the tile in eight registers and adds
// q f_x[a] f_y[b] f_z[c] for the particles of its share of the chunk.  The four
// partial tiles are summed in a fixed order and the tile is written once.
// No atomics; the lists are sorted, so the result is the same bit for bit on
// every run.
constexpr int kChunk = 64;

template <typename T>
__global__ void __launch_bounds__(256) spread_block_kernel(const double4* __restrict__ pos,
                                                          const int* __restrict__ idx,
                                                          const double* __restrict__ q,
                                                          const int* __restrict__ tile_start,
                                                          const int* __restrict__ entries,
                                                          T* __restrict__ grid, GridGeom g, int accumulate) {
  __shared__ T f_s[kChunk][3][kTile];
  __shared__ T red[kWaves][kTile3];
  const int tid = blockIdx.x;
  const int uz = tid % g.ntile[2];
  const int uy = (tid / g.ntile[2]) % g.ntile[1];
  const int ux = tid / (g.ntile[2] * g.ntile[1]);
  const int P = g.P;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int pa = lane >> 3, pb = lane & 7;
  T acc[kTile];
#pragma unroll
  for (int c = 0; c < kTile; ++c) acc[c] = 0;
  const int e0 = tile_start[tid], e1 = tile_start[tid + 1];
  for (int c0 = e0; c0 < e1; c0 += kChunk) {
    const int nc = min(kChunk, e1 - c0);
    // one thread per (particle, axis): the eight tile-local factors
    if ((int)threadIdx.x < 3 * nc) {
      const int c = threadIdx.x / 3;
      const int ax = threadIdx.x - 3 * c;
      const int i = entries[c0 + c];
      const double x = reinterpret_cast<const double*>(pos + i)[ax];
      double delta;
      const int m0 = support_start(x, sel3(ax, g.inv_h[0], g.inv_h[1], g.inv_h[2]), P, delta);
      const int N = sel3(ax, g.N[0], g.N[1], g.N[2]);
      const int u = ax == 0 ? ux : (ax == 1 ? uy : uz);
      // tile-local position of support point 0, taken in [1 - P, kTile - 1]
      int s0 = wrap_idx(m0, N) - kTile * u;
      if (s0 > kTile - 1) s0 -= N;
      if (s0 < 1 - P) s0 += N;
      const T scale = ax == 0 ? (T)q[idx[i]] : (T)1;
#pragma unroll
      for (int loc = 0; loc < kTile; ++loc) {
        const int j = loc - s0;
        f_s[c][ax][loc] = (j >= 0 && j < P) ? window<T>(g, ax, j, delta) * scale : (T)0;
      }
    }
    __syncthreads();
    for (int c = wv; c < nc; c += kWaves) {
      const T coef = f_s[c][0][pa] * f_s[c][1][pb];
#pragma unroll
      for (int z = 0; z < kTile; ++z) acc[z] += coef * f_s[c][2][z];
    }
    __syncthreads();
  }
#pragma unroll
  for (int z = 0; z < kTile; ++z) red[wv][lane * kTile + z] = acc[z];
  __syncthreads();
  for (int k = threadIdx.x; k < kTile3; k += blockDim.x) {
    const T v = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    const int a = k / (kTile * kTile), b = (k / kTile) % kTile, c = k % kTile;
    const int gx = kTile * ux + a, gy = kTile * uy + b, gz = kTile * uz + c;
    if (gx < g.N[0] && gy < g.N[1] && gz < g.N[2]) {
      const int64_t o = ((int64_t)gx * g.N[1] + gy) * g.N[2] + gz;
      grid[o] = accumulate ? grid[o] + v : v;
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

// Tile-staged contraction: one workgroup per home tile.  The grid region the
// supports of the tile's home particles can reach, (kTile + P - 1)^3 points
// from the tile's first point, is read once into LDS; then each group of 16
// lanes contracts one particle from LDS (four per wavefront), lane s taking
// the (y, z) lines s, s + 16, ... of the support and looping over x, and the
// group reduces with lane shuffles.  The result is the same sum as the
// per-particle kernel, in another order.  PP > 0 fixes P at compile time
// (the common support): the lines are unrolled, their P loads issued
// together, and the x factors held in registers.
constexpr int kGatherLDS = 48 * 1024;
constexpr int kGatherRow = 16;  // LDS row of the region with a compile-time support (P = 8)

// Single precision is held to 64 VGPRs (the field variant needs 65 unforced),
// eight wavefronts per SIMD; its LDS region of 15^3 floats still lets eight
// workgroups share a CU.  Double keeps the compiler's choice.
template <typename T, bool FIELD, int PP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1))) gather_tile_kernel(const double4* __restrict__ pos,
                                                          const int* __restrict__ idx,
                                                          const int* __restrict__ home_start,
                                                          const int* __restrict__ home_entries,
                                                          const int* __restrict__ home_tiles,
                                                          const T* __restrict__ grid, GridGeom g,
                                                          double* __restrict__ phi, double* __restrict__ E,
                                                          int accumulate) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* H = reinterpret_cast<T*>(smem_raw);
  __shared__ T w_s[16][3 * kMaxP];
  __shared__ T d_s[16][3 * kMaxP];
  __shared__ int gidx[3][kTile + kMaxP];  // wrapped grid index of each region plane, per axis
  static_assert(PP == 0 || (PP * PP) % 16 == 0, "lines of the support shared by 16 lanes");
  const int tile = home_tiles[xcd_remap(blockIdx.x, gridDim.x)];
  const int uz = tile % g.ntile[2];
  const int uy = (tile / g.ntile[2]) % g.ntile[1];
  const int ux = tile / (g.ntile[2] * g.ntile[1]);
  const int P = PP > 0 ? PP : g.P;
  const int Hs = kTile + P - 1;
  const int Hs2 = Hs * Hs;
  // LDS row (lx, ly) of the region: Hs z values, padded to 16 with a
  // compile-time support (16-byte aligned rows)
  const int Hrow = PP > 0 ? kGatherRow : Hs;
  const int Hx = Hs * Hrow;  // stride of lx
  static_assert(PP == 0 || kTile + PP - 1 <= kGatherRow, "region rows fit the padded LDS rows");
  if ((int)threadIdx.x < 3 * Hs) {
    const int ax = threadIdx.x / Hs, l = threadIdx.x - ax * Hs;
    const int u = ax == 0 ? ux : (ax == 1 ? uy : uz);
    gidx[ax][l] = wrap_idx(kTile * u + l, sel3(ax, g.N[0], g.N[1], g.N[2]));
  }
  __syncthreads();
  // single precision, a compile-time support, a region that does not wrap in
  // z and 16-byte aligned grid rows: four lanes per region row, each loading
  // four consecutive z values as one 16-byte vector (the 16th value of a row
  // is read and not used); all of a thread's loads are issued before its
  // stores
  constexpr int kVecPasses = PP > 0 ? (((kTile + PP - 1) * (kTile + PP - 1)) + 63) / 64 : 1;
  const bool vec_rows = sizeof(T) == 4 && PP > 0 && g.N[2] % 4 == 0 && kTile * uz + kGatherRow <= g.N[2];
  if constexpr (sizeof(T) == 4 && PP > 0) {
    if (vec_rows) {
      const int q4 = threadIdx.x & 3;
      float4 v[kVecPasses];
#pragma unroll
      for (int u = 0; u < kVecPasses; ++u) {
        const int row = (threadIdx.x >> 2) + 64 * u;
        const int lx = row / Hs;
        const int ly = row - lx * Hs;
        const int64_t o = row < Hs2
                              ? ((int64_t)gidx[0][lx] * g.N[1] + gidx[1][ly]) * g.N[2] + kTile * uz + 4 * q4
                              : 0;
        v[u] = *reinterpret_cast<const float4*>(grid + o);
      }
#pragma unroll
      for (int u = 0; u < kVecPasses; ++u) {
        const int row = (threadIdx.x >> 2) + 64 * u;
        if (row < Hs2) *reinterpret_cast<float4*>(H + row * Hrow + 4 * q4) = v[u];
      }
    }
  }
  // otherwise region rows (lx, ly) of Hs contiguous z values, 16 threads per
  // row (a second pass of 16 only where Hs > 16, which a compile-time P <= 9
  // excludes); eight rows' loads are issued before their stores, so their
  // latencies overlap
  constexpr int kHalves = PP > 0 ? (kTile + PP - 1 + 15) / 16 : 2;
  for (int r0 = threadIdx.x >> 4; r0 < (vec_rows ? 0 : Hs2); r0 += 16 * 8) {
    T v[8][kHalves];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = r0 + 16 * u;
      const int lx = row / Hs;
      const int ly = row - lx * Hs;
      const int64_t rb = row < Hs2 ? ((int64_t)gidx[0][lx] * g.N[1] + gidx[1][ly]) * g.N[2] : 0;
#pragma unroll
      for (int h = 0; h < kHalves; ++h) {
        // every load issued (a point outside the region reads grid[0]), so
        // no branch separates them
        const int lz = (threadIdx.x & 15) + 16 * h;
        const bool ok = row < Hs2 && lz < Hs;
        const T val = grid[ok ? rb + gidx[2][lz] : 0];
        v[u][h] = ok ? val : (T)0;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = r0 + 16 * u;
#pragma unroll
      for (int h = 0; h < kHalves; ++h) {
        const int lz = (threadIdx.x & 15) + 16 * h;
        if (row < Hs2 && lz < Hs) H[row * Hrow + lz] = v[u][h];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sub = lane >> 4, s = lane & 15;
  const int slot = 4 * wv + sub;
  const int e0 = home_start[tile], e1 = home_start[tile + 1];
  // the particle of the next round (entry and position) is loaded while
  // this round's is contracted (not in the single-precision field variant,
  // whose registers that would spill at eight wavefronts per SIMD)
  constexpr bool kAhead = !(FIELD && sizeof(T) == 4);
  int i_next = home_entries[min(e0 + slot, e1 - 1)];
  double4 p_next = pos[i_next];
  for (int base = e0; base < e1; base += 16) {
    const int e = base + slot;
    const bool valid = e < e1;
    const int i = kAhead ? i_next : home_entries[valid ? e : e1 - 1];
    const double4 p = kAhead ? p_next : pos[i];
    if (kAhead && base + 16 < e1) {
      i_next = home_entries[min(e + 16, e1 - 1)];
      p_next = pos[i_next];
    }
    // support of the three axes (placed in double), then the window factors
    // and displacements; in single precision the factors are formed in
    // float, the displacement (j + delta) h being below P h
    double dlx, dly, dlz;
    const int mx = support_start(p.x, g.inv_h[0], P, dlx);
    const int my = support_start(p.y, g.inv_h[1], P, dly);
    const int mz = support_start(p.z, g.inv_h[2], P, dlz);
    auto factor = [&](int k) {
      const int ax = k / P;
      const int j = k - ax * P;
      const double delta = sel3(ax, dlx, dly, dlz);
      const double h = sel3(ax, g.h[0], g.h[1], g.h[2]);
      if constexpr (sizeof(T) == 4) {
        const float d = ((float)j + (float)delta) * (float)h;
        w_s[slot][k] = (float)g.wnorm * __expf(-(float)g.wexp * d * d);
        if (FIELD) d_s[slot][k] = d;
      } else {
        const double d = ((double)j + delta) * h;
        w_s[slot][k] = (T)(g.wnorm * exp(-g.wexp * d * d));
        if (FIELD) d_s[slot][k] = (T)d;
      }
    };
    if constexpr (PP > 0 && kAhead) {
#pragma unroll
      for (int it = 0; it < (3 * PP + 15) / 16; ++it)
        if (s + 16 * it < 3 * PP) factor(s + 16 * it);
    } else {
      for (int k = s; k < 3 * P; k += 16) factor(k);
    }
    // first support point relative to the region origin, per axis
    const int ox = wrap_idx(mx, g.N[0]) - kTile * ux;
    const int oy = wrap_idx(my, g.N[1]) - kTile * uy;
    const int oz = wrap_idx(mz, g.N[2]) - kTile * uz;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const T* wsl = w_s[slot];
    const T* dsl = d_s[slot];
    T acc = 0, axf = 0, ayf = 0, azf = 0;
    if constexpr (PP > 0) {
      T wx[PP], dxv[PP];
#pragma unroll
      for (int j = 0; j < PP; ++j) {
        wx[j] = wsl[j];
        if (FIELD) dxv[j] = dsl[j];
      }
#pragma unroll
      for (int k = 0; k < PP * PP / 16; ++k) {
        const int t = s + 16 * k;
        const int jy = t / PP;
        const int jz = t - jy * PP;
        const T wyz = wsl[PP + jy] * wsl[2 * PP + jz];
        const T* col = H + (ox * Hs + oy + jy) * Hrow + oz + jz;
        T v[PP];
#pragma unroll
        for (int jx = 0; jx < PP; ++jx) v[jx] = col[jx * Hx];
        T lacc = 0, lx = 0;
#pragma unroll
        for (int jx = 0; jx < PP; ++jx) {
          const T u = v[jx] * wx[jx];
          lacc += u;
          if (FIELD) lx += u * dxv[jx];
        }
        acc += lacc * wyz;
        if (FIELD) {
          axf += lx * wyz;
          ayf += lacc * wyz * dsl[PP + jy];
          azf += lacc * wyz * dsl[2 * PP + jz];
        }
      }
    } else {
    for (int t = s; t < P * P; t += 16) {
      const int jy = t / P;
      const int jz = t - jy * P;
      const T wyz = wsl[P + jy] * wsl[2 * P + jz];
      const T* col = H + (ox * Hs + oy + jy) * Hrow + oz + jz;
      T lacc = 0, lx = 0;
      for (int jx = 0; jx < P; ++jx) {
        const T v = col[jx * Hx] * wsl[jx];
        lacc += v;
        if (FIELD) lx += v * dsl[jx];
      }
      acc += lacc * wyz;
      if (FIELD) {
        axf += lx * wyz;
        ayf += lacc * wyz * dsl[P + jy];
        azf += lacc * wyz * dsl[2 * P + jz];
      }
    }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
      acc += __shfl_xor(acc, o, 16);
      if (FIELD) {
        axf += __shfl_xor(axf, o, 16);
        ayf += __shfl_xor(ayf, o, 16);
        azf += __shfl_xor(azf, o, 16);
      }
    }
    if (valid && s == 0) {
      const int oi = idx[i];
      const double ph = (double)acc * (g.h3 / g.eps);
      if (accumulate) phi[oi] += ph; else phi[oi] = ph;
      if (FIELD) {
        const double ex = g.fcoef * (double)axf, ey = g.fcoef * (double)ayf, ez = g.fcoef * (double)azf;
        if (accumulate) {
          E[3 * oi] += ex; E[3 * oi + 1] += ey; E[3 * oi + 2] += ez;
        } else {
          E[3 * oi] = ex; E[3 * oi + 1] = ey; E[3 * oi + 2] = ez;
        }
      }
    }
    // the slot's factors are rewritten next round
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

}  // namespace

namespace {

// Spreading lists of a set (particles overlapping each tile), sorted within
// each tile so the accumulation order is the same on every run.
// Tile lists in two halves around one wait: the counts (and their copy to
// the host), then the offsets on the host, their upload and the fill.
void tile_lists_count(hipStream_t s, ParticleSet& ps, const GridGeom& g) {
  const int nt = g.ntile[0] * g.ntile[1] * g.ntile[2];
  ps.tile_start.ensure(nt + 1);
  ps.tile_count.ensure(2 * (size_t)nt);
  int* tcount = ps.tile_count.get();
  PE_HIP(hipMemsetAsync(tcount, 0, sizeof(int) * nt, s));
  if (ps.n > 0) {
    hipLaunchKernelGGL(tile_list_kernel<false>, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s, ps.pos.get(),
                       ps.n, g, tcount, (int*)nullptr);
    PE_CHECK_LAUNCH();
  }
  int* cnt = ps.h_tcnt.get<int>(nt);
  PE_HIP(hipMemcpyAsync(cnt, tcount, sizeof(int) * nt, hipMemcpyDeviceToHost, s));
}

// (the counts' copy has completed)
void tile_lists_finish(hipStream_t s, ParticleSet& ps, const GridGeom& g) {
  const int nt = g.ntile[0] * g.ntile[1] * g.ntile[2];
  int* tcount = ps.tile_count.get();
  const int* cnt = ps.h_tcnt.get<int>(nt);
  int* start = ps.h_tstart.get<int>((size_t)nt + 1);
  int run = 0, cmax = 0;
  start[0] = 0;
  for (int t = 0; t < nt; ++t) {
    const int k = cnt[t];
    run += k;
    cmax = std::max(cmax, k);
    start[t + 1] = run;
  }
  ps.n_entries = run;
  ps.tile_entries.ensure(std::max<int64_t>(ps.n_entries, 1));
  PE_HIP(hipMemcpyAsync(ps.tile_start.get(), start, sizeof(int) * (nt + 1), hipMemcpyHostToDevice, s));
  PE_HIP(hipMemcpyAsync(tcount, start, sizeof(int) * nt, hipMemcpyHostToDevice, s));
  if (ps.n > 0) {
    hipLaunchKernelGGL(tile_list_kernel<true>, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s, ps.pos.get(),
                       ps.n, g, tcount, ps.tile_entries.get());
    PE_CHECK_LAUNCH();
    launch_segment_sort(s, ps.tile_start.get(), nt, ps.tile_entries.get(), cmax);
  }
  ps.have_tile_lists = true;
}

void build_tile_lists(hipStream_t s, ParticleSet& ps, const GridGeom& g) {
  tile_lists_count(s, ps, g);
  PE_HIP(hipStreamSynchronize(s));
  tile_lists_finish(s, ps, g);
}

}  // namespace

// Home lists of a set (each particle once, under the tile of its first
// support point).  With spread_by_home the lists are sorted and serve the
// single-precision spreading too (a tile's particles are those of the home
// lists of the tile and of its lower neighbours), and the tile lists are
// built only if a double spread asks for them; otherwise the tile lists are
// built here.  A support spans at most two tiles per axis only when P <= 8 and
// every tile is full: a short last tile lets a support run from its lower
// neighbour across it into tile 0, so such meshes keep the tile lists.
void build_tiles(hipStream_t s, ParticleSet& ps, const GridGeom& g, bool spread_by_home) {
  const int nt = g.ntile[0] * g.ntile[1] * g.ntile[2];
  spread_by_home = spread_by_home && g.P <= kTile && g.N[0] % kTile == 0 && g.N[1] % kTile == 0 &&
                   g.N[2] % kTile == 0;
  ps.have_tile_lists = false;
  ps.wfac_valid = false;
  ps.spread_by_home = spread_by_home;
  // the tile lists' counts and the home lists' counts behind one wait
  if (!spread_by_home) tile_lists_count(s, ps, g);
  ps.tile_count.ensure(2 * (size_t)nt);
  int* hcount = ps.tile_count.get() + nt;
  PE_HIP(hipMemsetAsync(hcount, 0, sizeof(int) * nt, s));
  const unsigned nb = (unsigned)((ps.n + 255) / 256);
  if (ps.n > 0) {
    hipLaunchKernelGGL(home_count_kernel, dim3(nb), dim3(256), 0, s, ps.pos.get(), ps.n, g, hcount);
    PE_CHECK_LAUNCH();
  }
  int* cnt = ps.h_hcnt.get<int>(nt);
  PE_HIP(hipMemcpyAsync(cnt, hcount, sizeof(int) * nt, hipMemcpyDeviceToHost, s));
  PE_HIP(hipStreamSynchronize(s));
  if (!spread_by_home) tile_lists_finish(s, ps, g);
  int* hstart = ps.h_hstart.get<int>((size_t)nt + 1);
  int* htiles = ps.h_htiles.get<int>(nt);
  int nht = 0, run = 0, hmax = 0;
  hstart[0] = 0;
  for (int t = 0; t < nt; ++t) {
    const int k = cnt[t];
    run += k;
    hstart[t + 1] = run;
    hmax = std::max(hmax, k);
    if (k) htiles[nht++] = t;
  }
  ps.home_start.ensure(nt + 1);
  ps.home_entries.ensure(std::max<int64_t>(ps.n, 1));
  ps.n_home_tiles = nht;
  ps.home_tiles.ensure(std::max(nht, 1));
  PE_HIP(hipMemcpyAsync(ps.home_start.get(), hstart, sizeof(int) * (nt + 1), hipMemcpyHostToDevice, s));
  PE_HIP(hipMemcpyAsync(hcount, hstart, sizeof(int) * nt, hipMemcpyHostToDevice, s));
  if (nht) PE_HIP(hipMemcpyAsync(ps.home_tiles.get(), htiles, sizeof(int) * nht, hipMemcpyHostToDevice, s));
  if (ps.n > 0) {
    hipLaunchKernelGGL(home_fill_kernel, dim3(nb), dim3(256), 0, s, ps.pos.get(), ps.n, g, hcount,
                       ps.home_entries.get());
    PE_CHECK_LAUNCH();
    if (spread_by_home) launch_segment_sort(s, ps.home_start.get(), nt, ps.home_entries.get(), hmax);
  }
}

bool window_factors_apply(const GridGeom& g) {
  return g.P <= kTile && g.N[0] % kTile == 0 && g.N[1] % kTile == 0 && g.N[2] % kTile == 0;
}

void prepare_window_factors(hipStream_t s, ParticleSet& ps, const GridGeom& g) {
  if (ps.wfac_valid || !window_factors_apply(g)) return;
  ps.wfac.ensure(6 * (size_t)std::max<int64_t>(ps.n, 1));
  ps.wsta.ensure((size_t)std::max<int64_t>(ps.n, 1));
  if (ps.n > 0) {
    hipLaunchKernelGGL(window_factors_kernel, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s, ps.pos.get(),
                       ps.n, g, ps.wfac.get(), ps.wsta.get());
    PE_CHECK_LAUNCH();
  }
  ps.wfac_valid = true;
}

template <typename T>
void launch_spread(hipStream_t s, const ParticleSet& ps, const double* q, T* grid, const GridGeom& g,
                   bool accumulate) {
  if (ps.n == 0 && accumulate) return;
  require(g.P <= kMaxP, "support P must be <= 16");
  ParticleSet& m = const_cast<ParticleSet&>(ps);
  if constexpr (sizeof(T) == 4) {
    m.qspread.ensure((size_t)std::max<int64_t>(ps.n, 1));
    if (ps.n > 0) {
      hipLaunchKernelGGL(sorted_charges_kernel, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s, ps.idx.get(),
                         q, ps.n, m.qspread.get());
      PE_CHECK_LAUNCH();
    }
    const int nbz = (g.ntile[2] + kWaves - 1) / kWaves;
    const int nt = g.ntile[0] * g.ntile[1] * nbz;
    const int* start = ps.spread_by_home ? ps.home_start.get() : ps.tile_start.get();
    const int* entries = ps.spread_by_home ? ps.home_entries.get() : ps.tile_entries.get();
    // the tile lists of a set spread by every Krylov product (supports of at
    // most one tile on whole tiles): factors computed once per configuration
    if (!ps.spread_by_home && window_factors_apply(g)) {
      prepare_window_factors(s, m, g);
      hipLaunchKernelGGL((spread_tile_kernel<T, false, true>), dim3((unsigned)nt), dim3(256), 0, s, ps.pos.get(),
                         m.qspread.get(), start, entries, ps.wfac.get(), reinterpret_cast<const int*>(ps.wsta.get()),
                         ps.n, grid, g, accumulate ? 1 : 0);
    } else if (ps.spread_by_home) {
      hipLaunchKernelGGL((spread_tile_kernel<T, true, false>), dim3((unsigned)nt), dim3(256), 0, s, ps.pos.get(),
                         m.qspread.get(), start, entries, nullptr, nullptr, ps.n, grid, g, accumulate ? 1 : 0);
    } else {
      hipLaunchKernelGGL((spread_tile_kernel<T, false, false>), dim3((unsigned)nt), dim3(256), 0, s, ps.pos.get(),
                         m.qspread.get(), start, entries, nullptr, nullptr, ps.n, grid, g, accumulate ? 1 : 0);
    }
  } else if (ps.spread_by_home) {
    // a set spread from its sorted home lists (the ions in mixed precision,
    // whose double pass forms the right-hand side): no tile lists needed
    m.qspread.ensure((size_t)std::max<int64_t>(ps.n, 1));
    if (ps.n > 0) {
      hipLaunchKernelGGL(sorted_charges_kernel, dim3((unsigned)((ps.n + 255) / 256)), dim3(256), 0, s, ps.idx.get(),
                         q, ps.n, m.qspread.get());
      PE_CHECK_LAUNCH();
    }
    const int nbz = (g.ntile[2] + kWaves - 1) / kWaves;
    const int nt = g.ntile[0] * g.ntile[1] * nbz;
    hipLaunchKernelGGL((spread_tile_kernel<T, true, false>), dim3((unsigned)nt), dim3(256), 0, s, ps.pos.get(),
                       m.qspread.get(), ps.home_start.get(), ps.home_entries.get(), nullptr, nullptr, ps.n, grid, g,
                       accumulate ? 1 : 0);
  } else {
    if (!ps.have_tile_lists) build_tile_lists(s, m, g);
    // double: the window exponentials dominate, and spreading them over the
    // whole workgroup (one staging pass per 64 particles) measured faster
    const int nt = g.ntile[0] * g.ntile[1] * g.ntile[2];
    hipLaunchKernelGGL(spread_block_kernel<T>, dim3((unsigned)nt), dim3(256), 0, s, ps.pos.get(), ps.idx.get(), q,
                       ps.tile_start.get(), ps.tile_entries.get(), grid, g, accumulate ? 1 : 0);
  }
  PE_CHECK_LAUNCH();
}

template <typename T>
void launch_gather(hipStream_t s, const ParticleSet& ps, const T* grid, const GridGeom& g,
                   double* phi, double* E, bool accumulate) {
  if (ps.n == 0) return;
  require(g.P <= kMaxP, "support P must be <= 16");
  const int Hs = kTile + g.P - 1;
  const size_t region = (size_t)Hs * Hs * (g.P == 8 ? kGatherRow : Hs) * sizeof(T);
  // tile-staged in single precision, and in double for P = 8 (the unrolled
  // contraction: 187 -> 148 us per bead pass at cfg5); double with other
  // supports per particle (its region halves the workgroups an LDS holds)
  if ((sizeof(T) == 4 || g.P == 8) && region <= (size_t)kGatherLDS) {
    if (ps.n_home_tiles == 0) return;
    const dim3 blocks((unsigned)ps.n_home_tiles);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, blocks, dim3(256), region, s, ps.pos.get(), ps.idx.get(), ps.home_start.get(),
                         ps.home_entries.get(), ps.home_tiles.get(), grid, g, phi, E, accumulate ? 1 : 0);
    };
    if (g.P == 8) {
      if (E) go(gather_tile_kernel<T, true, 8>);
      else go(gather_tile_kernel<T, false, 8>);
    } else {
      if (E) go(gather_tile_kernel<T, true, 0>);
      else go(gather_tile_kernel<T, false, 0>);
    }
    PE_CHECK_LAUNCH();
    return;
  }
  const int64_t nb = (ps.n + kWaves - 1) / kWaves;
  if (E)
    hipLaunchKernelGGL((gather_kernel<T, true>), dim3((unsigned)nb), dim3(256), 0, s,
                       ps.pos.get(), ps.idx.get(), ps.n, grid, g, phi, E, accumulate ? 1 : 0);
  else
    hipLaunchKernelGGL((gather_kernel<T, false>), dim3((unsigned)nb), dim3(256), 0, s,
                       ps.pos.get(), ps.idx.get(), ps.n, grid, g, phi, E, accumulate ? 1 : 0);
  PE_CHECK_LAUNCH();
}

template void launch_spread<float>(hipStream_t, const ParticleSet&, const double*, float*, const GridGeom&, bool);
template void launch_spread<double>(hipStream_t, const ParticleSet&, const double*, double*, const GridGeom&, bool);
template void launch_gather<float>(hipStream_t, const ParticleSet&, const float*, const GridGeom&, double*, double*, bool);
template void launch_gather<double>(hipStream_t, const ParticleSet&, const double*, const GridGeom&, double*, double*, bool);

}  // namespace pe
