// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <deque>
#include <map>
#include <vector>

#include "../../include/pe.h"

namespace pe {

// ----------------------------------------------------------------- errors

struct Error : std::runtime_error {
  pe_status code;
  Error(pe_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PE_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::pe::Error(PE_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define PE_CHECK_LAUNCH() PE_HIP(hipGetLastError())

inline void require(bool ok, const std::string& msg) {
  if (!ok) throw Error(PE_ERR_ARG, msg);
}
// a literal message builds no string unless the check fails (checks on hot
// host paths allocate nothing)
inline void require(bool ok, const char* msg) {
  if (!ok) throw Error(PE_ERR_ARG, msg);
}

// -------------------------------------------------------- device workspace

// All device memory of a context lies in one region the caller registers
// with pe_set_workspace (a torch tensor, say); the library itself never
// allocates device memory.  Buffers are carved from the region first fit in
// 256-byte granules, freed blocks coalesce with their neighbours, and every
// live block records the address of the pointer that owns it, so that
// pe_set_workspace can move all live blocks into a new, larger region and
// repoint their owners.  A request that does not fit throws PE_ERR_NOMEM and
// records how large the region would have to be (`need`), which
// pe_workspace_size then reports.
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  char* base = nullptr;
  size_t size = 0;
  size_t in_use = 0;   // bytes in live blocks
  size_t peak = 0;     // largest in_use seen
  size_t need = 0;     // region size a failed request would have needed (0: none failed)

  void* alloc(size_t bytes, void** owner);
  void release(void* p);
  void reown(void* p, void** owner);
  // Moves every live block into [nb, nb + nsize) (copies on stream s, then
  // waits) and makes it the region.  Throws PE_ERR_NOMEM if they do not fit.
  void migrate(char* nb, size_t nsize, hipStream_t s);
  size_t live_blocks() const { return live_.size(); }

 private:
  struct Blk {
    size_t len;
    void** owner;
  };
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, Blk> live_;      // offset -> block
};

// The arena of the context whose entry point is running on this thread (set
// by every entry point); buffers remember the arena they came from.
extern thread_local Arena* tl_arena;
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a) : prev(tl_arena) { tl_arena = a; }
  ~ArenaScope() { tl_arena = prev; }
};

// Page-locked host memory for the set-up's transfers of counts and offsets
// (a pageable end makes each copy a blocking, staged one).  Grown on demand;
// each buffer carries one transfer per set-up call, and every set-up call
// ends with a stream synchronization, so no buffer is reallocated or
// rewritten under a copy in flight.
struct PinnedBuf {
  void* p = nullptr;
  size_t cap = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  template <typename T>
  T* get(size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (bytes > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess || !p)
        throw Error(PE_ERR_NOMEM, "page-locked host staging buffer");
      cap = bytes;
    }
    return static_cast<T*>(p);
  }
};

// A buffer in the context's workspace; grows on demand, never shrinks.
template <typename T>
struct DevBuf {
  T* ptr = nullptr;
  size_t cap = 0;  // elements
  Arena* arena = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr && arena) arena->release(ptr);
    ptr = nullptr;
    cap = 0;
  }
  T* ensure(size_t n) {
    if (n <= cap && ptr) return ptr;
    release();
    Arena* a = tl_arena;
    if (!a) throw Error(PE_ERR_STATE, "device buffer requested outside an entry point");
    const size_t bytes = (n ? n : 1) * sizeof(T);
    ptr = static_cast<T*>(a->alloc(bytes, reinterpret_cast<void**>(&ptr)));
    arena = a;
    cap = n ? n : 1;
    return ptr;
  }
  // exchange storage with o (the owners recorded in the arena follow)
  void swap(DevBuf& o) {
    std::swap(ptr, o.ptr);
    std::swap(cap, o.cap);
    std::swap(arena, o.arena);
    if (ptr) arena->reown(ptr, reinterpret_cast<void**>(&ptr));
    if (o.ptr) o.arena->reown(o.ptr, reinterpret_cast<void**>(&o.ptr));
  }
  T* get() const { return ptr; }
  operator T*() const { return ptr; }
};

// ---------------------------------------------------------------- geometry

// Spectral-Ewald grid geometry and window constants (passed by value).
struct GridGeom {
  int N[3];         // mesh
  int Nzc;          // N[2]/2 + 1
  int Nzs;          // row stride of the half spectrum: Nzc rounded up to a multiple of 16
  double h[3];      // spacing
  double inv_h[3];
  double L[3];
  int P;            // support per axis
  double wexp;      // 2 xi^2 / eta   (w = wnorm * exp(-wexp d^2) per axis)
  double wnorm;     // sqrt(2 xi^2 / (pi eta))
  double h3;        // h_x h_y h_z
  double eps;
  double fcoef;     // -4 xi^2 h3 / (eps eta)  (field prefactor)
  int ntile[3];     // spreading tiles per axis (ceil(N / 8))
};

// Workgroups are handed to the eight XCDs round robin (workgroup b to XCD
// b % 8), and each XCD has its own L2.  This maps workgroup b to a logical
// index so that each XCD receives one contiguous range of logical indices:
// work items that are neighbours in space (and share cached data) then run
// under one L2.  A bijection of [0, n).
constexpr int kNumXCD = 8;
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n / kNumXCD, r = n % kNumXCD;
  const int x = b % kNumXCD;
  return x * q + min(x, r) + b / kNumXCD;
}

// Real-space geometry.
struct RealGeom {
  double L[3];
  double inv_L[3];
  int nc[3];        // cells per axis (1 or >= 3)
  double cell_inv[3];
  double rc2;
  double xi;
  double eps;
  int reg;          // pe_reg
  double a;         // shell radius
  const float* erfcx = nullptr;  // device table of the scaled erfc (single-precision pair kernel)
};

// Piecewise table of the scaled complementary error function erfcx(x) =
// exp(x^2) erfc(x) on [0, kErfcxPieces / kErfcxInvWidth), pieces of width
// 1 / kErfcxInvWidth: per piece, the Taylor coefficients about its midpoint
// up to degree kErfcxDeg (kErfcxDeg + 1 floats per piece).
constexpr int kErfcxPieces = 24;
constexpr int kErfcxDeg = 7;
constexpr float kErfcxInvWidth = 4.0f;
void build_erfcx_table(hipStream_t s, DevBuf<float>& tab);

// Single-precision table of the Gaussian-regularized real-space kernel R(r)
// for one class of pairs (one value of s2 = sigma_t^2 + sigma_s^2): r in
// [0, r_c] cut into kPairTabPieces pieces of width h; on piece k,
// R(r) = sum_j a_j t^j with t = 2 (r - (k + 1/2) h) / h in [-1, 1], degree 6
// (interpolation at the 7 Chebyshev points of the piece; 8 floats per piece,
// the last zero).  dR/dr = (2 / h) sum_j j a_j t^(j-1) comes from the same
// coefficients.  build_pair_table fits the pieces in double, rounds them to
// float and checks value and slope against the closed form at 18 points per
// piece; it returns false (and the caller keeps the general kernel) if
// either misses by more than 1e-7 of its largest magnitude on [0, r_c].
constexpr int kPairTabPieces = 64;
constexpr int kPairTabFloats = 8 * kPairTabPieces;
bool build_pair_table(const RealGeom& rg, double s2, float* out);

// A particle set sorted by real-space cell.
struct ParticleSet {
  int64_t n = 0;
  DevBuf<double4> pos;      // sorted: wrapped x,y,z and sigma in w
  DevBuf<float4> posf;      // sorted: x, y relative to the cell origin, z (single precision); owner body as int bits
  DevBuf<uint4> posx;       // sorted: x, y, z in fixed point (2^32 units per box length); sigma as float bits
  DevBuf<int> idx;          // sorted slot -> caller index within the set
  DevBuf<int> cell_start;   // ncell + 1
  DevBuf<int> cell_count;   // ncell (scratch)
  DevBuf<int> cell_of;      // caller order (scratch)
  DevBuf<int> zsub;         // caller order: z slab of the particle within its cell (scratch)
  DevBuf<double4> tmp;      // caller order wrapped positions (scratch)
  DevBuf<int4> chunks;      // pair-traversal work units: (first, end sorted slot, first cell, cells), <= 64 each
  DevBuf<double> qsorted;   // charges in sorted order for the pair passes (scratch)
  DevBuf<float> qsortedf;   // the same in single precision (scratch)
  DevBuf<double> qspread;   // charges in sorted order for spreading (scratch)
  DevBuf<float4> wfac;      // sorted: single-precision window factors, 8 per axis, rotated (support <= 8)
  DevBuf<int4> wsta;        // sorted: wrapped mesh index of support point 0 per axis
  bool wfac_valid = false;  // window factors of the current configuration
  int n_chunks = 0;
  // grid tiles overlapped by each particle's support (spreading lists)
  DevBuf<int> tile_start;   // ntile + 1
  DevBuf<int> tile_count;   // 2 ntile (scratch: counts and cursors of both list kinds)
  // host copies of the counts and offsets (kept so the copies to the device
  // need no wait before the builders return)
  PinnedBuf h_tcnt, h_tstart, h_hcnt, h_hstart, h_htiles, h_ccnt, h_cstart, h_chunks;
  bool have_tile_lists = false;   // tile lists built for the current configuration
  bool spread_by_home = false;    // single-precision spreading walks the sorted home lists
  std::vector<int> h_colcur, h_colz;         // per column: next particle and its cell (scratch of the unit build)
  std::vector<int> h_start;                  // cell offsets on the host (scratch of the unit build)
  DevBuf<int> tile_entries; // sorted-particle indices, grouped by tile
  int64_t n_entries = 0;
  // home tile of each particle (the tile holding its first support point):
  // contraction lists
  DevBuf<int> home_start;   // ntile + 1
  DevBuf<int> home_entries; // sorted-particle indices, grouped by home tile
  DevBuf<int> home_tiles;   // tiles with at least one home particle
  int n_home_tiles = 0;
  // width check of the set: [0] nonzero if the widths differ, [1] the first
  // width's bits; sig_uniform is the width when all are equal, else 0
  DevBuf<unsigned long long> sig_check;
  double sig_uniform = 0.0;
};

// Pair tables of the classes (target set, source set) of one context's
// traversals whose sets both have uniform widths (see build_pair_table).
struct PairTables {
  DevBuf<float> buf;              // slots x kPairTabFloats
  double key[6] = {};             // xi, eps, rc2, reg and the two widths the tables were built for
  bool built = false;
  int slot[2][2] = {{-1, -1}, {-1, -1}};  // [target is ions][source is ions]; -1: no table
  const float4* get(bool tgt_ion, bool src_ion) const {
    const int k = slot[tgt_ion ? 1 : 0][src_ion ? 1 : 0];
    return k < 0 ? nullptr : reinterpret_cast<const float4*>(buf.get() + (size_t)k * kPairTabFloats);
  }
};

// 1-D FFT factorization (radices 8, 4, 2, 3, 5).
struct FFTPlan1D {
  int n;
  int nstage;
  int radix[16];
};

// ------------------------------------------------------------- profiling

// HIP events around kernel launches on the context stream, resolved after
// the stream has been synchronized.
struct Prof {
  bool on = false;
  uint32_t mask = 0xffffffffu;  // classes that record events
  double ms[2 * PE_PROF_NCLASS] = {};
  double cnt[2 * PE_PROF_NCLASS] = {};
  double work[2 * PE_PROF_NCLASS] = {};
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double work;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void reset() {
    flush();
    for (int i = 0; i < 2 * PE_PROF_NCLASS; ++i) ms[i] = cnt[i] = work[i] = 0;
  }
  // call only when the stream is idle
  void flush() {
    for (auto& r : pending) {
      float t = 0;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.cls] += t;
        cnt[r.cls] += 1;
        work[r.cls] += r.work;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  ~Prof() {
    for (auto& r : pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct ProfScope {
  Prof* p;
  hipStream_t s;
  int cls;
  double work;
  hipEvent_t a = nullptr;
  // dbl: the launch computes in double (its class is offset by PE_PROF_NCLASS);
  // w: work units of the launches inside the scope
  ProfScope(Prof& prof, hipStream_t st, int c, bool dbl, double w = 0)
      : p(prof.on && ((prof.mask >> c) & 1u) ? &prof : nullptr), s(st),
      cls(c + (dbl ? PE_PROF_NCLASS : 0)), work(w) {
    if (p) {
      a = p->take();
      (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (p) {
      hipEvent_t b = p->take();
      (void)hipEventRecord(b, s);
      p->pending.push_back({cls, a, b, work});
    }
  }
};

// ------------------------------------------------------------ body shapes

// One rigid-body shape: reference geometry (relative bead positions of the
// first body seen), widths, the distances of every bead to up to four
// reference beads (the matching signature), and the dense per-shape blocks:
// the inverse of the body saddle block (preconditioner) and the intra-body
// real-space block (near field).  `bodies` lists the bodies of the current
// configuration that have this shape.
struct BodyType {
  int N = 0;
  std::vector<double> ref, sig;
  int nref = 0;
  int refidx[4] = {0, 0, 0, 0};
  double scale = 0;                // largest reference distance
  double extent = 0;               // largest distance of a bead from the centroid
  DevBuf<double> dref;             // N x nref reference distances
  DevBuf<double> dsig;             // N widths
  DevBuf<int> drefidx;             // nref
  bool have_inv = false;
  DevBuf<double> Ainv;
  DevBuf<float> Ainv32;
  DevBuf<double> Minv;             // inverse of the free-space self block alone (N x N)
  bool near = false;               // intra-body real-space block stored densely
  DevBuf<double> R64;
  DevBuf<float> R32;
  std::vector<int> bodies;
  DevBuf<int> dbodies;
};

struct Precond {
  std::deque<BodyType> types;
  DevBuf<int> assigned;            // per body: type index
  DevBuf<unsigned char> dense;     // per body: intra-body pairs held by a dense block
  std::vector<unsigned char> dense_h;  // host copy
  PinnedBuf h_asg;                 // per body: type index, on the host
  int64_t near_beads = 0;          // beads of bodies with a dense block
  DevBuf<double> gemm_ws;          // partial tiles of the split per-shape products
};

// ----------------------------------------------------------------- context

struct LearnedGuess;  // defined in the guess translation unit

}  // namespace pe

struct pe_context {
  // declared first so that it is destroyed after every buffer carved from it
  pe::Arena arena;
  pe_params p;
  hipStream_t stream = nullptr;
  // second stream (default priority) for the real-space pair passes of the
  // one-off potentials, forked from and joined back into `stream` by events,
  // so they overlap the spread / FFT / gather of the same pass
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_est = nullptr;  // a Krylov step's residual estimate has reached the host
  bool bodies_uploaded = false; // off and body_of hold the body structure h_off describes
  pe::DevBuf<double> phi_pair, E_pair;  // the pair passes' own outputs (summed after the join)
  pe::DevBuf<double> phi_near;          // the near-field blocks' output of a Krylov product
  std::string err;

  int lds_per_block = 65536;  // device limit on LDS per workgroup (bytes)
  int device = 0;             // the GPU current at pe_create (the context's device)

  bool consts_ready = false;  // parameter tables built in the workspace
  // derived parameters
  double xi = 0, rc = 0, eta = 0, hmax = 0, V = 0;
  pe::GridGeom gg{};
  pe::RealGeom rg{};
  pe::FFTPlan1D plan[3]{};
  pe::DevBuf<double2> tw64[3];
  pe::DevBuf<float2> tw32[3];
  pe::DevBuf<double> gtab;   // separable Green's-function tables (exp factors, k_d^2)
  pe::DevBuf<float> erfcx_tab;  // scaled erfc pieces for the single-precision pair kernel
  pe::PairTables pair_tabs;     // per-class pair tables (uniform widths)

  // system
  bool have_system = false;
  bool have_solution = false;
  bool have_forces = false;
  int64_t n_body = 0, n_bead = 0, n_ion = 0;
  std::vector<int64_t> h_off;
  double E0[3] = {0, 0, 0};
  pe::DevBuf<int64_t> off;
  pe::DevBuf<int> body_of;
  pe::DevBuf<double> rel;          // n_bead x 3, r_ij
  pe::DevBuf<double> bead_x;       // n_bead x 3 unwrapped copy
  pe::DevBuf<double> ion_x;        // n_ion x 3 unwrapped copy
  pe::DevBuf<double> bead_sig, ion_sig, ion_q, body_Q, quat;
  pe::DevBuf<int> body_type;
  pe::ParticleSet B, I;
  double bead_sig_uniform = -1.0;  // >0 if all bead widths are equal

  // bead-bead real-space operator, CSR over sorted bead rows
  int64_t nnz = 0;
  pe::DevBuf<int64_t> row_ptr;
  pe::DevBuf<int64_t> scan_tmp;    // prefix-sum workspace
  // The pair structure is built with the cutoff r_c + skin and kept while no
  // bead has moved more than skin/2 since (rigid bodies in Brownian steps
  // move little); every configuration recomputes the values from the current
  // positions with the exact cutoff r_c, so the operator is the truncated
  // one either way.
  bool csr_valid = false;
  double csr_rc = 0, csr_skin = 0;
  std::vector<int64_t> csr_off;
  std::vector<unsigned char> csr_dense;
  pe::DevBuf<double> csr_x0;       // bead positions (caller order) at the build
  pe::PinnedBuf h_disp;             // per-block largest squared displacement since the build, on the host
  bool disp_pending = false;        // h_disp filled by launch_max_disp_early for this configuration
  unsigned disp_nbk = 0;
  pe::PinnedBuf h_stats;            // partials of the input checks, on the host
  pe::DevBuf<int> csr_row;         // caller bead index of every row
  pe::DevBuf<double> csr_part;     // displacement reduction partials
  pe::DevBuf<int> cnt;
  pe::DevBuf<int> col;
  pe::DevBuf<double> val64;
  pe::DevBuf<float> val32;
  bool have_val32 = false;

  // grids (sized for double; float reuses the same memory)
  pe::DevBuf<double> gridA, gridB;
  pe::DevBuf<double2> gridC;

  // per-particle scratch in caller order
  pe::DevBuf<double> phi_w, phi_all, E_all;   // (n_bead+n_ion), (n_bead+n_ion)x3
  pe::DevBuf<double> sums;                     // body sums / totals scratch
  pe::DevBuf<double> red;                      // reduction partials

  // Krylov
  pe::DevBuf<double> Vb;       // (m+1) x n basis
  pe::DevBuf<double> Zb;       // m x n preconditioned directions
  pe::DevBuf<double> kvec;     // x, b, r, w, ... (several n-vectors)
  pe::DevBuf<double> hs;       // Hessenberg, rotations, g, y, scalars
  pe::DevBuf<double> rhs_b;    // right-hand side
  pe::DevBuf<double> xsol;     // last solution [q; dpsi]
  pe::DevBuf<double> forces;   // f per particle (n_bead+n_ion) x 3
  pe::DevBuf<double> bodyF, bodyL;  // n_body x 3 from the last force pass
  pe::DevBuf<double> bd_R;     // per-body rotation of the last BD step
  // hard spheres of the BD step: cells over all particles, forces
  pe::DevBuf<int> hs_cell, hs_entries, hs_count, hs_start;
  pe::DevBuf<int64_t> hs_start64, hs_scan;
  pe::DevBuf<double> hs_f;
  pe::DevBuf<double> E_ion;    // n_bead x 3, field of the ions at the beads (learned-guess features)
  // single-precision ion parts kept from the right-hand side for the force
  // pass of the same configuration: the spread ion grid (before the
  // convolution) and the real-space ion -> bead potential and field
  pe::DevBuf<float> ion_grid32;
  pe::DevBuf<double> ion_rs_phi, ion_rs_E;
  bool ion_parts_valid = false;
  bool have_eion = false;
  double* pinned = nullptr;    // 512 doubles of pinned host memory for small reads (hipHostMalloc)

  // learned guess
  pe::LearnedGuess* guess = nullptr;

  pe::Prof prof;
  pe::DevBuf<unsigned long long> pair_count;  // [float, double] pairs evaluated while profiling
  pe::Precond pc;
};

namespace pe {

// ------------------------------------------------------------ launchers
// (each enqueues on the given stream; geometry passed by value)

// grid: spread charges q (indexed by caller index through idx) into grid (accumulate)
void build_tiles(hipStream_t s, ParticleSet& ps, const GridGeom& g, bool spread_by_home);
// single-precision window factors of the set's configuration (supports of at
// most 8 points on meshes of whole 8-point tiles): computed by the first
// single-precision spread of the set's tile lists after the configuration
// changed, used by every later one
bool window_factors_apply(const GridGeom& g);
void prepare_window_factors(hipStream_t s, ParticleSet& ps, const GridGeom& g);
template <typename T>
void launch_spread(hipStream_t s, const ParticleSet& ps, const double* q, T* grid, const GridGeom& g,
                   bool accumulate);
// grid: gather potential (and optionally field) at the particles of ps;
// writes (or adds, if accumulate) phi[idx] and E[idx*3+d]
template <typename T>
void launch_gather(hipStream_t s, const ParticleSet& ps, const T* grid, const GridGeom& g,
                   double* phi, double* E, bool accumulate);

// FFT pipeline: real grid A -> complex -> scaled -> real grid B
template <typename T>
void launch_wave_pipeline(hipStream_t s, pe_context* c, T* gridA, T* gridB, void* gridC);
void make_fft_plan(int n, FFTPlan1D& plan);
void build_green_tables(pe_context* c);

// real space
// owner (caller order, may be null): body of each particle, kept as a tag in
// the single-precision copy
void build_cells(hipStream_t s, ParticleSet& ps, const double* pos_caller, const double* sig_caller,
                 double sig_const, const int* owner, int64_t n, const RealGeom& rg);
// the same in two halves around the caller's wait on s: the cell counts (and
// their copy to the host), then the offsets, work units and sorted records
void cells_count(hipStream_t s, ParticleSet& ps, const double* pos_caller, const double* sig_caller,
                 double sig_const, int64_t n, const RealGeom& rg);
void cells_finish(hipStream_t s, ParticleSet& ps, const int* owner, const RealGeom& rg);
void build_bead_matrix(pe_context* c);
// the beads' largest displacement since the stored pair structure was built,
// launched early with its copy to the host (build_bead_matrix reads it after
// a later wait on the stream); only when a structure for the same bodies exists
void launch_max_disp_early(pe_context* c);
// phi_real[b] += sum_j R_bj q_j over the stored inter-body pairs
template <typename T>
void launch_spmv_add(hipStream_t s, pe_context* c, const double* q, double* phi_real);
// y_top[b] = -(phi_wave[b] + phi_real[b] - ck0_b) + dpsi[body(b)]
void launch_assemble(hipStream_t s, pe_context* c, const double* dpsi, const double* phi_wave,
                     const double* phi_real, const double* ck0, double* y_top);
// Adds the real-space potential (and field, if E) at the targets from up to
// two source sets; field_single evaluates the field in single precision.
// tab0 / tab1 (may be null): pair tables of the classes (tgt, src0) and
// (tgt, src1), used by the single-precision Gaussian passes when every
// source set has one.
template <typename T>
void launch_pair_onfly(hipStream_t s, const ParticleSet& tgt, const ParticleSet* src0, const double* q0,
                       const ParticleSet* src1, const double* q1, const RealGeom& rg, double* phi, double* E,
                       bool field_single = false, unsigned long long* npairs = nullptr,
                       const float4* tab0 = nullptr, const float4* tab1 = nullptr);
// (Re)builds the tables of the bead / ion classes when the geometry or the
// widths changed (after build_cells of both sets).
void update_pair_tables(hipStream_t s, PairTables& pt, const RealGeom& rg, const ParticleSet& beads,
                        const ParticleSet& ions);

// body shapes (shapes.hip): group bodies into shape types (device-side
// matching, types cached across configurations), build the per-shape blocks
void shape_setup(pe_context* c);
// the first half of shape_setup, launched earlier: the known shapes' matches
// and their copy to the host (shape_setup runs after a wait on the stream)
void shape_match_launch(pe_context* c);
// y[:, b] (+)= A x[:, b] for the bodies b of one shape: column b is the
// body's bead segment of x (plus its dPsi entry when bordered, A then
// (N+1) x (N+1)); accumulate adds into y.
// ws: workspace of body_gemm_workspace(N, nbt, bordered) doubles.
template <typename T>
void launch_body_gemm(hipStream_t s, const T* A, int N, bool bordered, bool accumulate, const int* bodies,
                      int nbt, const int64_t* off, int64_t n_bead, const double* x, double* y, double* ws);
size_t body_gemm_workspace(int N, int nbt, bool bordered);
// dense intra-body real-space block of one shape (realspace.hip)
void build_near_block(hipStream_t s, const BodyType& t, const RealGeom& rg, double* R64, float* R32);

// The saddle-point operator y = [-M q + Sigma^T dpsi; Sigma q] of the loaded
// configuration for x = [q; dpsi] (prec: PE_FP64 or PE_MIXED kernels).
void saddle_product(pe_context* c, int prec, const double* x, double* y);
// Grand capacitance C (device, row-major (4 n_body)^2) and the effective
// permittivity (host 3 x 3, may be null) of the loaded configuration.
void grand_capacitance(pe_context* c, double* C_out, double* eps_out, pe_solve_info* info);

// Device address of this GPU's copy of the allocation-free BD step's static
// scratch array (looked up once per device, with that device current).
double* bd_static_scratch(int dev);

// body / vector kernels
void launch_body_sums(hipStream_t s, pe_context* c, const double* q, double* out_sum, double* out_sig2);
void launch_seg_totals(hipStream_t s, int64_t n_body, const double* body_sum, const double* body_sig2,
                       double* totals);
void launch_zero(hipStream_t s, double* p, int64_t n);

}  // namespace pe
