// Internal declarations of the VIP library: context, sliced-ELL operators,
// device scalar blocks and helpers shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/vip.h"

namespace vip {

constexpr int kSlice = 64;      // rows per ELL slice = one wavefront
constexpr int kBlock = 256;     // threads per block of the row kernels
constexpr int kMaxWidth = 128;  // largest neighbour list of one evaluation point
constexpr int kNumXcd = 8;      // accelerator complex dies of the MI355X
constexpr int kMaxTaps = 32;    // taps of a canonical (lattice-interior) row

struct Error {
  int code;
  std::string msg;
};

// Rows of a sliced-ELL operator that are translation-invariant copies of one reference
// row: a lattice node whose stored entries sit at the same lattice offsets and hold, bit
// for bit, the same values.  Products over such rows read the weights from `w` and find
// the columns through the lattice map, and give the same bits as the general path.
// Lattice tiles (tile.h): tiles of kTileX x kTileY pixels, one wavefront wide.
constexpr int kTileX = 64;
constexpr int kTileY = 16;
// Rows of one canonical set (or a pair of sets) split into tile rows and irregular rows.
constexpr int kTileRecWords = 64;   // 32-bit words of a tile record

struct TilePart {
  uint64_t* bits = nullptr;         // device [nty*kTileY*ntx]: bit lx of word (y, tx): the node at
                                    // pixel (64 tx + lx, y) is a tile row
  int32_t* tiles = nullptr;         // device [ntiles]: tiles (ty * ntx + tx) holding tile rows
  int64_t ntiles = 0;
  int32_t* irr = nullptr;           // device [nirr]: every other row, ascending
  int64_t nirr = 0;
  uint32_t* rec = nullptr;          // device [ntiles * kTileRecWords]: per listed tile, in list order,
                                    // its record (tile.h, TileMeta): tx, ty, the 20 halo-row starts
                                    // and the 16 row masks in one 256-byte block
  int tile_blocks = 0, irr_blocks = 0;   // launch split of a tiled kernel
};
// Tile geometry of the lattice.
struct TileMap {
  int ntx = 0, nty = 0;
  int32_t* rowstart = nullptr;      // device [(nty*kTileY + 4) * ntx]: entry (yy, tx) is the node at
                                    // pixel (64 tx - 2, yy - 2) when pixels 64 tx - 2 .. 64 tx + 65
                                    // of that lattice row hold consecutive nodes, else -1
};

struct Canon {
  int K = 0;                        // taps of the reference row (0: none)
  int32_t dx[kMaxTaps], dy[kMaxTaps];
  int32_t off[kMaxTaps];            // pixel offsets dy*W + dx, in the row's slot order
  double w[4][kMaxTaps];            // reference values of FP64 value sets 0..3
  float w32[3][kMaxTaps];           // reference values of FP32 value sets 4..6
  float rsum32[3] = {0.0f, 0.0f, 0.0f};  // reference FP32 row sums of sets 4..6
  int disk = 0;                     // 1: the taps are the 21-point disk in slot order
  int box = 0;                      // 1: the taps are the 3 x 3 box in slot order (coarse level)
  int64_t ref_row = -1;             // reference row of the first marked set (-2: no repeated pattern)
  int64_t vref[7] = {-1, -1, -1, -1, -1, -1, -1};  // reference row of each marked value set
  int32_t* cpix[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // device [n]
                                    // per value set (0..3 FP64; 4..6 FP32: pressure, predictor u, v):
                                    // pixel of a canonical row, else -1
  int64_t count[7] = {0, 0, 0, 0, 0, 0, 0};
  // per 64-row slice and value set (disk taps only): the nodes 2 and 1 rows below and 1 and 2
  // rows above the slice's first row when all 64 rows are canonical and sit on consecutive
  // pixels of one lattice row (then row i0 + l reads them + l), else -1 in the first entry
  int32_t* sbase[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t described[7] = {0, 0, 0, 0, 0, 0, 0};   // rows in described slices, per set
  // tile partitions (disk taps only): [0] set 0, [1] set 4, [2] sets 1 and 2, [3] sets 5 and 6
  TilePart tpart[4];
};

// Sliced ELL matrix: rows grouped by 64; slice s holds width[s] columns stored
// column-major, element (row r, slot k) at ptr[s] + k*64 + (r - 64 s).
// Padding slots carry col = 0 (any in-range index) and value 0.
// Lattice-interior rows of the VIP and node operators (the per-step products of eqs. 12-15).
// A node is canonical here when its rows of the four VIP operators and of D^[0,0] and the
// Laplacian are all canonical (see Canon).  Each of those reference rows is stored as runs of
// consecutive lattice columns, one per stencil row dy = -3..3 in slot order, so a row's taps
// are rb[dy] + dx0 .. rb[dy] + dx0 + len - 1 with rb[dy] the node straight above or below.
constexpr int kVcOps = 5;           // e, w, n, s VIP operators; node operators (D^[0,0], Laplacian)
constexpr int kVcRows = 7;          // stencil rows dy = -3..3
struct VipCanon {
  int32_t* cpix = nullptr;          // device [n]: pixel of a canonical node, else -1
  int64_t count = 0;
  int8_t dx0[kVcOps][kVcRows] = {};
  int8_t len[kVcOps][kVcRows] = {};
  uint8_t used[kVcRows] = {};       // some operator has taps in this stencil row
  double w[kVcOps + 1][kMaxTaps] = {};  // e, w, n, s, D^[0,0], Laplacian; slot order
  TilePart tpart;                   // lattice tiles of the canonical interior nodes (taps within +-3)
};

struct Ell {
  int64_t nrows = 0;
  int64_t nslices = 0;
  int64_t nnz_slots = 0;            // ptr[nslices]
  int64_t* ptr = nullptr;           // device [nslices + 1]
  int32_t* width = nullptr;         // device [nslices]
  int32_t* rowlen = nullptr;        // device [nrows], true row length
  int32_t* cols = nullptr;          // device [nnz_slots]
  double* val[4] = {nullptr, nullptr, nullptr, nullptr};  // FP64 value sets
  float* val32 = nullptr;           // FP32 value set (pressure matrix only)
  float* rsum32 = nullptr;          // FP32 rows evaluated as rsum*x_i + sum a_ij (x_j - x_i)
  float* val32h[2] = {nullptr, nullptr};   // FP32 predictor matrices H D^-1, columns scaled by the
                                           // inverse diagonal (system layout only)
  float* rsum32h[2] = {nullptr, nullptr};
  int64_t max_width = 0;
  int64_t nnz = 0;                  // sum of row lengths
  Canon canon;                      // lattice-interior rows (system layout only)
  // row-relative columns: dcols[q] = cols[q] - row (0 in padding slots) in the 64-row slices
  // whose stored columns all lie within +-32767 of their rows (dfit[slice] = 1); the
  // solve-phase kernels read those 2-byte columns there and the int32 ones in the other
  // slices (rows next to far-numbered nodes, such as body-surface nodes listed last).  Null
  // when no slice fits (or VIP_NO_DELTA=1).
  int16_t* dcols = nullptr;
  uint8_t* dfit = nullptr;          // device [nslices]
  int64_t dfit_slices = 0;          // slices with dfit = 1
  int64_t dfit_nnz = 0;             // stored entries of those slices' rows
};

// The 21-point lattice disk of radius 2.5h in slot order (rows dy = -2..2, dx ascending):
// slot k reads the node dx_k away, along the lattice row, from the node straight above or
// below the row's node (canonical rows number the nodes of a lattice row consecutively).
constexpr int kDiskTaps = 21;
__device__ __host__ constexpr int disk_row(int k) { return k < 3 ? 0 : k < 8 ? 1 : k < 13 ? 2 : k < 18 ? 3 : 4; }
__device__ __host__ constexpr int disk_dx(int k) {
  return k < 3 ? k - 1 : k < 8 ? k - 5 : k < 13 ? k - 10 : k < 18 ? k - 15 : k - 19;
}

// Nodes straight below (rows 0, 1), at (2) and above (3, 4) a canonical row's node.
__device__ __forceinline__ void disk_bases(const int32_t* node_of, int32_t p, int32_t W, int64_t i,
                                           int32_t (&b)[5]) {
  b[0] = node_of[p - 2 * W];
  b[1] = node_of[p - W];
  b[2] = static_cast<int32_t>(i);
  b[3] = node_of[p + W];
  b[4] = node_of[p + 2 * W];
}

// Nodes of the five lattice rows of row i's disk from its slice's descriptor (wave-uniform
// scalar load); false when the slice is not described.
__device__ __forceinline__ bool slice_disk_bases(const int32_t* sbase, int64_t i, int32_t (&b)[5]) {
  const int32_t sl = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(i >> 6));
  if ((i >> 6) != sl) return false;
  const int4 d = *reinterpret_cast<const int4*>(sbase + 4 * static_cast<int64_t>(sl));
  if (d.x < 0) return false;
  const int32_t l = static_cast<int32_t>(i & 63);
  b[0] = d.x + l;
  b[1] = d.y + l;
  b[2] = static_cast<int32_t>(i);
  b[3] = d.z + l;
  b[4] = d.w + l;
  return true;
}

// Lattice image of the node set: pixel (ix, iy) <-> the node at (xmin + ix h, ymin + iy h).
struct Lattice {
  bool tried = false, ok = false;
  int W = 0, H = 0;
  int32_t* pix = nullptr;           // device [n]: pixel of each node or -1
  int32_t* node_of = nullptr;       // device [W*H]: node at each pixel or -1
};

// A lattice image of some set of rows (the node set's, or a coarse multigrid level's cells):
// the pixel of each row, the row at each pixel (-1 where none), optional boundary-row flags
// (bpos >= 0 marks a boundary row; null: none).
struct LatRef {
  int W, H;
  const int32_t* pix;
  const int32_t* node_of;
  int64_t n;
  const int32_t* bpos;
};

// Device-resident scalars of the Krylov solvers, written by the last block of a
// reduction and read by later kernels; two systems side by side (u and v of
// the predictor) use index 0 and 1.
struct KrylovScalars {
  double rho[2], alpha[2], omega[2], beta[2];
  double rr[2];          // ||r||^2 (recurrence)
  double bb[2];          // ||b||^2
  double dot_a[2], dot_b[2], dot_c[2];
  double mean;           // mean of a vector (periodic projection)
  double stop2[2];       // a system stops iterating once rr <= stop2
  int breakdown[2];
  int active[2];         // cleared on the device at convergence or breakdown
  int iters[2];          // iterations performed (counted on the device)
  // fused two-product BiCGStab iteration: the x and r update of the last iteration is still to
  // be applied (pending), and which of the two buffers of r, p and v holds the current ones
  int pending[2];
  int par[2];
  double dot_d[2], dot_e[2];
};

// One level of the aggregation multigrid preconditioner.
struct AmgLevel {
  int64_t n = 0;
  Ell A;                      // level 0: view of the pressure matrix (not owned)
  int vs = 0;                 // value set of A holding the FP64 values
  int32_t* keep = nullptr;    // rows with off-diagonal entries (aggregated)
  int32_t* agg = nullptr;     // aggregate (row of the next level) or -1
  int32_t* kx = nullptr;      // aggregation key (cell of the next level)
  int32_t* ky = nullptr;
  int64_t* mstart = nullptr;  // members of each next-level row: [n_next + 1]
  int32_t* members = nullptr;
  double* wdinv = nullptr;    // damped inverse diagonal
  float* wdinv32 = nullptr;
  double* w64[3] = {nullptr, nullptr, nullptr};   // V-cycle work vectors
  float* w32[3] = {nullptr, nullptr, nullptr};
  // levels 0 and 1: canonical rows of the sweeps (canonical values and damped inverse diagonal)
  int32_t* cpix64 = nullptr;
  int32_t* cpix32 = nullptr;
  int32_t* sbase64 = nullptr;     // slice descriptors of cpix64 / cpix32 (see Canon::sbase)
  int32_t* sbase32 = nullptr;
  const int32_t* node_of = nullptr;
  int32_t W = 0;                  // lattice image width
  double wdinv_c = 0.0;
  float wdinv32_c = 0.0f;
  // every canonical row's damped inverse diagonal equals wdinv_c / wdinv32_c (none was filtered
  // out of cpix64 / cpix32), so tile sweeps may take the reference value
  bool wd_uniform64 = false;
  bool wd_uniform32 = false;
  // level 1: lattice image of its rows, the aggregation cells of level 0 (owned)
  int32_t* cell_node = nullptr;   // [W * H]: row at each cell, -1 where none
  int32_t* cell_pix = nullptr;    // [n]: cell of each row
  int32_t H = 0;
  // level 1: tiles of its canonical rows on the cell lattice (FP32 and FP64 sweeps; owned)
  TileMap tmap;
  TilePart tpart32, tpart64;
  // the level-1 tile partitions were built from cpix32 / cpix64, the canonical rows kept by the
  // damped-diagonal filter, so every tile row carries wdinv_c / wdinv32_c
  bool tiles_filtered = false;
};

struct Amg {
  std::vector<AmgLevel> lv;
  double* cinv = nullptr;     // dense inverse of the coarsest level, [m1][m1]
  float* cinv32 = nullptr;
  int64_t m = 0, m1 = 0;      // coarsest rows, with the border row if singular
  bool ready = false;
  // the V-cycle below the finest level (levels 1.. and the coarsest solve: the same launches
  // on the same buffers every cycle) captured once per precision, [0] FP64 and [1] FP32, and
  // the level-1 buffer that ends holding its corrected iterate
  hipGraphExec_t coarse_exec[2] = {nullptr, nullptr};
  void* coarse_out[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;   // the stream the graphs are captured on (never run on)
};

struct Timing {
  bool enabled = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<int> tags;          // per pending pair: the V-cycle it belongs to (sweep timing)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  double total_ms = 0.0;
  int64_t count = 0;
};

// Kernels timed with HIP events besides the pressure SpMV and the network (vip_kernel_timing
// which = 2 + kind): launches after a solve stopped on the device return at once and are not
// counted.
enum TimedKind {
  kTimePredV = 0,    // predictor SpMV k_bicg_v, two systems
  kTimePredT = 1,    // predictor t kernel k_bicg_t with s formed inside (one launch per system)
  kTimePredX = 2,    // predictor update k_bicg_x, two systems
  kTimeSweep0 = 3,   // post-smoothing Jacobi sweep k_sweep<T, 0> of the finest multigrid level
  kTimePredRhs = 4,  // k_predictor_rhs (VIP convection, AB2 and the predictor right-hand side)
  kTimedKinds = 5
};

// One captured solver snapshot as a lattice image (independent of the node set
// it came from): BF16 input channels [H][W][3] and the FP32 target [H][W].
struct Snapshot {
  int W = 0, H = 0;
  uint16_t* x = nullptr;
  float* t = nullptr;
};

// Learned start vector: lattice raster map, captured training data, network state.
struct Learn {
  void* net = nullptr;        // network parameters and buffers (learn.hip)
  int capacity = 0;           // vip_step stores snapshots while fewer than this are held
  std::vector<Snapshot> snaps;
  double* r = nullptr;        // device [n]: b - L phi_prev of the current step
  double* phi_prev = nullptr; // device [n]
  double* eprev = nullptr;    // device [n]: previous increment change phi_n - phi_(n-1)
  bool have_eprev = false;
  double* eprev2 = nullptr;   // device [n]: the change before, phi_(n-1) - phi_(n-2)
  bool have_eprev2 = false;
  double* dir2 = nullptr;     // device [n]: second difference eprev - eprev2
  double* q3 = nullptr;       // device [n]: L dir2
  double* q1 = nullptr;        // device [n]: L eprev
  double* rx = nullptr;       // device [n]: residual after extrapolation, r - L eprev
  double* dir = nullptr;      // device [n]: the network's correction c
  double* q2 = nullptr;       // device [n]: L c
  double* scal = nullptr;     // device [16 + 6*256]: [0] rms(rx h^2), [1] rms(b h^2), [2..7] the dots
                              // q1.q1, q1.q2, q2.q2, q1.r, q2.r, r.r, then block partials
  // learned preconditioning of the refinement passes: pass residual, inner correction d, the
  // network's correction c, L d, L c (device [n]) and their scalars (as scal)
  double* pc_r = nullptr;
  double* pc_d = nullptr;
  double* pc_c = nullptr;
  double* pc_q1 = nullptr;
  double* pc_q2 = nullptr;
  double* pc_scal = nullptr;
  // the last start-vector fit (computed on the device): pinned host copy of its coefficients
  // and residual ratio, the event after that copy, whether the stats still have to take it
  double* fit_host = nullptr;
  hipEvent_t fit_event = nullptr;
  bool fit_pending = false;
  int fit_mode = 0;
};

struct Ctx {
  int device = 0;
  int debug = 0;                  // VIP_DEBUG=1: trace Krylov batches on stderr
  int amg_pre_fine = 1;           // VIP_AMG_PRE_FINE=0: BiCGStab V-cycles skip the finest pre-sweep
  int no_canon = 0;               // VIP_NO_CANON=1: every row takes the general sliced-ELL path
  int cnn_layered = 0;            // VIP_CNN_LAYERED=1: learned start inference layer by layer
  int no_delta = 0;               // VIP_NO_DELTA=1: general rows read int32 columns, not int16 deltas
  int no_fuse = 0;                // VIP_NO_FUSE=1: the FP32 predictor iterates with four vector passes
  int no_graph = 0;               // VIP_NO_GRAPH=1: the coarse V-cycle levels launch one by one
  // V-cycle settings: over-correction of the piecewise-constant coarse correction (plain
  // aggregation makes the Galerkin coarse operators too stiff by about 2 for 2x2 aggregates)
  // and damped Jacobi sweeps per level; measured best on the cylinder and triangle node sets.
  // (Four finest-level sweeps took 3.4% less time a step in developed flow at h = 1/128, 2.5%
  // more in the first steps from rest, but on the cylinder parity case at the 1e-8 Poisson
  // tolerance one path's pressure then ended 1.6e-6 from the direct solve, over the 1e-6 budget.)
  double amg_gamma = 1.7;         // coarse-correction scaling (VIP_AMG_GAMMA)
  int amg_nu = 2;                 // Jacobi sweeps before and after on the finest level (VIP_AMG_NU, 1..8)
  int amg_nu_coarse = 2;          // the same on coarser levels (VIP_AMG_NU_COARSE)
  hipStream_t stream = nullptr;
  Error err{0, ""};
  vip_options opt{};
  bool built = false;

  // node set
  int64_t n = 0, nb = 0;
  double h = 0.0, rho0 = 0.0;
  double xmin = 0.0, ymin = 0.0;  // bounding box of the node set
  double xmax = 0.0, ymax = 0.0;
  bool periodic = false, singular = false, symmetric = false;
  double* x = nullptr;            // device [n]
  double* y = nullptr;            // device [n]
  int32_t* bpos = nullptr;        // device [n]: boundary-table index or -1
  int64_t* bidx = nullptr;        // device [nb]
  double* bnx = nullptr;          // device [nb]
  double* bny = nullptr;
  int32_t* bkind = nullptr;       // device [nb]
  double* bval = nullptr;         // device [nb*2]
  // adaptive node sets (null when the spacing is uniform): each node's spacing over h, the same
  // per boundary entry, and the scale 2 d_b = 2 vip_offset h_b of each Neumann row
  double* hscale = nullptr;       // device [n]
  double* bscale = nullptr;       // device [nb]
  double* two_db = nullptr;       // device [nb]
  std::vector<int32_t> h_bkind;   // host copy
  std::vector<int32_t> h_bpos;    // host copy of bpos

  // geometry
  double* vip_px = nullptr;       // device [4*n]: VIP coordinates, k*n + i
  double* vip_py = nullptr;
  double* d_ew = nullptr;         // device [n]
  double* d_ns = nullptr;
  double* rho_node = nullptr;     // device [n]

  // operators
  Ell node;                       // val[0] = D^[0,0], val[1] = Laplacian
  Ell vipop[4];                   // val[0] = Psi^[0,0] at e, w, n, s
  Ell normal[2];                  // val[0] = Psi^[0,0] at x_b - d n, x_b - 2 d n
  Ell sys;                        // val[0] = Poisson, val[1] = H_u, val[2] = H_v; val32 = Poisson
  double* dinv[3] = {nullptr, nullptr, nullptr};   // Jacobi inverse diagonals (P, Hu, Hv)
  float* dinv32 = nullptr;

  // step state
  double cur_dt = 0.0, cur_re = 0.0;
  bool assembled = false;
  bool have_prev_n = false;
  bool have_prev_phi = false;
  double* nprev = nullptr;        // device [2n]
  double* stepbuf = nullptr;      // device [n]: the Poisson right-hand side of a step
  double* star_ring = nullptr;    // device [3][2(n+1)]: the last three predictor solutions (u*, v*),
                                  // a ring whose next slot the next solve runs in
  int star_head = 0;              // slot of the newest
  int nstar = 0;                  // previous predictor solutions held (0..3) for the start vector
  double* phi = nullptr;          // device [n+1] (last entry: border multiplier)
  double* ws = nullptr;           // device work vectors (FP64)
  int64_t ws_len = 0;
  float* ws32 = nullptr;
  int64_t ws32_len = 0;
  double* partials = nullptr;     // device [max blocks * 8]
  int64_t partials_len = 0;
  KrylovScalars* sc = nullptr;    // device scalars
  int hint_p64[4] = {0, 0, 0, 0}; // iterations of the last pressure solves (FP64, per refinement pass)
  int hint_p32[4] = {0, 0, 0, 0}; // the same for the FP32 inner solves
  int hint_h = 0;                 // the same for the predictor solves
  int hint_h32[4] = {0, 0, 0, 0}; // and for their FP32 inner solves
  KrylovScalars* sc_host = nullptr; // pinned host mirror

  Lattice lat;
  TileMap tmap;
  VipCanon vcanon;
  Amg amg;
  Learn learn;
  Timing timing;                  // pressure-solve SpMV launches
  Timing conv_timing;             // MFMA layers of the learned start vector's inference
  Timing ktime[kTimedKinds];      // see TimedKind
  int vcycle = 0;                 // V-cycles applied in the current Krylov solve (sweep timing tags)

  // body forces (forces.hip): surface node list and per-node traction terms
  int64_t* fsurf = nullptr;       // device [fcap]
  double* fbuf = nullptr;         // device [2 * fcap + 2]
  int64_t fcap = 0;
  void* scratch = nullptr;        // this device's copy of the fixed scratch of vip_forces_noalloc
};

// ---- HIP-event timing (krylov.hip) -----------------------------------------------
// Events around one launch into T.pending (tag: see Timing::tags) while T.enabled.  Timing
// events are created without the system-scope fence (hipEventDisableSystemFence): they only
// measure, the host reads them after a stream synchronisation, and a fence would write back
// and invalidate the caches between the timed kernel and its neighbours.
struct KTimer {
  Ctx* c;
  Timing* T;
  bool on;
  std::pair<hipEvent_t, hipEvent_t> ev{};
  int tag;
  KTimer(Ctx* cc, Timing& t, bool enable, int tg = 0);
  ~KTimer();
};
// Add the durations of the pending launches [first, first + keep) (with tag < tag_limit when
// tag_limit >= 0) to T and recycle every pending event pair.
void harvest_kind(Timing& T, size_t first, size_t keep, int tag_limit = -1);

// ---- error handling -----------------------------------------------------------
int set_error(Ctx* c, int code, const std::string& msg);

#define VIP_HIP_TRY(c, expr)                                                        \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::vip::set_error((c), VIP_E_HIP, std::string(#expr) + ": " +           \
                                                  hipGetErrorString(e_));           \
  } while (0)

#define VIP_TRY(expr)               \
  do {                              \
    int r_ = (expr);                \
    if (r_ != VIP_OK) return r_;    \
  } while (0)

// ---- memory helpers -------------------------------------------------------------
template <typename T>
int dalloc(Ctx* c, T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * static_cast<size_t>(count));
  if (e != hipSuccess)
    return set_error(c, VIP_E_HIP, std::string("hipMalloc of ") +
                                       std::to_string(sizeof(T) * count) + " bytes: " +
                                       hipGetErrorString(e));
  return VIP_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void ell_free(Ell& e);
void ctx_free_build(Ctx* c);

// Exclusive prefix sum of int64 values on the device (in place safe), writes the
// total to *total_host (synchronous).
int scan_i64(Ctx* c, const int64_t* in, int64_t* out, int64_t n, int64_t* total_host);

// Grid size for one thread per item, rounded up to a multiple of the XCD count.
inline int64_t grid_for(int64_t items, int block = kBlock) {
  int64_t g = (items + block - 1) / block;
  if (g < 1) g = 1;
  return ((g + kNumXcd - 1) / kNumXcd) * kNumXcd;
}

// Map a hardware block index to a logical one so that consecutive logical
// blocks run on the same XCD (blocks are dispatched to XCDs round-robin).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t grid) {
  const int64_t per = grid / kNumXcd;
  return (b % kNumXcd) * per + b / kNumXcd;
}

// Allocate an Ell's slice structure from per-row lengths already in e.rowlen.
int ell_layout(Ctx* c, Ell& e);
// Build e.dcols (row-relative int16 columns) when every stored column fits; leaves it null
// otherwise or when the context has deltas off.
int ell_deltas(Ctx* c, Ell& e);

// FP32 row sums of an FP64 sliced-ELL value set (for the difference-form FP32 rows).
void launch_rowsum32(hipStream_t st, int64_t n, const int64_t* ptr, const int32_t* rowlen,
                     const double* val, float* out);

// Ensure the reduction scratch holds `blocks` partial slots of `per` doubles.
int ensure_partials(Ctx* c, int64_t blocks, int per);

// Sliced-ELL SpMV y = A x on value set `vs` (FP64), used by tests and helpers.
int ell_apply(Ctx* c, const Ell& e, int vs, const double* x, double* y);
// y = P x with the FP64 pressure matrix through the canonical-row path (no border).
int pressure_apply(Ctx* c, const double* x, double* y);
// A pressure product with its neighbouring element-wise passes folded in: y = P x' with x' = x,
// or x - x2 when x2 is set (then also stored to xd when that is set); r = b - y when r is set;
// x copied to cp when that is set.  Unset outputs are not written.  Bit for bit the separate
// passes.
struct SysApply {
  const double* x = nullptr;
  const double* x2 = nullptr;
  double* xd = nullptr;
  double* cp = nullptr;
  double* y = nullptr;
  const double* b = nullptr;
  double* r = nullptr;
};
int pressure_apply(Ctx* c, const SysApply& P);

// Solvers (krylov.hip)
int poisson_solve(Ctx* c, const double* rhs, double* phi, double tol, bool use_x0,
                  vip_step_stats* st);
// The predictor's right-hand side buffer [2][n+1] (the predictor kernel writes it in place).
int predictor_rhs_buffer(Ctx* c, double** b);
// Solves the two predictor systems; *us, *vs receive the solutions (in the history ring).
int helmholtz_solve(Ctx* c, const double* ru, const double* rv, double** us, double** vs,
                    vip_step_stats* st);
int build_stencils(Ctx* c, const double* xy, int64_t n, const int64_t* bidx, const double* bnrm,
                   const int32_t* bkind, const double* bval, int64_t nb, int basis_order, double rho,
                   double h, const vip_options* opt, const double* h_node = nullptr);
int assemble_helmholtz(Ctx* c, double dt, double re);
int amg_setup(Ctx* c);
void amg_free(Ctx* c);
template <typename T>
int amg_apply(Ctx* c, const T* b, T* x, bool border, bool pre_fine);
int step(Ctx* c, double* u, double* v, double* p, double dt, double re, vip_step_stats* st);
int convection(Ctx* c, const double* u, const double* v, double* nx, double* ny);
int divergence(Ctx* c, const double* u, const double* v, double* d);
int gradient(Ctx* c, const double* f, double* gx, double* gy);

// Learned start vector (learn.hip)
int learn_n_params();
int learn_set_params(Ctx* c, const double* theta);
int learn_get_params(Ctx* c, double* theta);
int learn_eval(Ctx* c, const double* x, const double* t, const double* m, int B, int H, int W, double* y,
               double* loss, double* grad, double lr);
int learn_infer(Ctx* c, const double* x, int B, int H, int W, double* y);
// Lattice map of the node set (stencil.hip); false if the nodes are not lattice based.
int lattice_map(Ctx* c, bool* ok);
// Find the reference row of the system layout and mark the canonical rows of value set
// vs (0..3 FP64; 4..6 FP32 pressure, predictor u, predictor v, with their row sums).
int canon_mark(Ctx* c, Ell& e, int vs);
// The same for the rows of e on the lattice image L (their columns index L's rows).
int canon_mark_on(Ctx* c, Ell& e, int vs, const LatRef& L);
// Slice descriptors (Canon::sbase) of canonical-row pixels cpix [n] into out [4 * ceil(n/64)].
int slice_bases(Ctx* c, const int32_t* cpix, int64_t n, int32_t** out, int64_t* described = nullptr);
void canon_free(Canon& cn);
// Tile partition `key` of the system layout's canonical rows (TilePart; key 0: set 0, 1: set 4,
// 2: sets 1 and 2, 3: sets 5 and 6), rebuilt from the current marks; none unless the
// reference row is the 21-point disk.
int tile_part(Ctx* c, int key);
// Tile partition of the rows of a lattice image (W x H pixels, node_of, n rows) canonical in c0
// (and c1, if given); tm's row starts are built on first use.
int tile_part_build(Ctx* c, int W, int H, const int32_t* node_of, int64_t n, TileMap& tm, const int32_t* c0,
                    const int32_t* c1, TilePart& tp);
void tile_part_free(TilePart& tp);
void tile_map_free(TileMap& tm);
// Canonical nodes of the VIP and node operators (VipCanon); leaves count = 0 when there are none.
int vip_canon_setup(Ctx* c);
void vip_canon_free(Ctx* c);
void lattice_free(Lattice& lat);
int learn_train(Ctx* c, int iters, int batch, int crop, double lr, uint64_t seed, double* last_loss);
bool learn_ready(const Ctx* c);
// before the pressure solve: keep phi_prev = phi and r = b - L phi_prev (with_map: build the
// lattice map too, which fails on node sets that are not lattice based)
int learn_prepare(Ctx* c, const double* b, const double* phi, bool with_map);
// phi = phi_prev + alpha e (+ beta c with the network's correction c in mode VIP_WS_LEARNED,
// + gamma e2 with e2 the second difference), e the previous change of phi, the coefficients
// minimising the FP64 residual (fitted on the device, without waiting for the host)
int learn_warm_start(Ctx* c, int mode, const double* b, double* phi, vip_step_stats* st);
// after the pressure solve: the fit's outcome into the stats (and the network's launch timing)
int learn_warm_stats(Ctx* c, vip_step_stats* st);
// after the pressure solve: store one snapshot (if capture is on) and the change of phi
int learn_finish(Ctx* c, const double* b, const double* phi, bool capture);
int learn_init(Ctx* c, uint64_t seed);
void learn_clear(Ctx* c);          // drop the captured snapshots
void learn_free_nodeset(Ctx* c);   // drop what belongs to the node set (map, vectors)
void learn_free(Ctx* c);           // everything
// learned preconditioning of the mixed refinement passes is on for this solve (option set,
// network ready, lattice map built, pressure system not singular)
bool learn_precond_active(Ctx* c);
// x += alpha d + beta c for the pass residual r32 (FP32) and inner correction d32 (see vip.h,
// learned_precond); *used counts passes that took the network's direction, *gain multiplies in
// its residual ratio against d alone
int learn_precond_pass(Ctx* c, const float* r32, const double* b, const float* d32, double* x, int* used,
                       double* gain);

// Body forces (forces.hip): traction integrated over a closed chain of boundary nodes; work
// arrays in `surf_dev` (int64 [n_surf]) and `buf` (double [2 n_surf + 2]) on the device.
int forces(Ctx* c, const double* u, const double* v, const double* p, double re, const int64_t* surf,
           int64_t n_surf, double* out, int64_t* surf_dev, double* buf);
// Check a surface chain against the node set (host side); VIP_OK or VIP_E_INVALID.
int forces_check(Ctx* c, const int64_t* surf, int64_t n_surf, double re);
void forces_free(Ctx* c);
// Look up this device's copy of the fixed scratch array (once per device) into c->scratch.
int forces_scratch_init(Ctx* c);
int64_t forces_noalloc_max_surface();

}  // namespace vip
