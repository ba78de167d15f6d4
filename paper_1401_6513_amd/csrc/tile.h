// Lattice tiles of canonical rows (device side).
//
// On a lattice-based node set the canonical rows (translation-invariant 21-point disks, see
// Canon) are computed tile by tile: a block copies the input vector over a 64 x 16 pixel tile
// of the lattice plus a halo of two pixels into LDS (one coalesced row at a time where the
// row's nodes are numbered consecutively) and each lane then reads its 21 taps from LDS.
// Rows that are not canonical, and nodes off the lattice, form the irregular list, which the
// first blocks of the same launch take one row per thread through the row-by-row path.
// Every row is visited exactly once, in an order fixed by the partition alone, so reductions
// over the rows give the same bits whichever way a row's value is computed.
#pragma once

#include "vip_internal.h"

namespace vip {

constexpr int kTileLdsW = kTileX + 4;
constexpr int kTileLdsH = kTileY + 4;

struct TileView {
  const int32_t* tiles = nullptr;   // null: no tile partition
  int64_t ntiles = 0;
  const int32_t* irr = nullptr;
  int64_t nirr = 0;
  const uint32_t* rec = nullptr;    // per listed tile: its record (TileMeta layout)
  const int32_t* node_of = nullptr;
  int ntx = 0, W = 0, H = 0;
  int tile_blocks = 0;              // blocks taking tiles (a multiple of the XCD count)
  int irr_blocks = 0;               // blocks [0, irr_blocks) take the irregular rows (the same)
};

// View of a partition of the rows of a lattice image (W x H pixels, node_of, row starts in tm).
inline TileView tile_view_of(const TilePart& tp, const TileMap& tm, const int32_t* node_of, int W, int H) {
  TileView v;
  if (!tp.tiles && !tp.irr) return v;
  v.tiles = tp.tiles;
  v.ntiles = tp.ntiles;
  v.irr = tp.irr;
  v.nirr = tp.nirr;
  v.rec = tp.rec;
  v.node_of = node_of;
  v.ntx = tm.ntx;
  v.W = W;
  v.H = H;
  v.tile_blocks = tp.tile_blocks;
  v.irr_blocks = tp.irr_blocks;
  return v;
}

// View of a partition of the node lattice.
inline TileView tile_view(const Ctx* c, const TilePart& tp) {
  return tile_view_of(tp, c->tmap, c->lat.node_of, c->lat.W, c->lat.H);
}

// A tile's record, staged in LDS from its 256-byte block in the partition (one coalesced load):
// word 0 tx, 1 ty, 2..21 the start nodes of halo rows 0..19 (-1 where a row's 68 pixels are
// not consecutive nodes), 32..63 the 16 tile-row masks (bit lx: the node at pixel lx of the
// row is a tile row) as (low, high) word pairs.
struct TileMeta {
  uint32_t w[kTileRecWords];
  __device__ __forceinline__ int tx() const { return static_cast<int>(w[0]); }
  __device__ __forceinline__ int ty() const { return static_cast<int>(w[1]); }
  __device__ __forceinline__ int32_t rs(int r) const { return static_cast<int32_t>(w[2 + r]); }
  __device__ __forceinline__ uint64_t bits(int r) const {
    return static_cast<uint64_t>(w[32 + 2 * r]) | (static_cast<uint64_t>(w[33 + 2 * r]) << 32);
  }
};
static_assert(2 + kTileLdsH <= 32 && 32 + 2 * kTileY == kTileRecWords, "tile record layout");

// Stage listed tile k: its record, then (with load_x) the LDS copy of NS vectors over the
// tile and its halo (0 at pixels without a node), every thread issuing all of its loads before
// storing.  Starts and ends with a block barrier.
template <typename T, int NS, typename F>
__device__ __forceinline__ void tile_stage_fn(const TileView& V, int64_t k, F&& xf,
                                              T (&t)[NS][kTileLdsH][kTileLdsW], TileMeta& m, bool load_x);

template <typename T, int NS>
__device__ __forceinline__ void tile_stage(const TileView& V, int64_t k, const T* const (&x)[NS],
                                           T (&t)[NS][kTileLdsH][kTileLdsW], TileMeta& m, bool load_x) {
  tile_stage_fn<T, NS>(
      V, k, [&](int s, int32_t node) __attribute__((always_inline)) { return x[s][node]; }, t, m, load_x);
}

// Staging shape: wave w stages halo rows w, w + 4, ... at columns 0..63 (lane = column, one
// contiguous segment per load); the first 4 kTileLdsH threads stage columns 64..67 of every row.
// Few index values live across the tile loop this way (with a flat element index the per-thread
// row, column and LDS address of every element were kept in registers).
constexpr int kStageWaves = kBlock / 64;
constexpr int kStageRows = kTileLdsH / kStageWaves;   // halo rows per wave
constexpr int kStageEdge = kTileLdsW - 64;            // columns past the wavefront width
static_assert(kTileLdsH % kStageWaves == 0 && kStageEdge > 0 && kStageEdge * kTileLdsH <= kBlock,
              "tile staging shape");

// The nodes this thread stages for the tile of record m: node[j] for halo row wave + 4 j at
// its lane's column, node[kStageRows] for its edge element; -1 where there is no node.
__device__ __forceinline__ void tile_stage_nodes(const TileView& V, const TileMeta& m,
                                                 int32_t (&node)[kStageRows + 1]) {
  const int tid = static_cast<int>(threadIdx.x);
  const int wave = tid >> 6, lane = tid & 63;
  const int tx = m.tx(), ty = m.ty();
  auto node_at = [&](int r, int cc) __attribute__((always_inline)) -> int32_t {
    const int32_t rs = m.rs(r);
    if (rs >= 0) return rs + cc;
    const int gx = tx * kTileX + cc - 2, gy = ty * kTileY + r - 2;
    if (gx >= 0 && gx < V.W && gy >= 0 && gy < V.H) return V.node_of[static_cast<int64_t>(gy) * V.W + gx];
    return -1;
  };
#pragma unroll
  for (int j = 0; j < kStageRows; ++j) node[j] = node_at(wave + j * kStageWaves, lane);
  node[kStageRows] = tid < kStageEdge * kTileLdsH ? node_at(tid / kStageEdge, 64 + tid % kStageEdge) : -1;
}

// Store this thread's staged values (one per system and staged element) into the LDS tile.
template <typename T, int NS>
__device__ __forceinline__ void tile_stage_store(const T (&val)[NS][kStageRows + 1],
                                                 T (&t)[NS][kTileLdsH][kTileLdsW]) {
  const int tid = static_cast<int>(threadIdx.x);
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int j = 0; j < kStageRows; ++j)
#pragma unroll
    for (int s = 0; s < NS; ++s) t[s][wave + j * kStageWaves][lane] = val[s][j];
  if (tid < kStageEdge * kTileLdsH)
#pragma unroll
    for (int s = 0; s < NS; ++s) t[s][tid / kStageEdge][64 + tid % kStageEdge] = val[s][kStageRows];
}

// The same with the staged values given by xf(s, node) (system s at a node).
template <typename T, int NS, typename F>
__device__ __forceinline__ void tile_stage_fn(const TileView& V, int64_t k, F&& xf,
                                              T (&t)[NS][kTileLdsH][kTileLdsW], TileMeta& m, bool load_x) {
  const int tid = static_cast<int>(threadIdx.x);
  __syncthreads();
  if (tid < kTileRecWords) m.w[tid] = V.rec[k * kTileRecWords + tid];
  __syncthreads();
  if (!load_x) return;
  int32_t node[kStageRows + 1];
  tile_stage_nodes(V, m, node);
  T val[NS][kStageRows + 1];
#pragma unroll
  for (int j = 0; j <= kStageRows; ++j)
#pragma unroll
    for (int s = 0; s < NS; ++s) val[s][j] = node[j] >= 0 ? xf(s, node[j]) : T(0);
  tile_stage_store<T, NS>(val, t);
  __syncthreads();
}

constexpr int kTileRowsPerWave = kTileY / (kBlock / 64);

// The wave's local row ly = wave + 4 k of the staged tile: the lane's node, or -1 where its
// pixel is not a tile row.  The kernels walk k in a loop kept rolled, so that one row's stencil
// operands are live at a time: unrolled over the four rows, the register peak cut occupancy by
// one wave per SIMD, which cost the pressure SpMV about a tenth of its time (measured).
__device__ __forceinline__ int64_t tile_row_id(const TileView& V, const TileMeta& m, int k) {
  const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
  const int ly = wave + k * (kBlock / 64);
  if (!((m.bits(ly) >> lane) & 1ull)) return -1;
  const int32_t rs = m.rs(ly + 2);
  return rs >= 0 ? static_cast<int64_t>(rs) + 2 + lane
                 : static_cast<int64_t>(V.node_of[static_cast<int64_t>(m.ty() * kTileY + ly) * V.W + m.tx() * kTileX + lane]);
}

// Blocks [0, irr_blocks) call irr(i) for the irregular rows, one per thread (they start first
// and overlap the tiles).  The tile blocks call tile(k) for positions k of the tile list: blocks
// are dispatched to the XCDs round-robin, so each XCD gets an equal contiguous share of the
// list (neighbouring tiles then share its L2), which its blocks take in turn.
template <typename Tile, typename Irr>
__device__ __forceinline__ void tile_walk(const TileView& V, Tile&& tile, Irr&& irr) {
  if (static_cast<int>(blockIdx.x) < V.irr_blocks) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < V.nirr;
         k += static_cast<int64_t>(V.irr_blocks) * blockDim.x)
      irr(static_cast<int64_t>(V.irr[k]));
  } else {
    const int64_t b = static_cast<int64_t>(blockIdx.x) - V.irr_blocks;
    const int64_t xcd = b % kNumXcd, j = b / kNumXcd, per = V.tile_blocks / kNumXcd;
    const int64_t t1 = V.ntiles * (xcd + 1) / kNumXcd;
    for (int64_t k = V.ntiles * xcd / kNumXcd + j; k < t1; k += per) tile(k);
  }
}

// A software-pipelined tile walk for kernels whose staged values come from plain loads: while a
// tile is computed from LDS, the loads of the block's next tile are already in flight (its
// operands held in registers) and the record of the tile after that too, so a block always has
// memory requests outstanding (with one tile staged at a time, a block idled between its
// compute and its next tile's loads).  load(s, node) issues the loads of system s's operands at
// a node and returns them as R; value(s, r) forms the staged value from them (computed when the
// tile is stored, a tile later, with the arithmetic of the unpipelined staging).  issue(k, m) is
// called after tile k is in LDS and before the next tile's loads are issued: the place for the
// tile's own row loads (rhat), which the in-order completion counter would otherwise make wait
// for the whole prefetch; compute(k, m) then computes tile k from LDS (record m).  The record
// buffers m[2] alternate between consecutive tiles.  Irregular rows as in tile_walk.
template <typename T, int NS, typename R, typename Load, typename Value, typename Issue, typename Compute,
          typename Irr>
__device__ __forceinline__ void tile_walk_pp(const TileView& V, T (&t)[NS][kTileLdsH][kTileLdsW], TileMeta (&m)[2],
                                             Load&& load, Value&& value, Issue&& issue, Compute&& compute,
                                             Irr&& irr) {
  if (static_cast<int>(blockIdx.x) < V.irr_blocks) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < V.nirr;
         k += static_cast<int64_t>(V.irr_blocks) * blockDim.x)
      irr(static_cast<int64_t>(V.irr[k]));
    return;
  }
  const int tid = static_cast<int>(threadIdx.x);
  const int64_t b = static_cast<int64_t>(blockIdx.x) - V.irr_blocks;
  const int64_t xcd = b % kNumXcd, j = b / kNumXcd, per = V.tile_blocks / kNumXcd;
  const int64_t t0 = V.ntiles * xcd / kNumXcd + j, t1 = V.ntiles * (xcd + 1) / kNumXcd;
  if (t0 >= t1) return;   // block-uniform
  R raw[NS][kStageRows + 1];
  int32_t node[kStageRows + 1];
  auto issue_loads = [&](const TileMeta& mm) __attribute__((always_inline)) {
    tile_stage_nodes(V, mm, node);
#pragma unroll
    for (int jj = 0; jj <= kStageRows; ++jj)
#pragma unroll
      for (int s = 0; s < NS; ++s) raw[s][jj] = load(s, node[jj] >= 0 ? node[jj] : 0);
  };
  // prologue: record and loads of the first tile, record of the second
  uint32_t recw = tid < kTileRecWords ? V.rec[t0 * kTileRecWords + tid] : 0u;
  if (tid < kTileRecWords) m[0].w[tid] = recw;
  __syncthreads();
  issue_loads(m[0]);
  if (t0 + per < t1 && tid < kTileRecWords) recw = V.rec[(t0 + per) * kTileRecWords + tid];
  int cur = 0;
  for (int64_t k = t0; k < t1; k += per) {
    __syncthreads();   // every lane is done with the previous tile's LDS values and record
    {
      T val[NS][kStageRows + 1];
#pragma unroll
      for (int jj = 0; jj <= kStageRows; ++jj)
#pragma unroll
        for (int s = 0; s < NS; ++s) val[s][jj] = node[jj] >= 0 ? value(s, raw[s][jj]) : T(0);
      tile_stage_store<T, NS>(val, t);
    }
    const bool next = k + per < t1;
    if (next && tid < kTileRecWords) m[cur ^ 1].w[tid] = recw;
    __syncthreads();   // tile k staged; the next tile's record in place
    issue(k, m[cur]);
    if (next) {
      issue_loads(m[cur ^ 1]);
      if (k + 2 * per < t1 && tid < kTileRecWords) recw = V.rec[(k + 2 * per) * kTileRecWords + tid];
    }
    compute(k, m[cur]);
    cur ^= 1;
  }
}

}  // namespace vip
