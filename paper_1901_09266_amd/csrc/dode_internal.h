// Internal declarations shared by the host API and the kernel files of libdode.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dode.h"

// Device view of the incidence pattern (CSR by link and CSC by OD), and the
// sliced layouts of the two value copies.  Lines (links for W, ODs for WT)
// come in slices of 64; in WT entry k of a column sits 64*k after its first
// slot, so the 64 lanes that walk 64 neighbouring lines read one run of
// neighbouring values at every step.  In W entries come in pairs (entry k of a
// link at first + 128*(k/2) + k%2, first even), so one load brings two, and a
// slice's links are ranked by degree (longest first; link degrees vary along a
// corridor): the lanes still active at a step hold a prefix of the run and no
// padding is fetched.  Slots past a line's degree are padding (zero).
struct DevPat {
  int32_t P, L, T, H, K;
  int64_t nnz;
  const int32_t* row_ptr;   // [L+1]
  const int32_t* col;       // [nnz]  OD of CSR entry j
  const int32_t* col_ptr;   // [P+1]
  const int32_t* row;       // [nnz]  link of CSC entry jj
  int64_t sr_len, sc_len;   // values per (l, t) block of W / WT
  const int32_t* sr_first;  // [L]          first slot of each link
  const int32_t* sr_col;    // [sr_len]     OD of each W slot
  const int32_t* sr_pos;    // [nnz]        W slot of CSR entry j
  const int32_t* sc_off;    // [ceil(P/64)] first slot of each OD slice
  const int32_t* sc_row;    // [sc_len]     link of each WT slot
  const int32_t* sc_pos;    // [nnz]        WT slot of CSC entry jj
};

// Device view of the value arrays of all clusters.
//   W : sliced by link [C][K][T][sr_len]
//   WT: sliced by OD   [C][K][T][sc_len]
//   scale (FP8 only): [C][K][T][n_ptile], one float per 64-OD column tile
struct DevVals {
  const void* W;
  const void* WT;
  const float* scale;
  int64_t cstride_r;     // K*T*sr_len
  int64_t cstride_c;     // K*T*sc_len
  int32_t n_ptile;       // ceil(P/64)
};

// Forward link tiles come in groups of kFwdTileGroup that share one OD range
// (the range covering all of them): one wave multiplies the group's tiles
// with the same demand operand.
constexpr int32_t kFwdTileGroup = 2;

// Dense MFMA tiles of the assignment blocks (BF16 / FP8 storage).
//   forward:  link tile i (16 links) x OD hull [f_plo[i], f_plo[i] + 32*f_ks[i])
//   adjoint:  OD tile j (16 ODs) x link hull [g_alo[j], g_alo[j] + 32*g_ks[j])
// Values of block (c, l, t) are stored per 16x32 k-step in MFMA operand order
// (lane-major, 8 consecutive k per lane): Fv[c][l][t][kf_total][64 lanes][8].
// The entries are the same codes as the pattern-form arrays (bf16, or E4M3
// with the pattern form's scale per (c, l, t, 64-OD group): scale[...][n_ptile]).
struct DevTiles {
  int32_t nLT = 0, nPT = 0, kf_total = 0, kg_total = 0;
  const int32_t* f_plo = nullptr;
  const int32_t* f_ks = nullptr;
  const int32_t* f_koff = nullptr;
  const int32_t* g_alo = nullptr;
  const int32_t* g_ks = nullptr;
  const int32_t* g_koff = nullptr;
  const void* Fv = nullptr;
  const void* Gv = nullptr;
  const float* scale = nullptr;   // FP8 only: [C][K][T][n_ptile]
  int32_t n_ptile = 0;
  const void* Fc = nullptr;       // FP8 with correction: bf16 tiles, same packing
  const void* Gc = nullptr;
};

struct dode_dar {
  dode_dims dims{};
  int32_t C = 0;
  int64_t nnz = 0;
  dode_dtype storage = DODE_F32;
  int device = 0;
  int32_t* d_row_ptr = nullptr;
  int32_t* d_col = nullptr;
  int32_t* d_col_ptr = nullptr;
  int32_t* d_row = nullptr;
  int32_t* d_csc2csr = nullptr;   // CSC slot -> CSR slot
  int32_t* d_row_of_nz = nullptr; // link of CSR slot j
  int64_t sr_len = 0, sc_len = 0;   // sliced value layouts (see DevPat)
  int32_t* d_sr_first = nullptr;
  int32_t* d_sr_col = nullptr;
  int32_t* d_sr_pos = nullptr;
  int32_t* d_sc_off = nullptr;
  int32_t* d_sc_row = nullptr;
  int32_t* d_sc_pos = nullptr;
  void* d_W = nullptr;
  void* d_WT = nullptr;
  float* d_scale = nullptr;
  int64_t device_bytes = 0;
  std::vector<int32_t> h_row_ptr, h_col, h_col_ptr, h_row, h_csc2csr;
  // MFMA tile layout (BF16 / FP8 storage only)
  bool has_tiles = false;
  DevTiles tiles;
  int32_t* d_tile_meta = nullptr;   // f_plo | f_ks | f_koff | g_alo | g_ks | g_koff
  std::vector<int32_t> h_tile_meta; // host copy
  int32_t* d_posf = nullptr;        // [nnz] element offset of CSR slot j in a forward block
  int32_t* d_posg = nullptr;        // [nnz] element offset of CSC slot jj in an adjoint block
  void* d_Fv = nullptr;
  void* d_Gv = nullptr;
  void* d_Fc = nullptr;             // correction tiles (FP8 with DODE_DAR_CORRECTION)
  void* d_Gc = nullptr;
  bool has_corr = false;
  std::vector<int32_t> h_posf, h_posg;

  DevPat pat() const {
    return DevPat{dims.P, dims.L, dims.T, dims.H, dims.K, nnz, d_row_ptr, d_col, d_col_ptr, d_row,
                  sr_len, sc_len, d_sr_first, d_sr_col, d_sr_pos, d_sc_off, d_sc_row, d_sc_pos};
  }
  DevVals vals() const {
    return DevVals{d_W, d_WT, d_scale, (int64_t)dims.K * dims.T * sr_len,
                   (int64_t)dims.K * dims.T * sc_len, (dims.P + 63) / 64};
  }
};

// Device view of a route-choice structure (see dode_routes_create).
struct DevRoutes {
  int32_t P, L, T, H, K, n_paths;
  int64_t nnz, n_pairs;
  const int32_t* path_od;     // [n_paths]
  const int32_t* pair_ptr;    // [n_paths+1]
  const int32_t* pair_nz;     // [n_pairs]
  const int32_t* pair_path;   // [n_pairs]
  const int32_t* od_ptr;      // [P+1]   paths grouped by OD
  const int32_t* od_paths;    // [n_paths]
  const int32_t* nz_ptr;      // [nnz+1] pairs grouped by pattern entry
  const int32_t* nz_pairs;    // [n_pairs]
};

struct dode_routes {
  DevRoutes dv{};
  int device = 0;
  int32_t* d_buf = nullptr;   // all index arrays above, one allocation
};

// Element strides of the per-day state arrays.  Entry (day d, row r, col k)
// of an array with day stride sd, row stride sr and block stride sb sits at
//   d*sd + r*sr + (k/4)*sb + k%4
// (col_at): columns come in blocks of 4.
//   Q, A, G : (q_d, q_t, q_b), rows t, cols p     X, Xhat : (x_d, x_h, x_b)
//   R       : (r_d, r_s, r_b), rows = minibatch slot s (or h for full rows)
// Caller arrays are day-major and contiguous (q_d = T*P, q_t = P, q_b = 4).
// A plan keeps interval-major copies so a minibatch's rows are contiguous
// across days: the sparse pattern path uses q_d = P, q_t = D*P, q_b = 4; the
// matrix-core path uses day-blocked rows, [row][col/4][day][4] with nb
// blocks per row (q_d = 4, q_b = 4*D, q_t = nb*4*D), so the 16 days of an
// MFMA column tile read 4 consecutive columns as one 256-byte run.
struct Layout {
  int64_t q_d, q_t, x_d, x_h, r_d, r_s;
  int64_t q_b = 4, x_b = 4, r_b = 4;
};

__host__ __device__ __forceinline__ int64_t col_at(int64_t k, int64_t sb) {
  return (k >> 2) * sb + (k & 3);
}

inline Layout day_major(const dode_dims& dm) {
  return Layout{(int64_t)dm.T * dm.P, dm.P, (int64_t)dm.H * dm.L, dm.L, (int64_t)dm.H * dm.L, dm.L,
                4, 4, 4};
}

// Blocks per row of the day-blocked plan layout for n columns: the packed tile
// ranges reach at most 31 columns past the last one, so 8 zero blocks follow.
__host__ __device__ inline int64_t blocked_row_blocks(int64_t n) { return (n + 3) / 4 + 8; }

// Optimizer settings as the kernels see them.
struct StepArgs {
  double eta;
  double eps;
  int32_t optimizer;   // 0 Adagrad, 1 fixed step
};

// Schedule of one minibatch ("chunk") for the grouped kernels.  Minibatch j
// of an epoch holds positions j0 = j*bh .. j0+bh-1 of each cluster's
// permutation of the H observation intervals.
//   perm[c][H]      the epoch's permutation of cluster c
//   pos[c][H]       its inverse (position of interval h)
//   touched[c][mt][K+3]  descriptors of the departure intervals the minibatch
//                   reaches: [t, lag mask (low, high word), slot of t+0, ...,
//                   slot of t+K-1]; bit l of the mask is set when t+l is in the
//                   minibatch, slot -1 when it is not.  Entries with t = -1 pad
//                   the list; they are spread evenly between the used ones.
//   epoch           device epoch counter (graph replays) or nullptr; when set,
//                   the kernels add (*epoch) * perm_e / touched_e to the pointers
constexpr int kDescT = 0, kDescMask = 1, kDescSlot = 3;
__host__ __device__ inline int32_t desc_width(int32_t K) { return K + 3; }

struct ChunkSched {
  const int32_t* perm;
  const int32_t* pos;
  const int32_t* touched;
  int32_t j0;
  int32_t bh;
  int32_t max_touched;
  const int32_t* epoch;
  int64_t perm_e;
  int64_t touched_e;
  // item order of the matrix-core adjoint: 0 = (cluster, reached interval,
  // day group, OD tile), OD tile fastest, over the evenly spread descriptor
  // list; 1 = (cluster, OD tile, day group, reached interval), interval
  // fastest, over the descriptors sorted by t (consecutive waves then read the
  // same residual rows); 2 = as 1 with a chunk of up to kChunkT consecutive
  // reached intervals per wave (k_adj_chunk; the chunk lists replace the
  // descriptors)
  int32_t order = 0;
};

// Component schedule of one minibatch for the one-launch minibatch kernel.
// The minibatch's intervals of cluster c, sorted, split where two neighbours
// are K or more apart, form its components: the departure intervals one
// component reaches are a contiguous range that no other component reaches.
//   slot[c][bh]          minibatch slots sorted by interval (-1 past the end)
//   desc[c][mt][K+3]     reached-interval descriptors sorted by t (ChunkSched
//                        format, -1 past the end)
//   comp[c][max_comp][4] per component: first entry in slot, slot count,
//                        first entry in desc, descriptor count (count 0 pads)
struct CompSched {
  const int32_t* perm;   // [C][H] the epoch's permutations
  const int32_t* slot;
  const int32_t* desc;
  const int32_t* comp;
  int32_t j0, bh, mt, max_comp;
  const int32_t* epoch;  // device epoch counter (graph replays) or nullptr
  int64_t perm_e, slot_e, desc_e, comp_e;
};

// Reached-interval chunks of one minibatch for the chunked adjoint: each
// component's reached departure intervals cut into runs of up to kChunkT
// consecutive ones, each listed with the minibatch intervals that reach it:
//   chunk[c][max_chunks][w] = [t0, n_t, n_h, (h, slot) x n_h, ...] (n_t = 0 pads)
constexpr int32_t kChunkT = 6;
struct ChunkList {
  const int32_t* chunk;
  int32_t max_chunks, w;
  const int32_t* epoch;   // device epoch counter (graph replays) or nullptr
  int64_t chunk_e;
};

__device__ __forceinline__ ChunkList resolve_epoch(ChunkList ck) {
  if (ck.epoch) ck.chunk += *ck.epoch * ck.chunk_e;
  return ck;
}

// Resolve the epoch of a chunk schedule read from device memory (kernel side).
__device__ __forceinline__ ChunkSched resolve_epoch(ChunkSched cs) {
  if (cs.epoch) {
    const int64_t e = *cs.epoch;
    cs.perm += e * cs.perm_e;
    cs.pos += e * cs.perm_e;
    cs.touched += e * cs.touched_e;
  }
  return cs;
}

__device__ __forceinline__ CompSched resolve_epoch(CompSched ks) {
  if (ks.epoch) {
    const int64_t e = *ks.epoch;
    ks.perm += e * ks.perm_e;
    ks.slot += e * ks.slot_e;
    ks.desc += e * ks.desc_e;
    ks.comp += e * ks.comp_e;
  }
  return ks;
}

// Groups of up to `tile` days of one cluster (tile/16 MFMA column tiles).
// Plan days are grouped by cluster, so group g holds days first..first+count-1,
// and the groups of one cluster are consecutive: cbase[g] is the first group of
// g's cluster and cgroups[g] the number of groups of that cluster.
struct DayGroups {
  const int32_t* cluster;   // [n]
  const int32_t* first;     // [n] first plan day of the group
  const int32_t* count;     // [n] 1..tile
  const int32_t* cbase;     // [n]
  const int32_t* cgroups;   // [n]
  int32_t n;
  int32_t tile;             // days per group: 16, 32 or 64 (MFMA column tiles of a wave)
};

// Item order of the one-launch-per-minibatch kernel's workgroups: (cluster,
// row u, group of the cluster, tile k), k fastest (the separate launches take
// theirs from host-built work tables instead).  `per_cluster` is the row
// count, `n_tiles` the tiles per row.  Returns the group and writes its
// cluster, u and k.
__device__ __forceinline__ int decode_item(const DayGroups& dg, int item, int per_cluster,
                                           int n_tiles, int& c, int& u, int& k) {
  k = item % n_tiles;
  const int q = item / n_tiles;            // = per_cluster*g0 + u*ng + (g - g0)
  const int G = q / per_cluster;           // some group of the item's cluster
  const int g0 = dg.cbase[G], ng = dg.cgroups[G];
  c = dg.cluster[G];
  const int r = q - per_cluster * g0;
  u = r / ng;
  return g0 + (r - u * ng);
}

// One wave's work in a grouped matrix-core launch, decoded on the host: the
// cluster, the day group's first plan day and day count, the row (minibatch
// slot for the forward product, descriptor index for the adjoint), the tile
// (link tile / OD tile) and that tile's packed k-step count, first column
// (OD for the forward tiles, link for the adjoint tiles) and k-step offset.
// A wave reads its entry with one scalar load instead of decoding its item.
struct WaveWork {
  int32_t c, first, count, row, tile, nks, lo, koff;
};

// Work table of one grouped launch over a day-group list (work_tables.hip).
std::vector<WaveWork> work_table(const dode_dar* dar, const std::vector<int32_t>& gc,
                                 const std::vector<int32_t>& gf, const std::vector<int32_t>& gn,
                                 bool fwd, int32_t rows, bool tile_major, bool group_fastest);

// Zeroed elements past the end of each plan state array (X, Q, A, R).
constexpr int64_t kStatePad = 64;

// Minibatch schedule and scratch of spgd_run (see spgd_plan_create).
// Persistent epoch launch (kernel_path 3): the schedules of minibatch j in the
// device-counter form (the kernel takes the epoch as an argument instead), and
// the grid barrier's words (zeroed before each launch).
struct PersistMinibatch {
  ChunkSched cs;
  ChunkList ck;
};
struct PersistBarrier {
  unsigned count, gen, err, pad;
};

struct dode_plan {
  const dode_dar* dar = nullptr;
  int device = 0;
  int32_t D = 0, E = 0, C = 0, bh = 0, nch = 0, mt = 0;
  StepArgs sa{};
  int32_t* d_perm = nullptr;      // [E][C][H]
  int32_t* d_pos = nullptr;       // [E][C][H]
  int32_t* d_touched = nullptr;   // [E][nch][C][mt][K+3] reached-interval descriptors
  int32_t* d_kslot = nullptr;     // [E][nch][C][bh]  component schedule (CompSched)
  int32_t* d_kdesc = nullptr;     // [E][nch][C][kmt][K+3]
  int32_t* d_kcomp = nullptr;     // [E][nch][C][max_comp][4]
  int32_t kmt = 0, max_comp = 0;
  int32_t* d_kchunk = nullptr;    // [E][nch][C][max_chunks][chunk_w] (ChunkList)
  int32_t max_chunks = 0, chunk_w = 0;
  int32_t* d_kchunk_full = nullptr;   // refinement steps: [C][full_chunks][chunk_w]
  int32_t full_chunks = 0;
  bool one_launch = false;        // matrix-core minibatches as one launch each
  // every minibatch of an epoch in one cooperative launch (kernel_path 3):
  // the per-minibatch schedules and the grid barrier's words
  bool persistent = false;
  PersistMinibatch* d_mb = nullptr;
  PersistBarrier* d_bar = nullptr;
  int32_t adj_order = 0;          // ChunkSched::order of the matrix-core adjoint
  // Day slabs: the day groups split into n_slabs parts, each with its own
  // launches of every minibatch; slab 0 runs on the run's stream and slab k on
  // side stream k-1, forked and joined in every epoch, so the slabs' launches
  // overlap (days are independent, so the results do not depend on the slabs).
  // With kernel timing on, the slabs run one after another on the run's stream.
  int32_t n_slabs = 1;
  std::vector<hipStream_t> side_streams;
  std::vector<hipEvent_t> slab_events;   // [0] fork, [1 + k] join of side stream k
  int32_t* d_slabs = nullptr;      // per slab: cluster | first | count | cbase | cgroups
  std::vector<int64_t> slab_off;   // offset of slab k in d_slabs (elements)
  std::vector<int32_t> slab_n;     // groups of slab k
  std::vector<int32_t> h_gc, h_gf, h_gn;   // host copy of the day groups
  // Work tables of the grouped matrix-core launches (WaveWork, one entry per
  // wave): per slab (one entry when n_slabs == 1) the minibatch forward and
  // the adjoint in either item order, and on all groups the refinement
  // steps' forward and adjoint.
  struct WaveTables {
    WaveWork* fwd = nullptr;
    WaveWork* adj[3] = {nullptr, nullptr, nullptr};   // per adjoint order
    int64_t n_fwd = 0, n_adj[3] = {0, 0, 0};
  };
  std::vector<WaveTables> wt_mb;
  WaveTables wt_full;
  int32_t n_timed = 0;            // schedule candidates timed at load
  double tune_ms = 0.0;           // trial time of the chosen candidate
  int32_t* d_dc = nullptr;        // [D]
  void* d_R = nullptr;            // [bh][D][L] residual rows of the current minibatch
  double* d_part = nullptr;       // [D][H] loss partials
  void* d_X = nullptr;            // [H][D][L] plan copy of the observations
  void* d_Q = nullptr;            // [T][D][P] plan copy of the demand
  void* d_A = nullptr;            // [T][D][P] plan copy of the Adagrad accumulator
  double* d_loss = nullptr;       // [D] loss of the plan's days (plan order)
  int32_t* d_order = nullptr;     // [D] caller day of plan day i (days grouped by cluster)
  Layout ly{};                    // plan layout of X, Q, A, R
  int32_t* d_groups = nullptr;    // cluster | first | count | cbase | cgroups (n_groups each)
  int32_t n_groups = 0;
  int32_t day_tile = 32;          // days per group
  int32_t refine_steps = 0;       // full-batch steps per epoch on corrected values
  int32_t* d_full = nullptr;      // full-batch schedule: perm | pos [C][H], descriptors [C][T][K+3]
  bool tune_day_tile = false;     // choose day_tile by timing at the next load
  std::vector<int32_t> cluster_days;  // days of each cluster (plan days are grouped by cluster)
  bool use_mfma = false;
  bool check_finite = true;
  bool use_graph = true;
  int32_t* d_epoch = nullptr;         // epoch counter read by graph replays
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t last_stream = nullptr;
  bool timing = false;
  std::vector<hipEvent_t> event_pool;
  size_t event_next = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[3];

  DayGroups groups() const {
    return DayGroups{d_groups, d_groups + n_groups, d_groups + 2 * n_groups,
                     d_groups + 3 * n_groups, d_groups + 4 * n_groups, n_groups, day_tile};
  }
  // day groups of slab k (k < 0: all)
  DayGroups slab_groups(int32_t k) const {
    if (k < 0 || n_slabs <= 1) return groups();
    const int32_t* b = d_slabs + slab_off[k];
    const int32_t n = slab_n[k];
    return DayGroups{b, b + n, b + 2 * n, b + 3 * n, b + 4 * n, n, day_tile};
  }
  bool sorted_desc() const { return use_mfma && adj_order >= 1; }
  ChunkSched chunk(int32_t e, int32_t j) const {
    const int32_t H = dar->dims.H;
    const size_t dw = desc_width(dar->dims.K);
    if (sorted_desc())
      return ChunkSched{d_perm + (size_t)e * C * H, d_pos + (size_t)e * C * H,
                        d_kdesc + ((size_t)e * nch + j) * C * kmt * dw, j * bh, bh, kmt, nullptr, 0,
                        0, adj_order};
    return ChunkSched{d_perm + (size_t)e * C * H, d_pos + (size_t)e * C * H,
                      d_touched + ((size_t)e * nch + j) * C * mt * dw, j * bh, bh, mt, nullptr, 0, 0};
  }
  // the whole row set as one minibatch (identity order; refinement steps).
  // Its adjoint keeps the interval-major item order: with every interval in
  // the minibatch, the OD-tile-major order would walk all of an OD tile's
  // assignment tiles once per day group, far more than the L2 holds
  // (measured 14.4 -> 21.4 ms per epoch at 400 OD, 1500 links, FP8).
  ChunkSched chunk_full() const {
    const int32_t H = dar->dims.H;
    const int32_t* perm = d_full;
    const int32_t* pos = d_full + (size_t)C * H;
    return ChunkSched{perm, pos, d_full + 2 * (size_t)C * H, 0, H, dar->dims.T, nullptr, 0, 0};
  }
  // component schedule of minibatch j of epoch e (e < 0: the epoch held in
  // d_epoch, for graph replays)
  CompSched comps(int32_t e, int32_t j) const {
    const int32_t H = dar->dims.H;
    const size_t dw = desc_width(dar->dims.K);
    const int64_t ps = (int64_t)C * H, ss = (int64_t)nch * C * bh;
    const int64_t ds = (int64_t)nch * C * kmt * dw, cs = (int64_t)nch * C * max_comp * 4;
    const int64_t ee = e < 0 ? 0 : e;
    return CompSched{d_perm + ee * ps, d_kslot + ee * ss + (int64_t)j * C * bh,
                     d_kdesc + ee * ds + (int64_t)j * C * kmt * dw,
                     d_kcomp + ee * cs + (int64_t)j * C * max_comp * 4, j * bh, bh, kmt, max_comp,
                     e < 0 ? d_epoch : nullptr, ps, ss, ds, cs};
  }
  // reached-interval chunks of the full-batch refinement steps
  ChunkList chunks_full() const { return ChunkList{d_kchunk_full, full_chunks, chunk_w, nullptr, 0}; }
  // reached-interval chunks of minibatch j of epoch e (e < 0: the epoch in d_epoch)
  ChunkList chunks(int32_t e, int32_t j) const {
    const int64_t per_e = (int64_t)nch * C * max_chunks * chunk_w;
    const int64_t ee = e < 0 ? 0 : e;
    return ChunkList{d_kchunk + ee * per_e + (int64_t)j * C * max_chunks * chunk_w, max_chunks,
                     chunk_w, e < 0 ? d_epoch : nullptr, per_e};
  }
  // minibatch j of the epoch held in d_epoch (for graph replays)
  ChunkSched chunk_dev(int32_t j) const {
    const int32_t H = dar->dims.H;
    const size_t dw = desc_width(dar->dims.K);
    if (sorted_desc())
      return ChunkSched{d_perm, d_pos, d_kdesc + (size_t)j * C * kmt * dw, j * bh, bh, kmt, d_epoch,
                        (int64_t)C * H, (int64_t)(nch * C * kmt * dw), adj_order};
    return ChunkSched{d_perm, d_pos, d_touched + (size_t)j * C * mt * dw, j * bh, bh, mt, d_epoch,
                      (int64_t)C * H, (int64_t)(nch * C * mt * dw)};
  }
};

bool is_f64(const dode_dar* d);

// Host loop over [0, n) split into contiguous ranges on up to 16 threads;
// f(begin, end) must only touch what its range owns.  Used by the host-side
// conversion of the assignment values, whose iterations are independent.
template <typename F>
void host_parallel_for(int64_t n, F&& f) {
  const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
  const int64_t nt = std::min<int64_t>({hw, int64_t(16), std::max<int64_t>(1, n)});
  if (nt <= 1) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t per = (n + nt - 1) / nt;
  for (int64_t i = 0; i < nt; ++i) {
    const int64_t b = i * per, e = std::min(n, b + per);
    if (b < e) th.emplace_back([&f, b, e] { f(b, e); });
  }
  for (auto& t : th) t.join();
}

// ---- plain kernels (plain_kernels.hip) ---------------------------------
// All launchers return hipSuccess or the launch error.  `day_cluster` may be
// nullptr, then every day belongs to `cluster`.
hipError_t plain_chunk_resid(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                             const ChunkSched& cs, const Layout& ly, const void* Q, const void* X,
                             void* R, int32_t n_days, hipStream_t s);
hipError_t plain_chunk_adj_step(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                                const ChunkSched& cs, const Layout& ly, const void* R, void* Q,
                                void* A, int32_t n_days, const StepArgs& st, hipStream_t s);
// out (nullable, X layout) = rho Q (- X if X); part (nullable) = [n][H] row sums of squares
hipError_t plain_apply_rows(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                            const Layout& ly, const void* Q, const void* X, void* out, double* part,
                            int32_t n_days, hipStream_t s);
// G (Q layout) = rho^T R for full residual rows R (R layout with r_s = row stride of h)
hipError_t plain_adjoint_rows(const dode_dar* dar, const int32_t* day_cluster, int32_t cluster,
                              const Layout& ly, const void* R, void* G, int32_t n_days,
                              hipStream_t s);
// plan state copies: plan entry (day i, row r, col k) at i*sd + r*sr + col_at(k, sb)
// = src[order[i]][r][k] (gather) and back (scatter); clamp projects onto >= 0
// on the way in
hipError_t gather_rows(bool f64, const void* src, void* dst, const int32_t* order, int32_t D,
                       int32_t rows, int32_t n, int64_t sd, int64_t sr, int64_t sb, bool clamp,
                       hipStream_t s);
hipError_t scatter_rows(bool f64, const void* src, void* dst, const int32_t* order, int32_t D,
                        int32_t rows, int32_t n, int64_t sd, int64_t sr, int64_t sb, hipStream_t s);
hipError_t fill_zero(bool f64, void* x, int64_t n, hipStream_t s);
hipError_t permute_loss(const double* src, const int32_t* order, int32_t D, double* dst,
                        hipStream_t s);
hipError_t set_counter(int32_t* c, int32_t v, hipStream_t s);
hipError_t bump_counter(int32_t* c, hipStream_t s);

// ---- dynamic assignment ratios from link speeds (dar_kernels.hip) -------
constexpr int32_t kMaxDarLags = 16;
// flag = 1 if any of the n values is not positive and finite
hipError_t dar_check_speeds(bool f64, const void* speed, int64_t n, int32_t* flag, hipStream_t s);
// Rr[K][H][n_pairs] = day mean of the ratios; traj = scratch for `chunk` days.
// With cost non-null also cost[H][n_paths] = day mean of the path travel times
// (exit_time = scratch [chunk][n_paths][H+1], sums = FP64 scratch [n_paths][H]).
hipError_t dar_from_speeds(bool f64, int32_t n_paths, const int32_t* path_ptr,
                           const int32_t* path_link, int64_t n_pairs, int32_t L, const void* len,
                           const void* speed, int32_t n_days, int32_t H_speed, double dt, int32_t H,
                           int32_t K, void* traj, int32_t chunk, void* Rr, void* exit_time,
                           double* sums, void* cost, hipStream_t s);
// cost[T][n_paths] = day mean of the path travel times for departures at t*dt;
// partial = FP64 scratch [ceil(n_days/per_slice)][n_paths][T], per_slice % 4 == 0
hipError_t path_costs(bool f64, int32_t n_paths, const int32_t* path_ptr, const int32_t* path_link,
                      int32_t L, const void* len, const void* speed, int32_t n_days, int32_t H_speed,
                      double dt, int32_t T, int32_t per_slice, double* partial, void* cost,
                      hipStream_t s);

// ---- dense NNLS by Algorithm 1 (dense_kernels.hip) ----------------------
struct DenseArgs {
  int32_t m, n, E, chunk;
  const void* B;          // [m][n]
  const void* y;          // [m]
  void* q;                // [n]
  void* A;                // [n]
  const int32_t* perms;   // [E][m] (device)
  void* r;                // scratch [m]
  void* part;             // scratch [ceil(min(chunk, m) / dense_slice_rows())][n]
  double* loss;           // [E] (device) or nullptr
  StepArgs st;
};
int32_t dense_slice_rows();
// vec: B and q are 16-byte aligned and a row of B is a multiple of 16 bytes
hipError_t dense_spgd(const DenseArgs& a, bool f64, bool vec, hipStream_t s);
// B as bf16 bits, FP32 y, q, A (vec: B and q 16-byte aligned, n % 8 == 0)
hipError_t dense_spgd_bf16(const DenseArgs& a, bool vec, hipStream_t s);

// ---- MFMA tile kernels (mfma_kernels.hip) -------------------------------
// corr: multiply with the corrected FP8 values (refinement steps)
// wt: the launch's work table (n_items entries, one per wave)
hipError_t mfma_chunk_resid(const dode_dar* dar, const ChunkSched& cs, const WaveWork* wt,
                            int64_t n_items, int32_t day_tile, const Layout& ly, const float* Q,
                            const float* X, float* R, bool corr, hipStream_t s);
hipError_t mfma_chunk_adj_step(const dode_dar* dar, const ChunkSched& cs, const WaveWork* wt,
                               int64_t n_items, int32_t day_tile, const Layout& ly, const float* R,
                               float* Q, float* A, const StepArgs& st, bool corr, hipStream_t s);
// adjoint + step by reached-interval chunks (day tiles 16 and 32; corr: the
// corrected FP8 values of refinement steps)
hipError_t mfma_adj_chunks(const dode_dar* dar, const ChunkList& ck, const WaveWork* wt, int64_t n,
                           int32_t day_tile, const Layout& ly, const float* R, float* Q, float* A,
                           const StepArgs& st, bool corr, hipStream_t s);
// one whole minibatch (forward, residual, adjoint, step) in one launch
// Persistent epoch launch (kernel_path 3); the structs are defined before the plan.
hipError_t mfma_epoch_persistent(const dode_dar* dar, const PersistMinibatch* mb, int32_t nch,
                                 int32_t epoch, const WaveWork* wt_fwd, int64_t n_fwd,
                                 const WaveWork* wt_adj, int64_t n_adj, int32_t order,
                                 int32_t day_tile, const Layout& ly, const float* X, float* R,
                                 float* Q, float* A, const StepArgs& st, PersistBarrier* bar,
                                 uint32_t spin_limit, hipStream_t s);
hipError_t mfma_minibatch(const dode_dar* dar, const CompSched& ks, const DayGroups& dg,
                          const Layout& ly, const float* X, float* R, float* Q, float* A,
                          const StepArgs& st, hipStream_t s);
// host: tile layout (ranges, positions, device arrays), then each cluster's
// entries from its pattern-form codes (CSR order, storage type) (tiles.hip)
dode_status tiles_prepare(dode_dar* d, std::string& err);
dode_status tiles_fill_cluster(dode_dar* d, int32_t c, const void* codes_csr, std::string& err);
// bf16 correction codes of one cluster (CSR order) into the correction tiles
dode_status tiles_fill_correction(dode_dar* d, int32_t c, const uint16_t* corr_csr,
                                  std::string& err);

// ---- route choice and differentiation (route_kernels.hip) ---------------
// pi = FP64 scratch [n_paths] (free logits) or [T][n_paths] (costs)
hipError_t routes_rho(const DevRoutes& r, bool f64, const void* Rr, const void* z, void* W,
                      double* pi, hipStream_t s);
hipError_t routes_rho_costs(const DevRoutes& r, bool f64, const void* Rr, const void* cost,
                            double theta, void* portions, void* W, double* pi, hipStream_t s);
hipError_t routes_logits_bwd(const DevRoutes& r, bool f64, const void* Rr, const void* z,
                             const void* dW, void* dz, double* pi, double* dpi, hipStream_t s);
// R full residual rows [n][H][L], Q [n][T][P] (day-major)
hipError_t loss_bwd_dW(const dode_dar* dar, const void* R, const void* Q, int32_t n_days,
                       double scale, void* dW, hipStream_t s);
hipError_t scale_state(bool f64, void* x, int64_t n, double f, hipStream_t s);
// copy the pattern-form codes of one cluster into its MFMA tiles (after quantize_values)
hipError_t update_tiles(const dode_dar* dar, int32_t cluster, hipStream_t s);

// ---- small generic kernels (plain_kernels.hip) -------------------------
hipError_t sum_partials(const double* part, int32_t n_per, int32_t n_days, double* out,
                        hipStream_t s);
hipError_t kkt_partials(bool f64, const void* Q, const void* G, int32_t T, int32_t P,
                        int32_t n_days, double* part, hipStream_t s);
hipError_t max_partials(const double* part, int32_t n_per, int32_t n_days, double* out,
                        hipStream_t s);
hipError_t x_moment_partials(bool f64, const void* X, int32_t H, int32_t L, int32_t n_days,
                             const double* sum_x /* nullable: first moment pass */, double* part,
                             hipStream_t s);
hipError_t r2_finish(const double* loss, const double* sst, int32_t n_days, double* r2,
                     hipStream_t s);
hipError_t check_finite(bool f64, const void* X, int64_t n, int32_t* flag, hipStream_t s);
hipError_t clamp_nonneg(bool f64, void* Q, int64_t n, hipStream_t s);
hipError_t quantize_values(const dode_dar* dar, int32_t cluster, const void* W_state,
                           hipStream_t s);

// ---- number formats (host side, exact round-to-nearest-even) -----------
uint16_t host_f64_to_bf16(double v);
uint8_t host_f64_to_e4m3(double v);   // v already scaled into [-448, 448]
double host_bf16_to_f64(uint16_t b);
double host_e4m3_to_f64(uint8_t b);
