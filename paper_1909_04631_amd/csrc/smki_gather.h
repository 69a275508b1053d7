// Map-update structures shared by the HIP translation units (internal).
#pragma once
#include "smki_bucket.h"

#define SMKI_MAX_REACH 4            // largest stencil reach in voxels
#define SMKI_MAX_OFFS 729           // (2 * SMKI_MAX_REACH + 1)^3
#define SMKI_POLY_N 7               // coefficients of the kernel polynomial
#define SMKI_CHUNK 512              // default rows of one (class, block) per splat work unit
#define SMKI_STAT_COPIES 64         // copies of the insert counters (spread the atomics)
#define SMKI_TIMING_RING 64         // inserts whose kernel times are kept
#define SMKI_PART_HEAD 64           // zero words heading the partial sums (read for absent pieces)

// Sparse kernel of Eq. (8): f(1 - s) = s^5 Q(s^2) with s = 1 - d/l.  Q below is a
// degree-6 relative least-squares fit in u = s^2 on [0, 1] to the series
// Q(u) = sum_{n>=2} (-1)^n (2n-2) (2 pi)^(2n) u^(n-2) / (3 (2n+1)!), obtained by
// expanding cos and sin of 2 pi (1 - s); fit error 2.6e-7 relative, 1.3e-6 when
// evaluated in binary32 (kernel_poly.py derives it).  Highest degree first.
static constexpr double kSmkiQ[SMKI_POLY_N] = {
    0.04696689938778598, -0.41528081234338315, 1.9962683906096352, -6.394682424213184,
    13.385465187748379,  -16.277320609426397,  8.658583627197082};

// Block hash and pools of the persistent map.  A block holds, per class, either
// nothing (every voxel at the prior alpha0) or one class block of B^3
// concentrations: only classes that some row ever reached take memory.
struct MapDev {
  uint64_t* hkeys;      // [hcap] block keys, ~0 = empty
  int32_t* hvals;       // [hcap] pool slot
  int64_t hcap;         // power of two
  uint64_t* bkeys;      // [pool_cap] key of each pool slot
  int32_t* cslot;       // [pool_cap][K] class block of (block, class), -1: all alpha0
  float* calpha;        // [cpool_cap][B^3] concentrations of the allocated class blocks
  int32_t K, B, log2B;
  float alpha0;
  int64_t* counts;      // [2] blocks and class blocks in use, kept on the device for
                        // inserts whose launches do not know them when enqueued
};

// Voxel offset (relative to a row's cell) that can lie within l of a point of
// that cell: (dx, dy, dz, unused).
struct StencilOff {
  int32_t dx, dy, dz, pad;
};

struct SplatArgs {
  BucketGeom g;               // point grid (planes = classes)
  int32_t R;                  // stencil reach in voxels (region = block grown by R)
  int32_t noff;               // voxel offsets in offs
  const int4* offs;           // [noff] StencilOff
  const float4* cls;          // [K] kernel of each class: (l^2, 1/l, sigma0 * Q's leading
                              // coefficient, l); the stencil covers the largest l
  float mcoef[SMKI_POLY_N];   // Q / Q's leading coefficient (monic), highest degree first
  int32_t K;
  int32_t chunk;              // rows of one (class, block) per work unit
  // sorted rows
  const float4* pts;          // records: |row - its voxel centre| per axis; (cell << 3 | octant) bits
  const float* wts;           // row weights (soft measurements), nullptr: every row weighs 1
  const uint32_t* perm;       // sorted row -> index into pts / wts (nullptr: pts is sorted)
  const int32_t* dense;       // [n_blocks * K] (block, class) -> slot
  const int32_t* head;        // [slots + 1] first row of each slot
  const int32_t* slot_lin;    // [slots] (class, block) linear index
  const int32_t* nunits;      // [slots] chunks of the slot
  const int32_t* ustart;      // [slots] first unit of the slot
  const int4* units;          // [n_units] (first row, end row, slot, class)
  const int32_t* uorder;      // [n_units] unit of splat workgroup b (nullable: b itself)
  int64_t part_elems;         // SMKI_PART_HEAD + n_units (B + 2R)^3
  int32_t wide;               // 1: 64-bit offsets into part even below 4 GiB
  float* part;                // SMKI_PART_HEAD zeros (written by the splat), then
                              // [n_units][(B + 2R)^3] partial sums of each unit's region, by
                              // piece: the region split into the 27 parts that fall in the
                              // unit's block and its neighbours, each contiguous (x, y, z)
  uint32_t* umask;            // [n_units] bit d: piece d is non-zero (and written)
  uint32_t piece_mask;        // pieces a unit may contribute (all 27, or the own block and
                              // its 6 face neighbours for the extended-block selection)
  int4* sinfo;                // [slots] (first unit, units, union of the units' masks,
                              // the first unit's mask)
  int32_t n_slots;
  // targets (blocks within reach of a row block), on the extended grid
  int32_t eblo[3], enb[3];
  const int32_t* ext2t;       // [n_ext] extended-grid block -> target index or -1
  const int32_t* tgt_elin;    // [n_targets] extended-grid linear index
  int32_t* tgt_active;        // [n_targets] 1 if some row reaches the block (set by k_contrib)
  const int32_t* tgt_slot;    // [n_targets] pool slot (-1: inactive)
  const int32_t* contrib;     // [n_targets][K] 1: some row of the class reaches the block
  MapDev map;
  int64_t n_cold;             // class blocks in use before this insert (newer ones are fresh)
  float alpha0;               // prior concentration written to fresh class blocks
  unsigned long long* stats;  // [SMKI_STAT_COPIES][4]: [0] updated voxels, [1] in-support pairs;
                              // workgroup b adds to copy b % SMKI_STAT_COPIES
  // Device-resident counts (captured inserts, whose launches are sized for
  // capacities); all null for an insert sized on the host.
  const int32_t* dn_slots;    // slots (n_slots is then a capacity)
  const int32_t* dn_targets;  // active-target candidates (the n_targets argument: a capacity)
  const int32_t* dn_units;    // work units (the launch: a capacity)
  const uint32_t* abort_word; // non-zero: an error or a capacity overflow; nothing is written
                              // to the map (allocation and merge return at once)
  int32_t cap_units;          // work units the unit table may hold
};

hipError_t launch_mark_targets(const int32_t* slot_lin, const int32_t* d_nslots, int32_t max_slots,
                               const BucketGeom& g, const int32_t eblo[3], const int32_t enb[3],
                               int32_t DB, int32_t* mark, hipStream_t st);
hipError_t launch_list_targets(const int32_t* mark, const int32_t* mpos, int64_t n_ext,
                               int32_t* tgt_elin, int32_t* ext2t, hipStream_t st);
// cfirst (nullable, [K], zeroed): 1 + the first slot of each class that has one
hipError_t launch_slot_units(const int32_t* head, const int32_t* d_nslots, int32_t max_slots,
                             int32_t chunk, int32_t* nunits, hipStream_t st,
                             const int32_t* slot_lin = nullptr, int64_t n_blocks = 1,
                             int32_t* cfirst = nullptr);
// units of every slot, and (order, nullable) the splat's launch order
hipError_t launch_unit_table(const int32_t* nunits, const int32_t* ustart, const int32_t* head,
                             const int32_t* slot_lin, int64_t n_blocks, int32_t chunk,
                             int32_t max_slots, const int32_t* d_nslots, const int32_t* d_nunits,
                             int4* units, int32_t* order, hipStream_t st,
                             int32_t cap_units = INT32_MAX);
hipError_t launch_splat(const SplatArgs& a, int64_t n_units, hipStream_t st);
hipError_t launch_merge(const SplatArgs& a, int32_t n_targets, hipStream_t st);
// class blocks: which (target, class) pairs receive rows, which need a new
// class block, and their allocation (splat.hip)
hipError_t launch_contrib(const SplatArgs& a, bool own_block_only, int32_t* contrib,
                          hipStream_t st);
// need [targets][K]: 1 + the rank of a class needing a class block among the
// target's (0: none); need_t [targets]: their number
hipError_t launch_need(const MapDev& m, int32_t n_targets, const int32_t* contrib,
                       const int32_t* is_new, const int32_t* tgt_slot, int32_t* need,
                       int32_t* need_t, hipStream_t st, const int32_t* dn_targets = nullptr);
hipError_t launch_slot_info(const SplatArgs& a, hipStream_t st);
// one launch: clear nclear words from clr, then (independently) the target list
// of launch_list_targets and the slot summaries of launch_slot_info
hipError_t launch_after_splat(const SplatArgs& a, int32_t* clr, int64_t nclear,
                              const int32_t* mark, const int32_t* mpos, int64_t n_ext,
                              int32_t* tgt_elin, int32_t* ext2t, hipStream_t st);
hipError_t launch_map_lookup(const MapDev& m, const SplatArgs& a, int32_t n_targets,
                             int32_t* tgt_slot, int32_t* is_new, hipStream_t st);
// new map blocks (slot, key, hash entry) and class blocks, in one launch
// cpos [targets]: the exclusive scan of need_t.  cnt (nullable, an ordinary
// insert's new block and class block counts): also sets the map's device
// counts to (n_old + cnt[0], n_cold + cnt[1]) and copies cnt to cnt_copy.
hipError_t launch_assign(const MapDev& m, const SplatArgs& a, int32_t n_targets,
                         const int32_t* is_new, const int32_t* new_rank, int64_t n_old,
                         int32_t* tgt_slot, const int32_t* need, const int32_t* cpos,
                         int64_t n_cold, uint32_t* err, hipStream_t st,
                         const int32_t* cnt = nullptr, int32_t* cnt_copy = nullptr);
// An ordinary insert without allocations: counts = (n_blocks + cnt[0],
// n_cblocks + cnt[1]), out = cnt[0, 2) (one thread)
hipError_t launch_commit_counts(const int32_t* cnt, int64_t* counts, int64_t n_blocks,
                                int64_t n_cblocks, int32_t* out, hipStream_t st);

// Captured (graph) inserts: the steps that replace the host's reads of counts.
// hdr (device): [0] 1 if the map's counts below are to be installed, [1] blocks,
// [2] class blocks; the map's counts are set from it, the insert counters cleared.
hipError_t launch_batch_start(const int64_t* hdr, int64_t* counts, unsigned long long* stats,
                              hipStream_t st);
// sc: phase-one totals (int64 free samples, then int32 hit rows); pc <- [rows,
// hit rows, free samples] clamped to cap_rows (overflow: DEVERR_CAPACITY in err).
hipError_t launch_batch_rows(const int64_t* sc, int64_t cap_rows, int64_t* pc, uint32_t* err,
                             hipStream_t st);
// DEVERR_CAPACITY if the slots (si[0]) exceed cap_slots or the work units (si[2])
// exceed cap_units
hipError_t launch_batch_units(const int32_t* si, int64_t cap_slots, int64_t cap_units,
                              uint32_t* err, hipStream_t st);
// DEVERR_CAPACITY if the new blocks / class blocks (cnt[0], cnt[1]) do not fit the
// map's pools (blocks, class blocks; the hash at most half full)
hipError_t launch_batch_alloc_check(const int32_t* cnt, const int64_t* counts, int64_t pool_cap,
                                    int64_t cpool_cap, int64_t hcap, uint32_t* err,
                                    hipStream_t st);
// without an error: counts += (cnt[0], cnt[1]); with one: OR it into the map's
// sticky error word.  out (int64 [8]): error, new blocks, new class blocks,
// rows, hit rows, free samples, slots, targets, units (read by the host later)
hipError_t launch_batch_commit(const int32_t* cnt, int64_t* counts, const uint32_t* err,
                               uint32_t* map_err, const int64_t* pc, const int32_t* si,
                               int64_t* out, hipStream_t st);

// csm.hip: counting-model inserts
hipError_t launch_csm_counts(const SplatArgs& a, const void* keys, bool wide_keys, int64_t n,
                             uint32_t* vbits, int64_t n_targets, hipStream_t st);
hipError_t launch_fill_calpha0(const MapDev& m, int64_t c0, int64_t nc, hipStream_t st);

// map.hip
hipError_t launch_query(const MapDev& m, const int32_t* ijk, int64_t M, float* alpha, float* mean,
                        float* var, int32_t* label, float* p_occ, int32_t free_class,
                        hipStream_t st);
hipError_t launch_hash_clear(const MapDev& m, hipStream_t st);
hipError_t launch_hash_insert_slots(const MapDev& m, int64_t slot0, int64_t n, uint32_t* err,
                                    hipStream_t st);
hipError_t launch_gather_blocks(const MapDev& m, const uint32_t* order, int64_t n,
                                float* alpha_out, hipStream_t st);
// import: flags of the (block, class) pairs holding any value other than alpha0,
// then the copy of those into class blocks c0 + pos
hipError_t launch_import_flags(const MapDev& m, const float* alpha, int64_t n, int32_t* flag,
                               hipStream_t st);
hipError_t launch_import_copy(const MapDev& m, const float* alpha, int64_t n, const int32_t* flag,
                              const int32_t* pos, int64_t c0, hipStream_t st);
hipError_t launch_block_keys_to_ijk(const uint64_t* keys, int64_t n, int32_t* ijk, hipStream_t st);
// block coordinates -> keys; a block whose voxels leave [-2^20, 2^20) flags DEVERR_RANGE
hipError_t launch_ijk_to_block_keys(const int32_t* ijk, int64_t n, int32_t log2B, uint64_t* keys,
                                    uint32_t* err, hipStream_t st);
// DEVERR_DUP if two adjacent keys of a sorted array are equal
hipError_t launch_adjacent_dups(const uint64_t* sorted, int64_t n, uint32_t* err, hipStream_t st);
hipError_t launch_iota_u32(uint32_t* p, int64_t n, hipStream_t st);

__host__ __device__ inline uint64_t smki_block_key(int32_t bx, int32_t by, int32_t bz) {
  return ((uint64_t)(int64_t)(bx + (1 << 20)) << 42) | ((uint64_t)(int64_t)(by + (1 << 20)) << 21) |
         (uint64_t)(int64_t)(bz + (1 << 20));
}

__host__ __device__ inline uint64_t smki_mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}
