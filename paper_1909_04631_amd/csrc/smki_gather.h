// Map-update structures shared by the HIP translation units (internal).
#pragma once
#include "smki_bucket.h"

#define SMKI_TILE 4                 // sub-tile edge: 4^3 = 64 voxels = one wavefront
#define SMKI_MAX_BOX 16             // largest staged box edge (sub-tile + 2 * reach)
#define SMKI_MAX_COLS ((SMKI_MAX_BOX) * (SMKI_MAX_BOX))
#define SMKI_POLY_N 8               // coefficients of the kernel polynomial

// Block-hash and pool of the persistent map.
struct MapDev {
  uint64_t* hkeys;      // [hcap] block keys, ~0 = empty
  int32_t* hvals;       // [hcap] pool slot
  int64_t hcap;         // power of two
  uint64_t* bkeys;      // [pool_cap] key of each pool slot
  float* alpha;         // [pool_cap][K][B^3]
  int32_t K, B, log2B;
  float alpha0;
};

// One column of the voxel stencil: lateral offset (dx, dy) and half-height h:
// every voxel cell that can hold a point within l of the voxel centre.
struct StencilCol {
  int32_t dx, dy, h, pad;
};

struct GatherArgs {
  BucketGeom g;             // point grid
  int32_t eblo[3], enb[3];  // target (extended) grid
  int32_t R, D;             // stencil reach in voxels, staged box edge (SMKI_TILE + 2R)
  int32_t nsub;             // sub-tiles per block edge (B / SMKI_TILE)
  int32_t ncols;
  const StencilCol* cols;
  float l2, inv_l;
  float coef[SMKI_POLY_N];  // sigma0 * Q(u) coefficients, highest degree first
  int32_t K, free_class;
  // point sets: 0 = free samples, 1 = hits
  const float4* pts[2];
  const int32_t* dense[2];
  const int32_t* prefix[2];
  // targets
  const int32_t* tgt_elin;  // [n_targets] extended-grid linear index
  const int32_t* tgt_slot;  // [n_targets] pool slot (-1: inactive)
  const int4* plan;         // [n_targets * nsub^3]: (parts, window, partial base, 0)
  const int4* units;        // [n_units]: (target, sub-tile, part, 0)
  float* alpha;             // pool
  float* part_acc;          // [n_partials][K][64]
  int32_t* part_cnt;        // [n_partials][64]
  unsigned long long* stats;  // [0] = voxels with an in-support point, [1] = in-support pairs
  int32_t budget;           // per-lane candidate budget of one work unit
};

hipError_t launch_mark_targets(const int32_t* slot_lin, const int32_t* d_nslots, int32_t max_slots,
                               const BucketGeom& g, const int32_t eblo[3], const int32_t enb[3],
                               int32_t DB, int32_t* mark, hipStream_t st);
hipError_t launch_list_targets(const int32_t* mark, const int32_t* mpos, int64_t n_ext,
                               int32_t* tgt_elin, hipStream_t st);
hipError_t launch_plan(const GatherArgs& a, int32_t n_targets, float frac, int4* plan,
                       int32_t* active, hipStream_t st);
size_t gather_lds_bytes(const GatherArgs& a);
hipError_t launch_map_lookup(const MapDev& m, const GatherArgs& a, int32_t n_targets,
                             const int32_t* active, int32_t* tgt_slot, int32_t* is_new,
                             uint32_t* err, hipStream_t st);
hipError_t launch_assign_new(const MapDev& m, const GatherArgs& a, int32_t n_targets,
                             const int32_t* is_new, const int32_t* new_rank, int64_t n_old,
                             int32_t* tgt_slot, uint32_t* err, hipStream_t st);
hipError_t launch_fill_alpha0(const MapDev& m, int64_t slot0, int64_t nslots, hipStream_t st);
hipError_t launch_plan_counts(const int4* plan, int64_t n, int32_t* nparts, int32_t* nsplit,
                              hipStream_t st);
hipError_t launch_units(int4* plan, const int32_t* unit_off, const int32_t* split_off, int64_t n,
                        int32_t nsub3, int4* units, hipStream_t st);
hipError_t launch_gather(const GatherArgs& a, int64_t n_units, hipStream_t st);
hipError_t launch_merge(const GatherArgs& a, int64_t n_plan, hipStream_t st);

// map.hip
hipError_t launch_query(const MapDev& m, const int32_t* ijk, int64_t M, float* alpha, float* mean,
                        float* var, int32_t* label, float* p_occ, int32_t free_class,
                        hipStream_t st);
hipError_t launch_hash_clear(const MapDev& m, hipStream_t st);
hipError_t launch_hash_insert_slots(const MapDev& m, int64_t slot0, int64_t n, uint32_t* err,
                                    hipStream_t st);
hipError_t launch_gather_blocks(const MapDev& m, const uint32_t* order, int64_t n,
                                int32_t* block_ijk, float* alpha_out, hipStream_t st);
hipError_t launch_block_keys_to_ijk(const uint64_t* keys, int64_t n, int32_t* ijk, hipStream_t st);
hipError_t launch_ijk_to_block_keys(const int32_t* ijk, int64_t n, uint64_t* keys, uint32_t* err,
                                    hipStream_t st);
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
