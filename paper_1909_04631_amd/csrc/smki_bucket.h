// Bucketing structures shared by the HIP translation units (internal).
#pragma once
#include "smki_internal.h"

#define SMKI_COORD_LIM (1 << 20)
#define SMKI_MAX_SAMPLES_PER_RAY (1 << 20)
#define SMKI_BBOX_COPIES 32   // bounding-box accumulators (workgroup b updates copy b % 32)

// Dense grid of map blocks covering a bounding box of voxel indices.
struct BucketGeom {
  float res;        // voxel edge
  int32_t B;        // voxels per block edge (power of two)
  int32_t log2B;
  int32_t blo[3];   // lowest block coordinate of the grid
  int32_t nb[3];    // blocks per axis
  int64_t n_blocks; // nb[0] * nb[1] * nb[2]
  int32_t planes;   // label planes of the keys (K for a map insert, 1 otherwise)
  int32_t key_bits; // significant bits of a row key
};

// One sorted point set (hits, free samples, or explicit rows).
struct PointSet {
  int64_t n;          // rows
  float4* pts;        // sorted records: xyz relative to the row's block corner, label bits;
                      // nullptr: not gathered (read them through perm instead)
  float* wts;         // sorted row weights (soft measurements); nullptr: every row weighs 1
                      // (or, with pts nullptr, not gathered)
  const uint32_t* perm;   // after bucketing: sorted row -> row of the unsorted records
  int32_t* dense;     // [n_blocks * planes] (grid block, plane) -> slot, -1 if no row
  int32_t* slot_lin;  // [slots] (plane, grid block) linear index of each slot
  int32_t* prefix;    // [slots][B^3 + 1] first row of each voxel of the block (absolute);
                      // nullptr: not built (only the slot ranges in head)
  int32_t* head;      // [slots + 1] first row of each slot; head[slots] = rows
  int32_t* d_nslots;  // device scalar: number of slots
};

// Scratch used while building a point set (capacity = rows of the set).
struct BucketScratch {
  void* keys;         // u32 or u64 keys
  void* akeys;
  uint32_t* idx;
  uint32_t* aidx;
  float4* rec;        // unsorted records
  float* wt;          // unsorted row weights, or nullptr (then PointSet::wts is not written)
  int32_t* flag;
  int32_t* slot_excl;
  void* sort_tmp;
  void* scan_tmp;
};

// bbox: [SMKI_BBOX_COPIES][8] (min x, y, z, max x, y, z, -, -), every copy
// initialised to (INT32_MAX x3, INT32_MIN x3); the caller reduces the copies.
hipError_t launch_count(const float* xyz, const int32_t* label, const float* probs, int64_t n,
                        const int64_t* scan_off, const float* origins, int32_t S, float res,
                        float step, int32_t K, int64_t* nfree, int32_t* kept, int32_t* bbox,
                        uint32_t* err, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
// z0[0, n0) = 0, z1[0, n1) = 0, f[0, nf) = fv, in one launch
hipError_t launch_clear3(int32_t* z0, int64_t n0, int32_t* z1, int64_t n1, int32_t* f, int64_t nf,
                         int32_t fv, hipStream_t st);
// The rows of one insert, keyed, sorted and grouped into slots; ps.dense must
// hold -1 on entry (the caller clears it with its other buffers).
// dcnt (device, nullable): [rows, hit rows, free samples] of the insert, read
// by the kernels; nk, nf and ps.n are then capacities (launch sizes) and the
// free samples start at row dcnt[1].  Slots past cap_slots are not stored.
hipError_t bucket_scan(const float* xyz, const int32_t* label, const float* probs, int32_t K,
                       int64_t n, const int32_t* kept, const int32_t* kpos, int64_t nk,
                       const int64_t* off, int64_t nf, int32_t* wgbeam, const int64_t* scan_off,
                       const float* origins, int32_t S, float step, int32_t free_class,
                       const BucketGeom& g, PointSet& ps, BucketScratch& scr, uint32_t* err,
                       hipStream_t st, const int64_t* dcnt = nullptr,
                       int32_t cap_slots = INT32_MAX);
// entries of bucket_scan's wgbeam scratch for nf free samples
int64_t free_sample_workgroups(int64_t nf);
hipError_t bucket_rows(const float* xyz, const int32_t* label, int64_t n, const BucketGeom& g,
                       PointSet& ps, BucketScratch& scr, uint32_t* err, hipStream_t st);
hipError_t bucket_cells_sort(const float* xyz, int64_t n, const BucketGeom& g, BucketScratch& scr,
                             uint32_t* err, int32_t* d_ncells, hipStream_t st);
hipError_t bucket_cells_table(int64_t n, int64_t ncells, const BucketGeom& g, BucketScratch& scr,
                              uint64_t* cell_keys, int32_t* cell_start, int32_t* cell_count,
                              int32_t* order, hipStream_t st);
hipError_t launch_free_xyz(const float* xyz, int64_t n, const int64_t* off, int64_t nf,
                           const float* origin_dev, float step, float* out, int64_t* parent,
                           hipStream_t st);
