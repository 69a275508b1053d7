// Training-set construction and spatial bucketing.
//
// Rows of the training set (Sec. III and IV of Gan et al., arXiv 1909.04631):
// every labelled hit, plus free-space points interpolated along its beam and
// labelled with the free class.  The free-sample positions and the voxel index
// of every row follow a binary32 contract (each operation rounded once, no
// fused multiply-add), so that cell keys are bit-reproducible.
//
// Bucketing: rows are keyed by (map block, voxel inside the block) over a dense
// grid of the blocks that the scan's bounding box covers, radix sorted, and
// stored as float4 records (x, y, z relative to the exact centre of the row's
// own block; label bits).  A per-block prefix table of B^3 + 1 entries maps
// any voxel range inside a block to a contiguous row range.
#include "smki_bucket.h"

#pragma clang fp contract(off)

// Correctly rounded binary32 division and square root: the double-precision
// result rounded once to binary32 is the correctly rounded binary32 result
// (53 >= 2*24 + 2, so the double rounding is innocuous).
__device__ __forceinline__ float div_rn(float a, float b) { return (float)((double)a / (double)b); }
__device__ __forceinline__ float sqrt_rn(float a) { return (float)sqrt((double)a); }

// ---------------------------------------------------------------------------
// binary32 beam arithmetic (reading of the paper's free-space sampling):
//   v = p - o ; L = sqrt((vx*vx + vy*vy) + vz*vz) ; n = ceil(L/s) - 1 ;
//   q_j = o + (((float)j * s) / L) * v
// ---------------------------------------------------------------------------
__device__ __forceinline__ float beam_len(float px, float py, float pz, float ox, float oy,
                                          float oz, float* vx, float* vy, float* vz) {
  *vx = px - ox;
  *vy = py - oy;
  *vz = pz - oz;
  const float xx = *vx * *vx, yy = *vy * *vy, zz = *vz * *vz;
  const float a = xx + yy;
  const float L2 = a + zz;
  return sqrt_rn(L2);
}

__device__ __forceinline__ int voxel_index(float x, float res, int32_t* out) {
  float q = div_rn(x, res);
  float f = floorf(q);
  if (!(f >= -(float)SMKI_COORD_LIM && f < (float)SMKI_COORD_LIM)) return 0;
  *out = (int32_t)f;
  return 1;
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
  return isfinite(x) && isfinite(y) && isfinite(z);
}

// Which scan a hit belongs to (scan_off has S+1 entries, S >= 1).
__device__ __forceinline__ int32_t scan_of(const int64_t* scan_off, int32_t S, int64_t i) {
  int32_t lo = 0, hi = S - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (scan_off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Per hit: validation, hit rows (kept: 1 for a labelled hit; for soft weights
// the number of classes with a positive weight), number of free samples of a
// kept hit, voxel bounding box.  probs (nullable) replaces label: [n][K]
// weights, each finite and >= 0; all zero drops the hit and its beam.
__global__ void k_count(const float* __restrict__ xyz, const int32_t* __restrict__ label,
                        const float* __restrict__ probs, int64_t n,
                        const int64_t* __restrict__ scan_off, const float* __restrict__ origins,
                        int32_t S, float res, float step, int32_t K, int64_t* __restrict__ nfree,
                        int32_t* __restrict__ kept, int32_t* __restrict__ bbox,
                        uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
  int32_t hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  if (i < n) {
    const float px = xyz[3 * i], py = xyz[3 * i + 1], pz = xyz[3 * i + 2];
    uint32_t e = 0;
    int64_t c = 0;
    int32_t k = 0;
    if (probs) {
      for (int32_t j = 0; j < K; ++j) {
        const float w = probs[i * K + j];
        if (!(isfinite(w) && w >= 0.0f)) e |= DEVERR_LABEL;
        k += w > 0.0f ? 1 : 0;
      }
    } else {
      const int32_t y = label[i];
      if (y < -1 || y >= K) e |= DEVERR_LABEL;
      k = y != -1 ? 1 : 0;
    }
    if (!finite3(px, py, pz)) e |= DEVERR_NONFINITE;
    if (e == 0 && k > 0) {
      int32_t v[3];
      if (!voxel_index(px, res, &v[0]) || !voxel_index(py, res, &v[1]) ||
          !voxel_index(pz, res, &v[2])) {
        e |= DEVERR_RANGE;
      } else {
        for (int a = 0; a < 3; ++a) { lo[a] = v[a]; hi[a] = v[a]; }
      }
      if (step > 0.0f) {
        const int32_t s = scan_of(scan_off, S, i);
        const float ox = origins[3 * s], oy = origins[3 * s + 1], oz = origins[3 * s + 2];
        float vx, vy, vz;
        const float L = beam_len(px, py, pz, ox, oy, oz, &vx, &vy, &vz);
        if (L > 0.0f) {
          const float cf = ceilf(div_rn(L, step));
          if (!(cf - 1.0f <= (float)SMKI_MAX_SAMPLES_PER_RAY)) e |= DEVERR_RAY;
          else c = (int64_t)cf - 1;
        }
        if (c > 0) {
          int32_t vo[3];
          if (voxel_index(ox, res, &vo[0]) && voxel_index(oy, res, &vo[1]) &&
              voxel_index(oz, res, &vo[2])) {
            for (int a = 0; a < 3; ++a) { lo[a] = min(lo[a], vo[a]); hi[a] = max(hi[a], vo[a]); }
          } else {
            e |= DEVERR_RANGE;
          }
        }
      }
    }
    nfree[i] = e ? 0 : c;
    kept[i] = e ? 0 : k;
    if (e) atomicOr(err, e);
  }
  // workgroup reduction of the bounding box, then one atomic per workgroup
  __shared__ int32_t slo[3][256], shi[3][256];
  for (int a = 0; a < 3; ++a) { slo[a][threadIdx.x] = lo[a]; shi[a][threadIdx.x] = hi[a]; }
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      for (int a = 0; a < 3; ++a) {
        slo[a][threadIdx.x] = min(slo[a][threadIdx.x], slo[a][threadIdx.x + o]);
        shi[a][threadIdx.x] = max(shi[a][threadIdx.x], shi[a][threadIdx.x + o]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {   // spread over copies: workgroups rarely contend on one address
    int32_t* bb = bbox + (blockIdx.x % SMKI_BBOX_COPIES) * 8;
    for (int a = 0; a < 3; ++a) {
      if (slo[a][0] != INT32_MAX) atomicMin(&bb[a], slo[a][0]);
      if (shi[a][0] != INT32_MIN) atomicMax(&bb[3 + a], shi[a][0]);
    }
  }
}

__device__ __forceinline__ void block_of(const BucketGeom& g, const int32_t v[3], int32_t b[3],
                                         int32_t l[3]) {
  for (int a = 0; a < 3; ++a) {
    b[a] = v[a] >> g.log2B;             // floor division (arithmetic shift)
    l[a] = v[a] - b[a] * g.B;
  }
}

// Key of a row: (label plane, block of the grid, voxel inside the block), so a
// sort groups rows by class first (planes = K for the map, 1 otherwise), then
// by block, then by voxel with z fastest.
template <typename KeyT>
__device__ __forceinline__ KeyT make_key(const BucketGeom& g, int32_t plane, const int32_t b[3],
                                         const int32_t l[3]) {
  const int64_t lin = (int64_t)plane * g.n_blocks +
                      ((int64_t)(b[0] - g.blo[0]) * g.nb[1] + (b[1] - g.blo[1])) * g.nb[2] +
                      (b[2] - g.blo[2]);
  const int64_t loc = ((int64_t)l[0] << (2 * g.log2B)) | ((int64_t)l[1] << g.log2B) | l[2];
  return (KeyT)(((uint64_t)lin << (3 * g.log2B)) | (uint64_t)loc);
}

// Record of a row: coordinates relative to the exact centre ((b + 1/2) B res) of
// its own block, computed in double and rounded once; label bits in .w.
__device__ __forceinline__ float4 make_record(const BucketGeom& g, float x, float y, float z,
                                              const int32_t b[3], int32_t label) {
  const double r = (double)g.res, hb = 0.5 * (double)g.B;
  float4 o;
  o.x = (float)((double)x - ((double)(b[0] * g.B) + hb) * r);
  o.y = (float)((double)y - ((double)(b[1] * g.B) + hb) * r);
  o.z = (float)((double)z - ((double)(b[2] * g.B) + hb) * r);
  o.w = __int_as_float(label);
  return o;
}

// Record of a map row: |u| per axis, u = x - (v + 1/2) res the row relative to
// the centre of its voxel (double, rounded once), and in .w the row's cell
// within its block and the octant of u:  (cell << 3) | (ux < 0) | (uy < 0) << 1
// | (uz < 0) << 2.  The class is the row's plane in the key, not stored here.
__device__ __forceinline__ float4 make_map_record(const BucketGeom& g, float x, float y, float z,
                                                  const int32_t v[3], const int32_t l[3]) {
  const double r = (double)g.res;
  const double ux = (double)x - ((double)v[0] + 0.5) * r;
  const double uy = (double)y - ((double)v[1] + 0.5) * r;
  const double uz = (double)z - ((double)v[2] + 0.5) * r;
  const int32_t cell = (l[0] << (2 * g.log2B)) | (l[1] << g.log2B) | l[2];
  const int32_t oct = (ux < 0.0 ? 1 : 0) | (uy < 0.0 ? 2 : 0) | (uz < 0.0 ? 4 : 0);
  float4 o;
  o.x = (float)fabs(ux);
  o.y = (float)fabs(uy);
  o.z = (float)fabs(uz);
  o.w = __int_as_float((cell << 3) | oct);
  return o;
}

__device__ __forceinline__ bool in_grid(const BucketGeom& g, const int32_t b[3]) {
  return b[0] >= g.blo[0] && b[0] < g.blo[0] + g.nb[0] && b[1] >= g.blo[1] &&
         b[1] < g.blo[1] + g.nb[1] && b[2] >= g.blo[2] && b[2] < g.blo[2] + g.nb[2];
}

// Kept hits -> (key, index) and records (unsorted), at rows kpos[i]...  With
// soft weights (probs non-null) a hit gives one row per class of positive
// weight, in class order, and wt[row] = that weight.  Also, for the free-sample
// kernel (workgroups of FREE_WG samples): wgbeam[b] = the beam that holds free
// sample b FREE_WG (each such sample lies in exactly one beam's range).
constexpr int FREE_WG = 256;
// dcnt (device, nullable): row counts [total, hits, free samples] of the
// insert, read here instead of nf (a capacity then).
template <typename KeyT>
__global__ void k_hit_keys(const float* __restrict__ xyz, const int32_t* __restrict__ label,
                           const float* __restrict__ probs, int32_t K, int64_t n,
                           const int32_t* __restrict__ kept, const int32_t* __restrict__ kpos,
                           const int64_t* __restrict__ off, int64_t nf_cap,
                           const int64_t* __restrict__ dcnt,
                           int32_t* __restrict__ wgbeam, BucketGeom g, KeyT* __restrict__ keys,
                           float4* __restrict__ rec,
                           float* __restrict__ wt, uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t nf = dcnt ? dcnt[2] : nf_cap;
  if (nf > 0) {
    // (clamped: a captured insert may hold fewer samples than its beams ask for)
    const int64_t a0 = min(off[i], nf), a1 = min(i + 1 < n ? off[i + 1] : nf, nf);
    for (int64_t b = (a0 + FREE_WG - 1) / FREE_WG; b * FREE_WG < a1; ++b) wgbeam[b] = (int32_t)i;
  }
  if (!kept[i]) return;
  const float px = xyz[3 * i], py = xyz[3 * i + 1], pz = xyz[3 * i + 2];
  int32_t v[3], b[3], l[3];
  voxel_index(px, g.res, &v[0]);
  voxel_index(py, g.res, &v[1]);
  voxel_index(pz, g.res, &v[2]);
  block_of(g, v, b, l);
  int32_t w = kpos[i];
  const int32_t rows = kept[i];
  if (!in_grid(g, b)) {
    atomicOr(err, DEVERR_RANGE);
    for (int32_t r = 0; r < rows; ++r, ++w) {
      keys[w] = (KeyT)0; rec[w] = make_float4(0, 0, 0, 0);
      if (wt) wt[w] = 0.0f;
    }
    return;
  }
  const float4 r4 = make_map_record(g, px, py, pz, v, l);
  if (!probs) {
    keys[w] = make_key<KeyT>(g, label[i], b, l);
    rec[w] = r4;
    return;
  }
  for (int32_t k = 0; k < K; ++k) {
    const float p = probs[i * K + k];
    if (!(p > 0.0f)) continue;
    keys[w] = make_key<KeyT>(g, k, b, l);
    rec[w] = r4;
    wt[w] = p;
    ++w;
  }
}

// Free sample f -> its beam (largest i with off[i] <= f), its position, key and record.
template <typename KeyT>
__global__ void k_free_keys(const float* __restrict__ xyz, int64_t n,
                            const int64_t* __restrict__ off, int64_t nf_cap,
                            const int64_t* __restrict__ dcnt,
                            const int64_t* __restrict__ scan_off,
                            const float* __restrict__ origins, int32_t S, float step,
                            int32_t free_class, BucketGeom g, int64_t out_base_h,
                            KeyT* __restrict__ keys, float4* __restrict__ rec, float* __restrict__ wrow,
                            const int32_t* __restrict__ wgbeam, uint32_t* __restrict__ err) {
  // The beams of this workgroup's samples lie between the beam of its first
  // sample and the beam of the next workgroup's first sample (wgbeam, written
  // by k_hit_keys); every sample searches only between them.
  // The beam offsets of that range go to LDS first when they fit (one round of
  // global loads instead of a chain of them per search).
  constexpr int MAXB = FREE_WG;
  __shared__ int64_t soff[MAXB];
  const int64_t nf = dcnt ? dcnt[2] : nf_cap;             // (launch sized for nf_cap)
  const int64_t out_base = dcnt ? dcnt[1] : out_base_h;   // free samples follow the hits
  const int64_t nwg = (nf + FREE_WG - 1) / FREE_WG;
  if ((int64_t)blockIdx.x >= nwg) return;   // (the whole workgroup)
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t lo = wgbeam[blockIdx.x];
  int64_t hi = (int64_t)blockIdx.x + 1 < nwg ? wgbeam[blockIdx.x + 1] : n - 1;
  if (hi - lo < MAXB) {   // (the same range for the whole workgroup)
    if (threadIdx.x <= hi - lo) soff[threadIdx.x] = off[lo + threadIdx.x];
    __syncthreads();
    int32_t a = 0, c = (int32_t)(hi - lo);
    while (a < c) {
      const int32_t mid = (a + c + 1) >> 1;
      if (soff[mid] <= f) a = mid; else c = mid - 1;
    }
    lo += a;
  } else {
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (off[mid] <= f) lo = mid; else hi = mid - 1;
    }
  }
  if (f >= nf) return;
  const int64_t i = lo;
  const int64_t j = f - off[i] + 1;
  const int32_t s = scan_of(scan_off, S, i);
  const float ox = origins[3 * s], oy = origins[3 * s + 1], oz = origins[3 * s + 2];
  float vx, vy, vz;
  const float L = beam_len(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], ox, oy, oz, &vx, &vy, &vz);
  const float t = (float)j * step;
  const float wt = div_rn(t, L);
  const float mx = wt * vx, my = wt * vy, mz = wt * vz;
  const float qx = ox + mx, qy = oy + my, qz = oz + mz;
  const int64_t w = out_base + f;
  int32_t v[3], b[3], l[3];
  if (!voxel_index(qx, g.res, &v[0]) || !voxel_index(qy, g.res, &v[1]) ||
      !voxel_index(qz, g.res, &v[2])) {
    atomicOr(err, DEVERR_RANGE);
    keys[w] = (KeyT)0; rec[w] = make_float4(0, 0, 0, 0);
    if (wrow) wrow[w] = 0.0f;
    return;
  }
  block_of(g, v, b, l);
  if (!in_grid(g, b)) {
    atomicOr(err, DEVERR_RANGE);
    keys[w] = (KeyT)0; rec[w] = make_float4(0, 0, 0, 0);
    if (wrow) wrow[w] = 0.0f;
    return;
  }
  keys[w] = make_key<KeyT>(g, free_class, b, l);
  rec[w] = make_map_record(g, qx, qy, qz, v, l);
  if (wrow) wrow[w] = 1.0f;
}

// Explicit training rows (differentiable form, tests): keys and records.
template <typename KeyT>
__global__ void k_row_keys(const float* __restrict__ xyz, const int32_t* __restrict__ label,
                           int64_t n, BucketGeom g, KeyT* __restrict__ keys,
                           uint32_t* __restrict__ idx, float4* __restrict__ rec,
                           uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float px = xyz[3 * i], py = xyz[3 * i + 1], pz = xyz[3 * i + 2];
  int32_t v[3], b[3], l[3];
  if (!finite3(px, py, pz) || !voxel_index(px, g.res, &v[0]) || !voxel_index(py, g.res, &v[1]) ||
      !voxel_index(pz, g.res, &v[2])) {
    atomicOr(err, DEVERR_RANGE);
    keys[i] = (KeyT)0; idx[i] = (uint32_t)i; rec[i] = make_float4(0, 0, 0, 0);
    return;
  }
  block_of(g, v, b, l);
  if (!in_grid(g, b)) { atomicOr(err, DEVERR_RANGE); keys[i] = (KeyT)0; idx[i] = (uint32_t)i; rec[i] = make_float4(0, 0, 0, 0); return; }
  keys[i] = make_key<KeyT>(g, 0, b, l);
  idx[i] = (uint32_t)i;
  rec[i] = make_record(g, px, py, pz, b, label ? label[i] : 0);
}

// Sorted records: out[i] = rec[idx[i]] (and the weights alike when present).
__global__ void k_permute_rec(const float4* __restrict__ rec, const float* __restrict__ wt,
                              const uint32_t* __restrict__ idx, int64_t n,
                              float4* __restrict__ out, float* __restrict__ wout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = idx[i];
  out[i] = rec[j];
  if (wt) wout[i] = wt[j];
}

// Slots: the runs of sorted rows that share (plane, block) = key >> log2B3.
// A row heads a slot when its block differs from the previous row's.  Tiles of
// HT rows (one workgroup; wavefront w takes rows [w HS, (w+1) HS) of it, 64 per
// round) first count their heads; after the scan of the counts, they give
// their heads consecutive slot numbers in row order with wave ballots.
constexpr int HT_THREADS = 256;
constexpr int HT_ROUNDS = 16;
constexpr int HS = HT_ROUNDS * SMKI_WAVE;      // rows per wavefront
constexpr int HT = HT_THREADS * HT_ROUNDS;     // rows per tile

template <typename KeyT>
__device__ __forceinline__ bool heads_slot(const KeyT* __restrict__ keys, int64_t i, int64_t n,
                                           int shift) {
  // (n is the row count; launches past it see no heads)
  if (i >= n) return false;
  return i == 0 || (uint64_t)(keys[i] >> shift) != (uint64_t)(keys[i - 1] >> shift);
}

template <typename KeyT>
__global__ void __launch_bounds__(HT_THREADS) k_head_counts(const KeyT* __restrict__ keys,
                                                            int64_t ncap,
                                                            const int64_t* __restrict__ dn,
                                                            int shift,
                                                            int32_t* __restrict__ tcount) {
  const int64_t n = eff_n(ncap, dn);
  __shared__ int32_t wc[HT_THREADS / SMKI_WAVE];
  const int lane = threadIdx.x & (SMKI_WAVE - 1), w = threadIdx.x / SMKI_WAVE;
  const int64_t base = (int64_t)blockIdx.x * HT + (int64_t)w * HS + lane;
  int32_t c = 0;
#pragma unroll 4
  for (int r = 0; r < HT_ROUNDS; ++r)
    c += (int32_t)__popcll(__ballot(heads_slot(keys, base + r * SMKI_WAVE, n, shift)));
  if (lane == 0) wc[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int q = 0; q < HT_THREADS / SMKI_WAVE; ++q) t += wc[q];
    tcount[blockIdx.x] = t;
  }
}

// After the scan of the tile counts (tstart, total in *d_nslots): the first
// row of every slot, the dense grid -> slot index and each slot's grid
// position.  The dense table is block-major: entry (block * planes + plane),
// so the classes of one block share a cache line.
template <typename KeyT>
__global__ void __launch_bounds__(HT_THREADS) k_slot_heads(const KeyT* __restrict__ keys,
                                                           int64_t ncap,
                                                           const int64_t* __restrict__ dn,
                                                           int log2B3, int64_t n_blocks,
                                                           int32_t planes,
                                                           const int32_t* __restrict__ tstart,
                                                           int32_t* __restrict__ dense,
                                                           int32_t* __restrict__ slot_lin,
                                                           int32_t* __restrict__ head,
                                                           const int32_t* __restrict__ d_nslots,
                                                           int32_t cap_slots) {
  // (slots past cap_slots are not stored: a captured insert whose rows make
  // more slots than it was sized for is failed by its capacity check)
  const int64_t n = eff_n(ncap, dn);
  __shared__ int32_t wc[HT_THREADS / SMKI_WAVE];
  const int lane = threadIdx.x & (SMKI_WAVE - 1), w = threadIdx.x / SMKI_WAVE;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (SMKI_WAVE - lane));
  const int64_t base = (int64_t)blockIdx.x * HT + (int64_t)w * HS + lane;
  if (blockIdx.x == 0 && threadIdx.x == 0 && *d_nslots <= cap_slots) head[*d_nslots] = (int32_t)n;
  uint64_t hb[HT_ROUNDS];
  int32_t c = 0;
#pragma unroll
  for (int r = 0; r < HT_ROUNDS; ++r) {
    hb[r] = __ballot(heads_slot(keys, base + r * SMKI_WAVE, n, log2B3));
    c += (int32_t)__popcll(hb[r]);
  }
  if (lane == 0) wc[w] = c;
  __syncthreads();
  int32_t slot = tstart[blockIdx.x];
  for (int q = 0; q < w; ++q) slot += wc[q];
#pragma unroll
  for (int r = 0; r < HT_ROUNDS; ++r) {
    if ((hb[r] >> lane) & 1ull) {
      const int64_t i = base + r * SMKI_WAVE;
      const int64_t blk = (int64_t)((uint64_t)keys[i] >> log2B3);   // plane * n_blocks + block
      const int32_t sl = slot + (int32_t)__popcll(hb[r] & lt_mask);
      if (sl < cap_slots) {
        dense[(blk % n_blocks) * planes + blk / n_blocks] = sl;
        slot_lin[sl] = (int32_t)blk;
        head[sl] = (int32_t)i;
      }
    }
    slot += (int32_t)__popcll(hb[r]);
  }
}

// Per slot (grid-stride over slots): histogram of the rows' voxel cells in LDS,
// then the exclusive scan -> prefix[slot][c] = first row of cell c, [B3] = end.
template <typename KeyT, int LOG2B3>
__global__ void __launch_bounds__(256) k_slot_prefix(const KeyT* __restrict__ keys, int64_t n,
                                                     const int32_t* __restrict__ head,
                                                     const int32_t* __restrict__ d_nslots,
                                                     int32_t* __restrict__ prefix) {
  constexpr int B3 = 1 << LOG2B3;
  constexpr int PER = (B3 + 255) / 256;
  __shared__ int32_t cnt[B3];
  __shared__ int32_t wsum[256 / SMKI_WAVE];
  const int32_t ns = *d_nslots;
  const int tid = threadIdx.x;
  for (int32_t s = blockIdx.x; s < ns; s += gridDim.x) {
    const int32_t r0 = head[s];
    const int32_t r1 = (s + 1 < ns) ? head[s + 1] : (int32_t)n;
    for (int c = tid; c < B3; c += 256) cnt[c] = 0;
    __syncthreads();
    for (int32_t r = r0 + tid; r < r1; r += 256)
      atomicAdd(&cnt[(uint32_t)((uint64_t)keys[r] & (uint64_t)(B3 - 1))], 1);
    __syncthreads();
    // exclusive scan of cnt: thread tid owns cells [tid * PER, tid * PER + PER)
    int32_t loc[PER];
    int32_t tot = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int c = tid * PER + j;
      loc[j] = c < B3 ? cnt[c] : 0;
      tot += loc[j];
    }
    int32_t inc = tot;   // inclusive scan over the wavefront
#pragma unroll
    for (int o = 1; o < SMKI_WAVE; o <<= 1) {
      const int32_t v = __shfl_up(inc, o, SMKI_WAVE);
      if ((tid & (SMKI_WAVE - 1)) >= o) inc += v;
    }
    if ((tid & (SMKI_WAVE - 1)) == SMKI_WAVE - 1) wsum[tid / SMKI_WAVE] = inc;
    __syncthreads();
    int32_t base = r0;
    for (int w = 0; w < tid / SMKI_WAVE; ++w) base += wsum[w];
    int32_t run = base + inc - tot;
    int32_t* P = prefix + (int64_t)s * (B3 + 1);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int c = tid * PER + j;
      if (c < B3) P[c] = run;
      run += loc[j];
    }
    if (tid == 0) P[B3] = r1;
    __syncthreads();
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int t) { return (unsigned)ceil_div_i64(n > 0 ? n : 1, t); }

hipError_t launch_count(const float* xyz, const int32_t* label, const float* probs, int64_t n,
                        const int64_t* scan_off, const float* origins, int32_t S, float res,
                        float step, int32_t K, int64_t* nfree, int32_t* kept, int32_t* bbox,
                        uint32_t* err, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count, dim3(nblk(n, 256)), dim3(256), 0, st, xyz, label, probs, n,
                     scan_off, origins, S, res, step, K, nfree, kept, bbox, err);
  return hipGetLastError();
}

// Three ranges in one launch: z0[0, n0) = 0, z1[0, n1) = 0, f[0, nf) = fv.
__global__ void k_clear3(int32_t* __restrict__ z0, int64_t n0, int32_t* __restrict__ z1, int64_t n1,
                         int32_t* __restrict__ f, int64_t nf, int32_t fv) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0 + n1 + nf; i += stride) {
    if (i < n0)
      z0[i] = 0;
    else if (i < n0 + n1)
      z1[i - n0] = 0;
    else
      f[i - n0 - n1] = fv;
  }
}

hipError_t launch_clear3(int32_t* z0, int64_t n0, int32_t* z1, int64_t n1, int32_t* f, int64_t nf,
                         int32_t fv, hipStream_t st) {
  const int64_t n = n0 + n1 + nf;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear3, dim3((unsigned)std::min<int64_t>(nblk(n, 256), 4096)), dim3(256), 0,
                     st, z0, n0, z1, n1, f, nf, fv);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// Keys, sort, records and block tables of one point set.
template <typename KeyT>
// idx_iota: idx was not written (row i's value is i): the first radix pass
// takes the indices itself.
// dn (device, nullable): the row count; ps.n is then the capacity.
static hipError_t finish_set(PointSet& ps, KeyT* keys, uint32_t* idx, KeyT* akeys, uint32_t* aidx,
                             float4* rec_unsorted, const BucketGeom& g, int key_bits,
                             BucketScratch& scr, hipStream_t st, bool idx_iota = false,
                             const int64_t* dn = nullptr, int32_t cap_slots = INT32_MAX) {
  const int64_t n = ps.n;
  if (n <= 0) return hipSuccess;
  hipError_t e;
  if (idx_iota && n == 1 && !dn) {   // no radix pass: the single index by hand
    e = hipMemsetAsync(idx, 0, sizeof(uint32_t), st);
    if (e != hipSuccess) return e;
  }
  // the last radix pass gathers the records (and weights) into sorted order,
  // if the set keeps sorted records; else they are read through the permutation
  const SortPayload pl{rec_unsorted, ps.pts, scr.wt, ps.wts};
  const SortPayload* plp = (n > 1 && ps.pts && !dn) ? &pl : nullptr;
  if (sizeof(KeyT) == 4)
    e = radix_sort_u32((uint32_t*)keys, idx, (uint32_t*)akeys, aidx, n, key_bits, scr.sort_tmp, st,
                       plp, idx_iota, dn);
  else
    e = radix_sort_u64((uint64_t*)keys, idx, (uint64_t*)akeys, aidx, n, key_bits, scr.sort_tmp, st,
                       plp, idx_iota, dn);
  if (e != hipSuccess) return e;
  if (!plp && ps.pts)
    hipLaunchKernelGGL(k_permute_rec, dim3(nblk(n, 256)), dim3(256), 0, st, rec_unsorted,
                       (const float*)scr.wt, idx, n, ps.pts, ps.wts);
  ps.perm = idx;
  const int log2B3 = 3 * g.log2B;
  // slot heads: per-tile counts (in scr.flag), their scan (scr.slot_excl), numbering
  const int64_t ntiles = ceil_div_i64(n, HT);
  hipLaunchKernelGGL(k_head_counts<KeyT>, dim3((unsigned)ntiles), dim3(HT_THREADS), 0, st, keys, n,
                     dn, log2B3, scr.flag);
  e = scan_excl_i32(scr.flag, scr.slot_excl, ntiles, ps.d_nslots, scr.scan_tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_slot_heads<KeyT>, dim3((unsigned)ntiles), dim3(HT_THREADS), 0, st, keys, n,
                     dn, log2B3, g.n_blocks, g.planes, scr.slot_excl, ps.dense, ps.slot_lin,
                     ps.head, ps.d_nslots, cap_slots);
  if (!ps.prefix) return hipGetLastError();
  if (dn) return hipErrorInvalidValue;   // (per-cell tables are built for host counts only)
  const unsigned grid = (unsigned)std::min<int64_t>(n, 8192);
  switch (log2B3) {
    case 6:
      hipLaunchKernelGGL((k_slot_prefix<KeyT, 6>), dim3(grid), dim3(256), 0, st, keys, n,
                         ps.head, ps.d_nslots, ps.prefix);
      break;
    case 9:
      hipLaunchKernelGGL((k_slot_prefix<KeyT, 9>), dim3(grid), dim3(256), 0, st, keys, n,
                         ps.head, ps.d_nslots, ps.prefix);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename KeyT>
static hipError_t bucket_scan_t(const float* xyz, const int32_t* label, const float* probs,
                                int32_t K, int64_t n, const int32_t* kept, const int32_t* kpos,
                                int64_t nk, const int64_t* off, int64_t nf, int32_t* wgbeam,
                                const int64_t* scan_off, const float* origins, int32_t S,
                                float step, int32_t free_class, const BucketGeom& g, PointSet& ps,
                                BucketScratch& scr, uint32_t* err, hipStream_t st,
                                const int64_t* dcnt, int32_t cap_slots) {
  if (nk > 0 || dcnt)
    hipLaunchKernelGGL(k_hit_keys<KeyT>, dim3(nblk(n, 256)), dim3(256), 0, st, xyz, label, probs,
                       K, n, kept, kpos, off, nf, dcnt, wgbeam, g, (KeyT*)scr.keys, scr.rec,
                       scr.wt, err);
  if (nf > 0)
    hipLaunchKernelGGL(k_free_keys<KeyT>, dim3(nblk(nf, FREE_WG)), dim3(FREE_WG), 0, st, xyz, n,
                       off, nf, dcnt, scan_off, origins, S, step, free_class, g, nk,
                       (KeyT*)scr.keys, scr.rec, scr.wt, (const int32_t*)wgbeam, err);
  return finish_set<KeyT>(ps, (KeyT*)scr.keys, scr.idx, (KeyT*)scr.akeys, scr.aidx, scr.rec, g,
                          g.key_bits, scr, st, true, dcnt, cap_slots);
}

// All training rows of an insert in one sorted set: kept hits at [0, nk), free
// samples after them; keys carry the class plane, so each (class, block) is a
// contiguous range.  wgbeam: scratch of free_sample_workgroups(nf) entries.
hipError_t bucket_scan(const float* xyz, const int32_t* label, const float* probs, int32_t K,
                       int64_t n, const int32_t* kept, const int32_t* kpos, int64_t nk,
                       const int64_t* off, int64_t nf, int32_t* wgbeam, const int64_t* scan_off,
                       const float* origins, int32_t S, float step, int32_t free_class,
                       const BucketGeom& g, PointSet& ps, BucketScratch& scr, uint32_t* err,
                       hipStream_t st, const int64_t* dcnt, int32_t cap_slots) {
  if (ps.n <= 0) return hipSuccess;
  if (g.key_bits <= 32)
    return bucket_scan_t<uint32_t>(xyz, label, probs, K, n, kept, kpos, nk, off, nf, wgbeam,
                                   scan_off, origins, S, step, free_class, g, ps, scr, err, st,
                                   dcnt, cap_slots);
  return bucket_scan_t<uint64_t>(xyz, label, probs, K, n, kept, kpos, nk, off, nf, wgbeam,
                                 scan_off, origins, S, step, free_class, g, ps, scr, err, st,
                                 dcnt, cap_slots);
}

int64_t free_sample_workgroups(int64_t nf) { return nf > 0 ? ceil_div_i64(nf, FREE_WG) : 1; }

hipError_t bucket_rows(const float* xyz, const int32_t* label, int64_t n, const BucketGeom& g,
                       PointSet& ps, BucketScratch& scr, uint32_t* err, hipStream_t st) {
  hipError_t e = launch_fill_i32(ps.dense, g.n_blocks * g.planes, -1, st);
  if (e != hipSuccess || n <= 0) return e;
  if (g.key_bits <= 32) {
    hipLaunchKernelGGL(k_row_keys<uint32_t>, dim3(nblk(n, 256)), dim3(256), 0, st, xyz, label, n,
                       g, (uint32_t*)scr.keys, scr.idx, scr.rec, err);
    return finish_set<uint32_t>(ps, (uint32_t*)scr.keys, scr.idx, (uint32_t*)scr.akeys, scr.aidx,
                                scr.rec, g, g.key_bits, scr, st);
  }
  hipLaunchKernelGGL(k_row_keys<uint64_t>, dim3(nblk(n, 256)), dim3(256), 0, st, xyz, label, n, g,
                     (uint64_t*)scr.keys, scr.idx, scr.rec, err);
  return finish_set<uint64_t>(ps, (uint64_t*)scr.keys, scr.idx, (uint64_t*)scr.akeys, scr.aidx,
                              scr.rec, g, g.key_bits, scr, st);
}

// ---------------------------------------------------------------------------
// cell table of a sorted row set (the bucketing entry point)
// ---------------------------------------------------------------------------
template <typename KeyT>
__global__ void k_cell_flags(const KeyT* __restrict__ keys, int64_t n, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

template <typename KeyT>
__global__ void k_cell_starts(const KeyT* __restrict__ keys, int64_t n, BucketGeom g,
                              const int32_t* __restrict__ flag, const int32_t* __restrict__ cpos,
                              uint64_t* __restrict__ cell_keys, int32_t* __restrict__ cell_start) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  const int l3 = 3 * g.log2B;
  const uint64_t key = (uint64_t)keys[i];
  int64_t lin = (int64_t)(key >> l3);
  const int32_t loc = (int32_t)(key & ((1ull << l3) - 1));
  const int32_t pz = (int32_t)(lin % g.nb[2]);
  lin /= g.nb[2];
  const int32_t py = (int32_t)(lin % g.nb[1]);
  const int32_t px = (int32_t)(lin / g.nb[1]);
  const int32_t B = g.B;
  const int32_t vx = (px + g.blo[0]) * B + (loc >> (2 * g.log2B));
  const int32_t vy = (py + g.blo[1]) * B + ((loc >> g.log2B) & (B - 1));
  const int32_t vz = (pz + g.blo[2]) * B + (loc & (B - 1));
  const int32_t c = cpos[i];
  cell_start[c] = (int32_t)i;
  cell_keys[c] = ((uint64_t)(int64_t)(vx + SMKI_COORD_LIM) << 42) |
                 ((uint64_t)(int64_t)(vy + SMKI_COORD_LIM) << 21) |
                 (uint64_t)(int64_t)(vz + SMKI_COORD_LIM);
}

__global__ void k_cell_counts(const int32_t* __restrict__ cell_start, int64_t ncells, int64_t n,
                              int32_t* __restrict__ cell_count) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const int64_t e = (c + 1 < ncells) ? cell_start[c + 1] : n;
  cell_count[c] = (int32_t)(e - cell_start[c]);
}

__global__ void k_copy_order(const uint32_t* __restrict__ idx, int64_t n, int32_t* __restrict__ o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = (int32_t)idx[i];
}

// Sort rows by key (keys/idx filled by k_row_keys into scr), then count cells.
hipError_t bucket_cells_sort(const float* xyz, int64_t n, const BucketGeom& g, BucketScratch& scr,
                             uint32_t* err, int32_t* d_ncells, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipError_t e;
  if (g.key_bits <= 32) {
    hipLaunchKernelGGL(k_row_keys<uint32_t>, dim3(nblk(n, 256)), dim3(256), 0, st, xyz,
                       (const int32_t*)nullptr, n, g, (uint32_t*)scr.keys, scr.idx, scr.rec, err);
    e = radix_sort_u32((uint32_t*)scr.keys, scr.idx, (uint32_t*)scr.akeys, scr.aidx, n, g.key_bits,
                       scr.sort_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_flags<uint32_t>, dim3(nblk(n, 256)), dim3(256), 0, st,
                       (const uint32_t*)scr.keys, n, scr.flag);
  } else {
    hipLaunchKernelGGL(k_row_keys<uint64_t>, dim3(nblk(n, 256)), dim3(256), 0, st, xyz,
                       (const int32_t*)nullptr, n, g, (uint64_t*)scr.keys, scr.idx, scr.rec, err);
    e = radix_sort_u64((uint64_t*)scr.keys, scr.idx, (uint64_t*)scr.akeys, scr.aidx, n, g.key_bits,
                       scr.sort_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_flags<uint64_t>, dim3(nblk(n, 256)), dim3(256), 0, st,
                       (const uint64_t*)scr.keys, n, scr.flag);
  }
  return scan_excl_i32(scr.flag, scr.slot_excl, n, d_ncells, scr.scan_tmp, st);
}

hipError_t bucket_cells_table(int64_t n, int64_t ncells, const BucketGeom& g, BucketScratch& scr,
                              uint64_t* cell_keys, int32_t* cell_start, int32_t* cell_count,
                              int32_t* order, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (g.key_bits <= 32)
    hipLaunchKernelGGL(k_cell_starts<uint32_t>, dim3(nblk(n, 256)), dim3(256), 0, st,
                       (const uint32_t*)scr.keys, n, g, scr.flag, scr.slot_excl, cell_keys,
                       cell_start);
  else
    hipLaunchKernelGGL(k_cell_starts<uint64_t>, dim3(nblk(n, 256)), dim3(256), 0, st,
                       (const uint64_t*)scr.keys, n, g, scr.flag, scr.slot_excl, cell_keys,
                       cell_start);
  hipLaunchKernelGGL(k_cell_counts, dim3(nblk(ncells, 256)), dim3(256), 0, st, cell_start, ncells,
                     n, cell_count);
  if (order)
    hipLaunchKernelGGL(k_copy_order, dim3(nblk(n, 256)), dim3(256), 0, st, scr.idx, n, order);
  return hipGetLastError();
}

__global__ void k_free_xyz(const float* __restrict__ xyz, int64_t n, const int64_t* __restrict__ off,
                           int64_t nf, const float* __restrict__ origin, float step,
                           float* __restrict__ out, int64_t* __restrict__ parent) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= f) lo = mid; else hi = mid - 1;
  }
  const int64_t i = lo;
  const int64_t j = f - off[i] + 1;
  float vx, vy, vz;
  const float L = beam_len(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], origin[0], origin[1],
                           origin[2], &vx, &vy, &vz);
  const float t = (float)j * step;
  const float w = div_rn(t, L);
  const float mx = w * vx, my = w * vy, mz = w * vz;
  out[3 * f] = origin[0] + mx;
  out[3 * f + 1] = origin[1] + my;
  out[3 * f + 2] = origin[2] + mz;
  if (parent) parent[f] = i;
}

hipError_t launch_free_xyz(const float* xyz, int64_t n, const int64_t* off, int64_t nf,
                           const float* origin_dev, float step, float* out, int64_t* parent,
                           hipStream_t st) {
  if (nf <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_free_xyz, dim3(nblk(nf, 256)), dim3(256), 0, st, xyz, n, off, nf,
                     origin_dev, step, out, parent);
  return hipGetLastError();
}
