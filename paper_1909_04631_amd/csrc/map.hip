// Persistent map: block hash, readout (Eq. 3-4), export / import.
#include "smki_gather.h"

namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)ceil_div_i64(n > 0 ? n : 1, t); }

__device__ __forceinline__ int32_t hash_find(const MapDev& m, uint64_t key) {
  uint64_t h = smki_mix64(key) & (uint64_t)(m.hcap - 1);
  for (int64_t probe = 0; probe < m.hcap; ++probe) {
    const uint64_t k = m.hkeys[h];
    if (k == key) return m.hvals[h];
    if (k == ~0ull) return -1;
    h = (h + 1) & (uint64_t)(m.hcap - 1);
  }
  return -1;
}

__global__ void k_hash_clear(uint64_t* keys, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = ~0ull;
}

// Readout of Eq. (3)-(4): mean alpha/S, variance mean(1-mean)/(S+1), label =
// argmax (lowest index on ties), occupancy = 1 - mean of the free class.
// SEG consecutive lanes serve one query, lane kl holding classes kl, kl + SEG,
// ... (at most 8; SEG >= K / 8): every lane finds the query's block and loads
// its classes' alpha (all loads in flight together), and the segment reduces
// the sum, the free class's alpha and the argmax with shuffles.  Few lanes per
// query keep the number of wavefronts, each waiting on the same chain of
// dependent loads, small.
template <int SEG>
__global__ void __launch_bounds__(256) k_query(MapDev m, const int32_t* __restrict__ ijk,
                                               int64_t M, float* __restrict__ alpha,
                                               float* __restrict__ mean, float* __restrict__ var,
                                               int32_t* __restrict__ label,
                                               float* __restrict__ p_occ, int32_t free_class) {
  constexpr int MAXC = 8;   // classes per lane
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / SEG;
  const int kl = (int)(t % SEG);
  const bool live = i < M;   // whole segments are live or not; shuffles stay inside a segment
  const int32_t K = m.K, B = m.B, B3 = B * B * B;
  int32_t slot = -1, v = 0;
  if (live) {
    const int32_t vx = ijk[3 * i], vy = ijk[3 * i + 1], vz = ijk[3 * i + 2];
    const int32_t bx = vx >> m.log2B, by = vy >> m.log2B, bz = vz >> m.log2B;
    if (vx >= -(1 << 20) && vx < (1 << 20) && vy >= -(1 << 20) && vy < (1 << 20) &&
        vz >= -(1 << 20) && vz < (1 << 20))
      slot = hash_find(m, smki_block_key(bx, by, bz));
    v = ((vx - bx * B) * B + (vy - by * B)) * B + (vz - bz * B);
  }
  // this lane's classes kl, kl + SEG, ...; classes without a class block hold alpha0
  // (all class-slot loads, then all alpha loads: each set in flight together)
  int32_t cb[MAXC];
#pragma unroll
  for (int j = 0; j < MAXC; ++j) {
    const int k = kl + j * SEG;
    cb[j] = (live && k < K && slot >= 0) ? m.cslot[(int64_t)slot * K + k] : -1;
  }
  float a[MAXC];
#pragma unroll
  for (int j = 0; j < MAXC; ++j) a[j] = cb[j] >= 0 ? m.calpha[(int64_t)cb[j] * B3 + v] : m.alpha0;
  double S = 0.0, af = 0.0;
  float bestv = -1.0f;
  int32_t best = 0;
#pragma unroll
  for (int j = 0; j < MAXC; ++j) {
    const int k = kl + j * SEG;
    if (live && k < K) {
      S += (double)a[j];
      if (k == free_class) af = (double)a[j];
      if (a[j] > bestv) {
        bestv = a[j];
        best = k;
      }
    }
  }
  // moments in double: 1 - mean cancels when one class dominates
#pragma unroll
  for (int o = 1; o < SEG; o <<= 1) {
    S += __shfl_xor(S, o, SEG);
    af += __shfl_xor(af, o, SEG);
    const float ov = __shfl_xor(bestv, o, SEG);
    const int32_t ok = __shfl_xor(best, o, SEG);
    if (ov > bestv || (ov == bestv && ok < best)) {
      bestv = ov;
      best = ok;
    }
  }
  if (!live) return;
  const double inv_s = 1.0 / S, inv_s1 = 1.0 / (S + 1.0);
#pragma unroll
  for (int j = 0; j < MAXC; ++j) {
    const int k = kl + j * SEG;
    if (k >= K) continue;
    if (alpha) alpha[i * K + k] = a[j];
    const double e = (double)a[j] * inv_s;
    if (mean) mean[i * K + k] = (float)e;
    if (var) var[i * K + k] = (float)(e * ((S - (double)a[j]) * inv_s) * inv_s1);
  }
  if (kl == 0) {
    if (label) label[i] = best;
    if (p_occ) p_occ[i] = (float)((S - af) * inv_s);
  }
}

__global__ void k_hash_insert_slots(MapDev m, int64_t slot0, int64_t n, uint32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t slot = (int32_t)(slot0 + i);
  const uint64_t key = m.bkeys[slot];
  uint64_t h = smki_mix64(key) & (uint64_t)(m.hcap - 1);
  for (int64_t probe = 0; probe < m.hcap; ++probe) {
    const unsigned long long old =
        atomicCAS((unsigned long long*)&m.hkeys[h], ~0ull, (unsigned long long)key);
    if (old == ~0ull || old == key) {
      m.hvals[h] = slot;
      return;
    }
    h = (h + 1) & (uint64_t)(m.hcap - 1);
  }
  atomicOr(err, DEVERR_HASH);
}

// out block b <- pool slot order[b], dense [K][B^3] (alpha0 where a class has no class block)
__global__ void k_gather_blocks(MapDev m, const uint32_t* __restrict__ order, int64_t n,
                                float* __restrict__ out) {
  const int64_t B3 = (int64_t)m.B * m.B * m.B;
  const int64_t per = (int64_t)m.K * B3;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * per) return;
  const int64_t b = i / per, r = i % per, k = r / B3, v = r % B3;
  const int32_t cb = m.cslot[(int64_t)order[b] * m.K + k];
  out[i] = cb >= 0 ? m.calpha[cb * B3 + v] : m.alpha0;
}

// import: flag[b][k] = 1 if any voxel of class k in input block b differs from alpha0
__global__ void k_import_flags(MapDev m, const float* __restrict__ alpha, int64_t n,
                               int32_t* __restrict__ flag) {
  const int64_t B3 = (int64_t)m.B * m.B * m.B;
  const int64_t bk = blockIdx.x;   // (block, class)
  if (bk >= n * m.K) return;
  int any = 0;
  for (int64_t v = threadIdx.x; v < B3; v += blockDim.x) any |= alpha[bk * B3 + v] != m.alpha0;
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) flag[bk] = any ? 1 : 0;
}

// import: (block b, class k) flagged -> class block c0 + pos[b][k]; others alpha0 (no block)
__global__ void k_import_copy(MapDev m, const float* __restrict__ alpha, int64_t n,
                              const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                              int64_t c0) {
  const int64_t B3 = (int64_t)m.B * m.B * m.B;
  const int64_t bk = blockIdx.x;
  if (bk >= n * m.K) return;
  const int32_t cb = flag[bk] ? (int32_t)(c0 + pos[bk]) : -1;
  if (threadIdx.x == 0) m.cslot[bk] = cb;
  if (cb < 0) return;
  for (int64_t v = threadIdx.x; v < B3; v += blockDim.x)
    m.calpha[(int64_t)cb * B3 + v] = alpha[bk * B3 + v];
}

__global__ void k_keys_to_ijk(const uint64_t* __restrict__ keys, int64_t n, int32_t* ijk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = keys[i];
  ijk[3 * i] = (int32_t)((k >> 42) & 0x1FFFFF) - (1 << 20);
  ijk[3 * i + 1] = (int32_t)((k >> 21) & 0x1FFFFF) - (1 << 20);
  ijk[3 * i + 2] = (int32_t)(k & 0x1FFFFF) - (1 << 20);
}

__global__ void k_ijk_to_keys(const int32_t* __restrict__ ijk, int64_t n, int32_t log2B,
                              uint64_t* keys, uint32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t bx = ijk[3 * i], by = ijk[3 * i + 1], bz = ijk[3 * i + 2];
  const int32_t lim = (1 << 20) >> log2B;   // the block's voxels stay in [-2^20, 2^20)
  if (bx < -lim || bx >= lim || by < -lim || by >= lim || bz < -lim || bz >= lim) {
    atomicOr(err, DEVERR_RANGE);
    keys[i] = 0;
    return;
  }
  keys[i] = smki_block_key(bx, by, bz);
}

__global__ void k_adjacent_dups(const uint64_t* __restrict__ s, int64_t n, uint32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i + 1 < n && s[i] == s[i + 1]) atomicOr(err, DEVERR_DUP);
}

__global__ void k_iota(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// captured inserts: device-side counts and checks (single small workgroups)
// ---------------------------------------------------------------------------
__global__ void k_batch_start(const int64_t* __restrict__ hdr, int64_t* __restrict__ counts,
                              unsigned long long* __restrict__ stats) {
  if (threadIdx.x == 0 && hdr[0]) {
    counts[0] = hdr[1];
    counts[1] = hdr[2];
  }
  for (int i = threadIdx.x; i < 4 * SMKI_STAT_COPIES; i += blockDim.x) stats[i] = 0ull;
}

__global__ void k_batch_rows(const int64_t* __restrict__ sc, int64_t cap_rows,
                             int64_t* __restrict__ pc, uint32_t* __restrict__ err) {
  const int64_t nf = sc[0];
  const int64_t nk = (int64_t)((const int32_t*)(sc + 1))[0];
  int64_t nt = nk + nf;
  if (nt > cap_rows) {
    atomicOr(err, DEVERR_CAPACITY);
    nt = cap_rows;   // (hit rows never exceed cap_rows: it is at least the hits)
  }
  pc[0] = nt;
  pc[1] = nk;
  pc[2] = nt - nk;
}

__global__ void k_batch_units(const int32_t* __restrict__ si, int64_t cap_slots,
                              int64_t cap_units, uint32_t* __restrict__ err) {
  if (si[0] > cap_slots || si[2] > cap_units) atomicOr(err, DEVERR_CAPACITY);
}

__global__ void k_batch_alloc_check(const int32_t* __restrict__ cnt,
                                    const int64_t* __restrict__ counts, int64_t pool_cap,
                                    int64_t cpool_cap, int64_t hcap, uint32_t* __restrict__ err) {
  const int64_t nb = counts[0] + cnt[0], nc = counts[1] + cnt[1];
  if (nb > pool_cap || nc > cpool_cap || 2 * nb > hcap) atomicOr(err, DEVERR_CAPACITY);
}

__global__ void k_batch_commit(const int32_t* __restrict__ cnt, int64_t* __restrict__ counts,
                               const uint32_t* __restrict__ err, uint32_t* __restrict__ map_err,
                               const int64_t* __restrict__ pc, const int32_t* __restrict__ si,
                               int64_t* __restrict__ out) {
  const uint32_t e = *err;
  if (e == 0) {
    counts[0] += cnt[0];
    counts[1] += cnt[1];
  } else {
    atomicOr(map_err, e);
  }
  out[0] = e;
  out[1] = e ? 0 : cnt[0];
  out[2] = e ? 0 : cnt[1];
  out[3] = pc[0];
  out[4] = pc[1];
  out[5] = pc[2];
  out[6] = si[0];
  out[7] = si[1];
  out[8] = si[2];
}

// An ordinary insert's new block counts, added on the device to the counts the
// host held before it (the host reads them back at its next synchronisation),
// and copied to out (read back with the insert counters).  The allocation
// kernel does the same when it runs; this serves an insert with no targets.
__global__ void k_commit_counts(const int32_t* __restrict__ cnt, int64_t* __restrict__ counts,
                                int64_t n_blocks, int64_t n_cblocks, int32_t* __restrict__ out) {
  counts[0] = n_blocks + cnt[0];
  counts[1] = n_cblocks + cnt[1];
  out[0] = cnt[0];
  out[1] = cnt[1];
}

}  // namespace

hipError_t launch_commit_counts(const int32_t* cnt, int64_t* counts, int64_t n_blocks,
                                int64_t n_cblocks, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_commit_counts, dim3(1), dim3(1), 0, st, cnt, counts, n_blocks, n_cblocks,
                     out);
  return hipGetLastError();
}

hipError_t launch_batch_start(const int64_t* hdr, int64_t* counts, unsigned long long* stats,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_batch_start, dim3(1), dim3(256), 0, st, hdr, counts, stats);
  return hipGetLastError();
}

hipError_t launch_batch_rows(const int64_t* sc, int64_t cap_rows, int64_t* pc, uint32_t* err,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_batch_rows, dim3(1), dim3(1), 0, st, sc, cap_rows, pc, err);
  return hipGetLastError();
}

hipError_t launch_batch_units(const int32_t* si, int64_t cap_slots, int64_t cap_units,
                              uint32_t* err, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_units, dim3(1), dim3(1), 0, st, si, cap_slots, cap_units, err);
  return hipGetLastError();
}

hipError_t launch_batch_alloc_check(const int32_t* cnt, const int64_t* counts, int64_t pool_cap,
                                    int64_t cpool_cap, int64_t hcap, uint32_t* err,
                                    hipStream_t st) {
  hipLaunchKernelGGL(k_batch_alloc_check, dim3(1), dim3(1), 0, st, cnt, counts, pool_cap,
                     cpool_cap, hcap, err);
  return hipGetLastError();
}

hipError_t launch_batch_commit(const int32_t* cnt, int64_t* counts, const uint32_t* err,
                               uint32_t* map_err, const int64_t* pc, const int32_t* si,
                               int64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_commit, dim3(1), dim3(1), 0, st, cnt, counts, err, map_err, pc, si,
                     out);
  return hipGetLastError();
}

hipError_t launch_query(const MapDev& m, const int32_t* ijk, int64_t M, float* alpha, float* mean,
                        float* var, int32_t* label, float* p_occ, int32_t free_class,
                        hipStream_t st) {
  if (M <= 0) return hipSuccess;
  // K <= 255: at most 8 classes per lane
  const int seg = m.K <= 32 ? 4 : m.K <= 64 ? 8 : m.K <= 128 ? 16 : 32;
  const unsigned grid = nblk(M * seg, 256);
  switch (seg) {
    case 4:
      hipLaunchKernelGGL(k_query<4>, dim3(grid), dim3(256), 0, st, m, ijk, M, alpha, mean, var,
                         label, p_occ, free_class);
      break;
    case 8:
      hipLaunchKernelGGL(k_query<8>, dim3(grid), dim3(256), 0, st, m, ijk, M, alpha, mean, var,
                         label, p_occ, free_class);
      break;
    case 16:
      hipLaunchKernelGGL(k_query<16>, dim3(grid), dim3(256), 0, st, m, ijk, M, alpha, mean, var,
                         label, p_occ, free_class);
      break;
    default:
      hipLaunchKernelGGL(k_query<32>, dim3(grid), dim3(256), 0, st, m, ijk, M, alpha, mean, var,
                         label, p_occ, free_class);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_hash_clear(const MapDev& m, hipStream_t st) {
  hipLaunchKernelGGL(k_hash_clear, dim3(nblk(m.hcap, 256)), dim3(256), 0, st, m.hkeys, m.hcap);
  return hipGetLastError();
}

hipError_t launch_hash_insert_slots(const MapDev& m, int64_t slot0, int64_t n, uint32_t* err,
                                    hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hash_insert_slots, dim3(nblk(n, 256)), dim3(256), 0, st, m, slot0, n, err);
  return hipGetLastError();
}

hipError_t launch_gather_blocks(const MapDev& m, const uint32_t* order, int64_t n,
                                float* alpha_out, hipStream_t st) {
  const int64_t tot = n * (int64_t)m.K * m.B * m.B * m.B;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_blocks, dim3(nblk(tot, 256)), dim3(256), 0, st, m, order, n,
                     alpha_out);
  return hipGetLastError();
}

hipError_t launch_import_flags(const MapDev& m, const float* alpha, int64_t n, int32_t* flag,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_import_flags, dim3((unsigned)(n * m.K)), dim3(256), 0, st, m, alpha, n,
                     flag);
  return hipGetLastError();
}

hipError_t launch_import_copy(const MapDev& m, const float* alpha, int64_t n, const int32_t* flag,
                              const int32_t* pos, int64_t c0, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_import_copy, dim3((unsigned)(n * m.K)), dim3(256), 0, st, m, alpha, n,
                     flag, pos, c0);
  return hipGetLastError();
}

hipError_t launch_block_keys_to_ijk(const uint64_t* keys, int64_t n, int32_t* ijk, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_keys_to_ijk, dim3(nblk(n, 256)), dim3(256), 0, st, keys, n, ijk);
  return hipGetLastError();
}

hipError_t launch_ijk_to_block_keys(const int32_t* ijk, int64_t n, int32_t log2B, uint64_t* keys,
                                    uint32_t* err, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ijk_to_keys, dim3(nblk(n, 256)), dim3(256), 0, st, ijk, n, log2B, keys,
                     err);
  return hipGetLastError();
}

hipError_t launch_adjacent_dups(const uint64_t* sorted, int64_t n, uint32_t* err, hipStream_t st) {
  if (n <= 1) return hipSuccess;
  hipLaunchKernelGGL(k_adjacent_dups, dim3(nblk(n, 256)), dim3(256), 0, st, sorted, n, err);
  return hipGetLastError();
}

hipError_t launch_iota_u32(uint32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(nblk(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}
