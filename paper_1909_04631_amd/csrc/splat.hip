// The S-BKI map update: Eq. (7) of Gan et al. (arXiv 1909.04631) at the
// centroid of every voxel near the scan, with the sparse kernel of Eq. (8):
//
//   alpha_v^k += sum over rows t with |x_t - c_v| < l of  sigma0 f(|x_t - c_v| / l) [y_t = k]
//
// Organisation (deterministic, no floating-point atomics):
//
//   splat   Rows are sorted by (class, block, voxel cell).  One wavefront takes
//           a chunk of at most `chunk` rows of one (class, block) and keeps,
//           in LDS, the partial sums of the region that those rows can reach:
//           the block grown by the stencil reach R on every side.  For each
//           row (taken in sorted order, uniform across the wavefront), lane i
//           handles the voxel offsets i, i + 64, ... of the list of voxels that
//           can lie within l of a point of the row's cell; lanes accumulate in
//           registers while consecutive rows share a cell and add to LDS when
//           the cell changes.  Every lane owns distinct LDS addresses, so the
//           sum order of every voxel is the row order: run-to-run identical.
//           The region is written out as the chunk's partial sums.
//   merge   One workgroup per target block: for every class and every
//           neighbouring (class, block) whose region covers a voxel, add the
//           partial sums of its chunks in chunk order (compensated), then add
//           the total to the voxel's concentration: one exclusive write per
//           (voxel, class).
//
// Kernel evaluation: with s = 1 - r, f(1 - s) = s^5 Q(s^2) exactly (the Taylor
// series of the sparse kernel about r = 1 has only odd powers from s^5 on);
// Q is a degree-7 polynomial fit, which keeps f relatively accurate up to the
// support edge where the direct formula cancels.
#include "smki_gather.h"

namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)ceil_div_i64(n > 0 ? n : 1, t); }

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = SMKI_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SMKI_WAVE);
  return v;
}

__device__ __forceinline__ void unlin3(int64_t lin, const int32_t n[3], int32_t out[3]) {
  out[2] = (int32_t)(lin % n[2]);
  lin /= n[2];
  out[1] = (int32_t)(lin % n[1]);
  out[0] = (int32_t)(lin / n[1]);
}

// sigma0 f(r) from s = 1 - r: s^5 * (sigma0 Q)(s^2)
__device__ __forceinline__ float kernel_weight(const float* c, float s) {
  const float u = s * s;
  float q = c[0];
#pragma unroll
  for (int i = 1; i < SMKI_POLY_N; ++i) q = fmaf(q, u, c[i]);
  return (u * u) * (s * q);
}

// ---------------------------------------------------------------------------
// target blocks and work units
// ---------------------------------------------------------------------------
__global__ void k_mark_targets(const int32_t* __restrict__ slot_lin,
                               const int32_t* __restrict__ d_nslots, int32_t max_slots,
                               BucketGeom g, int3 eblo, int3 enb, int32_t DB,
                               int32_t* __restrict__ mark) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= max_slots || s >= *d_nslots) return;
  int32_t p[3];
  unlin3(slot_lin[s] % g.n_blocks, g.nb, p);
  const int32_t ex = p[0] + (g.blo[0] - eblo.x), ey = p[1] + (g.blo[1] - eblo.y),
                ez = p[2] + (g.blo[2] - eblo.z);
  for (int dx = -DB; dx <= DB; ++dx)
    for (int dy = -DB; dy <= DB; ++dy)
      for (int dz = -DB; dz <= DB; ++dz)
        mark[((int64_t)(ex + dx) * enb.y + (ey + dy)) * enb.z + (ez + dz)] = 1;
}

__global__ void k_list_targets(const int32_t* __restrict__ mark, const int32_t* __restrict__ mpos,
                               int64_t n, int32_t* __restrict__ tgt, int32_t* __restrict__ ext2t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (mark[i]) {
    tgt[mpos[i]] = (int32_t)i;
    ext2t[i] = mpos[i];
  } else {
    ext2t[i] = -1;
  }
}

// chunks of every (class, block) slot
__global__ void k_slot_units(const int32_t* __restrict__ prefix, const int32_t* __restrict__ d_nslots,
                             int32_t max_slots, int32_t B3, int32_t chunk,
                             int32_t* __restrict__ nunits) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= max_slots) return;
  int32_t u = 0;
  if (s < *d_nslots) {
    const int32_t* P = prefix + (int64_t)s * (B3 + 1);
    u = (P[B3] - P[0] + chunk - 1) / chunk;
  }
  nunits[s] = u;
}

__global__ void k_unit_table(const int32_t* __restrict__ nunits, const int32_t* __restrict__ ustart,
                             int32_t max_slots, int2* __restrict__ units) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= max_slots) return;
  const int32_t n = nunits[s], b = ustart[s];
  for (int32_t k = 0; k < n; ++k) units[b + k] = make_int2(s, k);
}

// ---------------------------------------------------------------------------
// splat
// ---------------------------------------------------------------------------
// NS: steps of 64 voxel offsets, enough for any stencil of reach R.
template <int R>
struct Steps {
  static constexpr int NS = ((2 * R + 1) * (2 * R + 1) * (2 * R + 1) + SMKI_WAVE - 1) / SMKI_WAVE;
};

template <int B, int R>
__global__ void __launch_bounds__(SMKI_WAVE) k_splat(SplatArgs a) {
  constexpr int DR = B + 2 * R;                 // region edge (voxels)
  constexpr int DR3 = DR * DR * DR;
  constexpr int B3 = B * B * B;
  constexpr int NS = Steps<R>::NS;
  __shared__ float acc[DR3];
  const int lane = threadIdx.x;
  const int2 u = a.units[blockIdx.x];
  const int32_t slot = u.x;
  const int32_t* P = a.prefix + (int64_t)slot * (B3 + 1);
  const int32_t r0 = P[0] + u.y * a.chunk;
  const int32_t r1 = min(P[B3], r0 + a.chunk);
  for (int i = lane; i < DR3; i += SMKI_WAVE) acc[i] = 0.0f;
  // per-lane offset data for each step: voxel-centre offset (in the frame of
  // the row's cell, minus the block-centre shift) and region-index offset
  float wx[NS], wy[NS], wz[NS];
  int32_t wl[NS];
  const float res = a.g.res;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int o = s * SMKI_WAVE + lane;
    if (o < a.noff) {
      const int4 off = a.offs[o];
      wx[s] = ((float)off.x + (0.5f - 0.5f * B)) * res;
      wy[s] = ((float)off.y + (0.5f - 0.5f * B)) * res;
      wz[s] = ((float)off.z + (0.5f - 0.5f * B)) * res;
      wl[s] = (off.x * DR + off.y) * DR + off.z;
    } else {
      wx[s] = wy[s] = wz[s] = 1.0e30f;   // never within l
      wl[s] = 0;
    }
  }
  const int ns = (a.noff + SMKI_WAVE - 1) / SMKI_WAVE;
  __syncthreads();
  // first cell holding row r0
  int32_t lo = 0, hi = B3 - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (P[mid] <= r0) lo = mid; else hi = mid - 1;
  }
  const float4* __restrict__ pts = a.pts;
  int32_t npair = 0;
  for (int32_t c = lo; c < B3; ++c) {
    const int32_t c0 = max(P[c], r0), c1 = min(P[c + 1], r1);
    if (c0 >= r1) break;
    if (c0 >= c1) continue;
    const int32_t cx = c / (B * B), cy = (c / B) % B, cz = c % B;
    const float ux0 = (float)cx * res, uy0 = (float)cy * res, uz0 = (float)cz * res;
    float sum[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) sum[s] = 0.0f;
    for (int32_t r = c0; r < c1; ++r) {
      const float4 q = pts[r];
      const float ux = q.x - ux0, uy = q.y - uy0, uz = q.z - uz0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s < ns) {
          const float dx = ux - wx[s], dy = uy - wy[s], dz = uz - wz[s];
          const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          if (d2 < a.l2) {
            const float d = __builtin_amdgcn_sqrtf(d2);
            const float sv = fmaxf(fmaf(-d, a.inv_l, 1.0f), 0.0f);
            sum[s] += kernel_weight(a.coef, sv);
            ++npair;
          }
        }
      }
    }
    const int32_t cb = ((cx + R) * DR + (cy + R)) * DR + (cz + R);
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (s < ns && sum[s] != 0.0f) acc[cb + wl[s]] += sum[s];
    // the next cell's lanes may own these addresses: keep the LDS order
    __syncthreads();
  }
  __syncthreads();
  float* out = a.part + (int64_t)blockIdx.x * DR3;
  for (int i = lane; i < DR3; i += SMKI_WAVE) out[i] = acc[i];
  // which target blocks received a contribution
  const int32_t plane_lin = a.slot_lin[slot];
  const int32_t blin = plane_lin % a.g.n_blocks;
  int32_t pb[3];
  unlin3(blin, a.g.nb, pb);
  uint32_t touched = 0;   // bit (dx+1)*9 + (dy+1)*3 + (dz+1) for DB = 1
  for (int i = lane; i < DR3; i += SMKI_WAVE) {
    if (acc[i] != 0.0f) {
      const int vx = i / (DR * DR) - R, vy = (i / DR) % DR - R, vz = i % DR - R;
      const int dx = vx < 0 ? -1 : (vx >= B ? 1 : 0);
      const int dy = vy < 0 ? -1 : (vy >= B ? 1 : 0);
      const int dz = vz < 0 ? -1 : (vz >= B ? 1 : 0);
      touched |= 1u << ((dx + 1) * 9 + (dy + 1) * 3 + (dz + 1));
    }
  }
#pragma unroll
  for (int o = SMKI_WAVE / 2; o > 0; o >>= 1) touched |= __shfl_xor(touched, o, SMKI_WAVE);
  if (lane < 27 && ((touched >> lane) & 1u)) {
    const int dx = lane / 9 - 1, dy = (lane / 3) % 3 - 1, dz = lane % 3 - 1;
    const int64_t e = ((int64_t)(pb[0] + a.g.blo[0] - a.eblo[0] + dx) * a.enb[1] +
                       (pb[1] + a.g.blo[1] - a.eblo[1] + dy)) * a.enb[2] +
                      (pb[2] + a.g.blo[2] - a.eblo[2] + dz);
    const int32_t t = a.ext2t[e];
    if (t >= 0) a.tgt_active[t] = 1;
  }
  const int64_t np = wave_sum_i64((int64_t)npair);
  if (lane == 0) atomicAdd(&a.stats[1], (unsigned long long)np);
}

// ---------------------------------------------------------------------------
// merge: one workgroup of 256 threads per target block, 2 voxels per thread
// ---------------------------------------------------------------------------
template <int B, int R>
__global__ void __launch_bounds__(256) k_merge(SplatArgs a, int32_t n_targets) {
  constexpr int DR = B + 2 * R;
  constexpr int DR3 = DR * DR * DR;
  constexpr int B3 = B * B * B;
  constexpr int VPT = (B3 + 255) / 256;
  const int32_t t = blockIdx.x;
  if (t >= n_targets || !a.tgt_active[t]) return;
  const int32_t mslot = a.tgt_slot[t];
  int32_t bt[3];
  unlin3(a.tgt_elin[t], a.enb, bt);
  for (int q = 0; q < 3; ++q) bt[q] += a.eblo[q];
  float* A = a.alpha + (int64_t)mslot * a.K * B3;
  bool upd[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) upd[j] = false;
  for (int y = 0; y < a.K; ++y) {
    float sum[VPT], comp[VPT];
#pragma unroll
    for (int j = 0; j < VPT; ++j) sum[j] = comp[j] = 0.0f;
    bool any = false;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const int px = bt[0] + dx - a.g.blo[0], py = bt[1] + dy - a.g.blo[1],
                    pz = bt[2] + dz - a.g.blo[2];
          if (px < 0 || py < 0 || pz < 0 || px >= a.g.nb[0] || py >= a.g.nb[1] || pz >= a.g.nb[2])
            continue;
          const int32_t s = a.dense[(int64_t)y * a.g.n_blocks +
                                    ((int64_t)px * a.g.nb[1] + py) * a.g.nb[2] + pz];
          if (s < 0) continue;
          const int32_t u0 = a.ustart[s], u1 = u0 + a.nunits[s];
          any = true;
#pragma unroll
          for (int j = 0; j < VPT; ++j) {
            const int v = threadIdx.x + 256 * j;
            if (v >= B3) continue;
            // voxel v of the target block in the region of the neighbour block
            const int rx = v / (B * B) - dx * B + R, ry = (v / B) % B - dy * B + R,
                      rz = v % B - dz * B + R;
            if (rx < 0 || ry < 0 || rz < 0 || rx >= DR || ry >= DR || rz >= DR) continue;
            const int ri = (rx * DR + ry) * DR + rz;
            for (int32_t w = u0; w < u1; ++w) {
              const float yv = a.part[(int64_t)w * DR3 + ri] - comp[j];
              const float tv = sum[j] + yv;
              comp[j] = (tv - sum[j]) - yv;
              sum[j] = tv;
            }
          }
        }
    if (!any) continue;
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const int v = threadIdx.x + 256 * j;
      if (v < B3 && sum[j] != 0.0f) {
        A[(int64_t)y * B3 + v] += sum[j];
        upd[j] = true;
      }
    }
  }
  int32_t nup = 0;
#pragma unroll
  for (int j = 0; j < VPT; ++j) nup += upd[j] ? 1 : 0;
  __shared__ int32_t red[256 / SMKI_WAVE];
  const int64_t wsum = wave_sum_i64(nup);
  if ((threadIdx.x & (SMKI_WAVE - 1)) == 0) red[threadIdx.x / SMKI_WAVE] = (int32_t)wsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t tot = 0;
    for (int i = 0; i < 256 / SMKI_WAVE; ++i) tot += red[i];
    atomicAdd(&a.stats[0], (unsigned long long)tot);
  }
}

// map-slot lookup of the active targets; new blocks are marked for allocation
__global__ void k_map_lookup(MapDev m, SplatArgs a, int32_t n_targets,
                             int32_t* __restrict__ tgt_slot, int32_t* __restrict__ is_new) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_targets) return;
  if (!a.tgt_active[t]) {
    tgt_slot[t] = -1;
    is_new[t] = 0;
    return;
  }
  int32_t bt[3];
  unlin3(a.tgt_elin[t], a.enb, bt);
  const uint64_t key = smki_block_key(bt[0] + a.eblo[0], bt[1] + a.eblo[1], bt[2] + a.eblo[2]);
  uint64_t h = smki_mix64(key) & (uint64_t)(m.hcap - 1);
  int32_t slot = -1;
  for (int64_t probe = 0; probe < m.hcap; ++probe) {
    const uint64_t k = m.hkeys[h];
    if (k == key) { slot = m.hvals[h]; break; }
    if (k == ~0ull) break;
    h = (h + 1) & (uint64_t)(m.hcap - 1);
  }
  tgt_slot[t] = slot;
  is_new[t] = slot < 0 ? 1 : 0;
}

__global__ void k_assign_new(MapDev m, SplatArgs a, int32_t n_targets,
                             const int32_t* __restrict__ is_new, const int32_t* __restrict__ rank,
                             int64_t n_old, int32_t* __restrict__ tgt_slot,
                             uint32_t* __restrict__ err) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_targets || !is_new[t]) return;
  int32_t bt[3];
  unlin3(a.tgt_elin[t], a.enb, bt);
  const uint64_t key = smki_block_key(bt[0] + a.eblo[0], bt[1] + a.eblo[1], bt[2] + a.eblo[2]);
  const int32_t slot = (int32_t)(n_old + rank[t]);
  tgt_slot[t] = slot;
  m.bkeys[slot] = key;
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

__global__ void k_fill_alpha0(float* __restrict__ alpha, int64_t n, float a0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) alpha[i] = a0;
}

template <int B, int R>
hipError_t launch_splat_br(const SplatArgs& a, int64_t n_units, int32_t n_targets, bool merge,
                           hipStream_t st) {
  if (!merge) {
    if (n_units > 0)
      hipLaunchKernelGGL((k_splat<B, R>), dim3((unsigned)n_units), dim3(SMKI_WAVE), 0, st, a);
  } else {
    if (n_targets > 0)
      hipLaunchKernelGGL((k_merge<B, R>), dim3((unsigned)n_targets), dim3(256), 0, st, a,
                         n_targets);
  }
  return hipGetLastError();
}

template <int B>
hipError_t launch_splat_b(const SplatArgs& a, int64_t n_units, int32_t n_targets, bool merge,
                          hipStream_t st) {
  switch (a.R) {
    case 0: return launch_splat_br<B, 0>(a, n_units, n_targets, merge, st);
    case 1: return launch_splat_br<B, 1>(a, n_units, n_targets, merge, st);
    case 2: return launch_splat_br<B, 2>(a, n_units, n_targets, merge, st);
    case 3: return launch_splat_br<B, 3>(a, n_units, n_targets, merge, st);
    case 4: return launch_splat_br<B, 4>(a, n_units, n_targets, merge, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_splat_any(const SplatArgs& a, int64_t n_units, int32_t n_targets, bool merge,
                            hipStream_t st) {
  if (a.noff > SMKI_WAVE * ((2 * a.R + 1) * (2 * a.R + 1) * (2 * a.R + 1) + SMKI_WAVE - 1) / SMKI_WAVE)
    return hipErrorInvalidValue;
  switch (a.g.B) {
    case 4: return launch_splat_b<4>(a, n_units, n_targets, merge, st);
    case 8: return launch_splat_b<8>(a, n_units, n_targets, merge, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_mark_targets(const int32_t* slot_lin, const int32_t* d_nslots, int32_t max_slots,
                               const BucketGeom& g, const int32_t eblo[3], const int32_t enb[3],
                               int32_t DB, int32_t* mark, hipStream_t st) {
  if (max_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_targets, dim3(nblk(max_slots, 256)), dim3(256), 0, st, slot_lin,
                     d_nslots, max_slots, g, make_int3(eblo[0], eblo[1], eblo[2]),
                     make_int3(enb[0], enb[1], enb[2]), DB, mark);
  return hipGetLastError();
}

hipError_t launch_list_targets(const int32_t* mark, const int32_t* mpos, int64_t n_ext,
                               int32_t* tgt_elin, int32_t* ext2t, hipStream_t st) {
  if (n_ext <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_list_targets, dim3(nblk(n_ext, 256)), dim3(256), 0, st, mark, mpos, n_ext,
                     tgt_elin, ext2t);
  return hipGetLastError();
}

hipError_t launch_slot_units(const int32_t* prefix, const int32_t* d_nslots, int32_t max_slots,
                             int32_t B3, int32_t chunk, int32_t* nunits, hipStream_t st) {
  if (max_slots <= 0) return hipSuccess;
  if (chunk <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_slot_units, dim3(nblk(max_slots, 256)), dim3(256), 0, st, prefix, d_nslots,
                     max_slots, B3, chunk, nunits);
  return hipGetLastError();
}

hipError_t launch_unit_table(const int32_t* nunits, const int32_t* ustart, int32_t max_slots,
                             int2* units, hipStream_t st) {
  if (max_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_table, dim3(nblk(max_slots, 256)), dim3(256), 0, st, nunits, ustart,
                     max_slots, units);
  return hipGetLastError();
}

hipError_t launch_splat(const SplatArgs& a, int64_t n_units, hipStream_t st) {
  return launch_splat_any(a, n_units, 0, false, st);
}

hipError_t launch_merge(const SplatArgs& a, int32_t n_targets, hipStream_t st) {
  return launch_splat_any(a, 0, n_targets, true, st);
}

hipError_t launch_map_lookup(const MapDev& m, const SplatArgs& a, int32_t n_targets,
                             int32_t* tgt_slot, int32_t* is_new, hipStream_t st) {
  if (n_targets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_map_lookup, dim3(nblk(n_targets, 256)), dim3(256), 0, st, m, a, n_targets,
                     tgt_slot, is_new);
  return hipGetLastError();
}

hipError_t launch_assign_new(const MapDev& m, const SplatArgs& a, int32_t n_targets,
                             const int32_t* is_new, const int32_t* new_rank, int64_t n_old,
                             int32_t* tgt_slot, uint32_t* err, hipStream_t st) {
  if (n_targets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_assign_new, dim3(nblk(n_targets, 256)), dim3(256), 0, st, m, a, n_targets,
                     is_new, new_rank, n_old, tgt_slot, err);
  return hipGetLastError();
}

hipError_t launch_fill_alpha0(const MapDev& m, int64_t slot0, int64_t nslots, hipStream_t st) {
  const int64_t per = (int64_t)m.K * m.B * m.B * m.B;
  const int64_t n = nslots * per;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_alpha0, dim3(nblk(n, 256)), dim3(256), 0, st, m.alpha + slot0 * per,
                     n, m.alpha0);
  return hipGetLastError();
}
