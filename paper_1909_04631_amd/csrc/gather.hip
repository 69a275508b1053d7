// The S-BKI map update: Eq. (7) of Gan et al. (arXiv 1909.04631) evaluated at
// the centroid of every voxel near the scan, with the sparse kernel of Eq. (8):
//
//   alpha_v^k += sum over rows t with |x_t - c_v| < l of  sigma0 f(|x_t - c_v| / l) [y_t = k]
//
// Organisation (gather, deterministic, no floating-point atomics):
//   * target blocks = map blocks within reach of a block that holds rows;
//   * one wavefront per (target block, 4^3 sub-tile, part): each lane owns one
//     voxel, the (start, end) row ranges of the sub-tile's staged box of voxel
//     cells sit in LDS, and the lane walks the columns of its own stencil
//     (every cell that can hold a row within l of its centre), reading the
//     sorted rows coalesced-by-locality from HBM;
//   * rows too dense for one wavefront are split into parts by a per-lane
//     window over the lane's candidate sequence; parts write partial sums that a
//     second kernel adds in part order, so the result is run-to-run identical.
//
// Kernel evaluation: with s = 1 - r, f(1 - s) = s^5 Q(s^2) exactly (the Taylor
// series of the sparse kernel about r = 1 has only odd powers from s^5 on);
// Q is a degree-7 polynomial fit, which keeps f relatively accurate up to the
// support edge where the direct formula cancels.
#include "smki_gather.h"

namespace {

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

// Slot of the point-grid block holding voxel v (-1 outside the grid / empty).
__device__ __forceinline__ int32_t slot_of_block(const BucketGeom& g, const int32_t* dense,
                                                 int32_t bx, int32_t by, int32_t bz) {
  const int32_t px = bx - g.blo[0], py = by - g.blo[1], pz = bz - g.blo[2];
  if (px < 0 || py < 0 || pz < 0 || px >= g.nb[0] || py >= g.nb[1] || pz >= g.nb[2]) return -1;
  return dense[((int64_t)px * g.nb[1] + py) * g.nb[2] + pz];
}

// Rows in the box [U0, U0 + D)^3 of voxel cells (one set); lanes split the columns.
__device__ int64_t box_count(const GatherArgs& a, int set, const int32_t U0[3]) {
  const BucketGeom& g = a.g;
  const int32_t B = g.B, B3 = B * B * B;
  const int32_t* dense = a.dense[set];
  const int32_t* prefix = a.prefix[set];
  int64_t cnt = 0;
  for (int col = threadIdx.x; col < a.D * a.D; col += SMKI_WAVE) {
    const int32_t vx = U0[0] + col / a.D, vy = U0[1] + col % a.D;
    const int32_t bx = vx >> g.log2B, by = vy >> g.log2B;
    const int32_t lx = vx - bx * B, ly = vy - by * B;
    int32_t z = U0[2];
    const int32_t zl = U0[2] + a.D - 1;
    while (z <= zl) {
      const int32_t bz = z >> g.log2B;
      const int32_t ze = min(zl, (bz + 1) * B - 1);
      const int32_t slot = slot_of_block(g, dense, bx, by, bz);
      if (slot >= 0) {
        const int32_t* P = prefix + (int64_t)slot * (B3 + 1);
        const int32_t base = (lx * B + ly) * B;
        cnt += P[base + (ze - bz * B) + 1] - P[base + (z - bz * B)];
      }
      z = ze + 1;
    }
  }
  return cnt;
}

__global__ void k_mark_targets(const int32_t* __restrict__ slot_lin,
                               const int32_t* __restrict__ d_nslots, int32_t max_slots,
                               BucketGeom g, int3 eblo, int3 enb, int32_t DB,
                               int32_t* __restrict__ mark) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= max_slots || s >= *d_nslots) return;
  int32_t p[3];
  unlin3(slot_lin[s], g.nb, p);
  const int32_t ex = p[0] + (g.blo[0] - eblo.x), ey = p[1] + (g.blo[1] - eblo.y),
                ez = p[2] + (g.blo[2] - eblo.z);
  for (int dx = -DB; dx <= DB; ++dx)
    for (int dy = -DB; dy <= DB; ++dy)
      for (int dz = -DB; dz <= DB; ++dz)
        mark[((int64_t)(ex + dx) * enb.y + (ey + dy)) * enb.z + (ez + dz)] = 1;
}

__global__ void k_list_targets(const int32_t* __restrict__ mark, const int32_t* __restrict__ mpos,
                               int64_t n, int32_t* __restrict__ tgt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && mark[i]) tgt[mpos[i]] = (int32_t)i;
}

__device__ __forceinline__ void target_block(const GatherArgs& a, int32_t elin, int32_t bt[3]) {
  unlin3(elin, a.enb, bt);
  bt[0] += a.eblo[0];
  bt[1] += a.eblo[1];
  bt[2] += a.eblo[2];
}

__device__ __forceinline__ void sub_tile_origin(const GatherArgs& a, const int32_t bt[3],
                                                int32_t gsub, int32_t U0[3], int32_t goff[3]) {
  const int32_t ns = a.nsub;
  goff[0] = (gsub / (ns * ns)) * SMKI_TILE;
  goff[1] = ((gsub / ns) % ns) * SMKI_TILE;
  goff[2] = (gsub % ns) * SMKI_TILE;
  for (int q = 0; q < 3; ++q) U0[q] = bt[q] * a.g.B + goff[q] - a.R;
}

__global__ void __launch_bounds__(SMKI_WAVE) k_plan(GatherArgs a, int32_t n_targets, float frac,
                                                    int4* __restrict__ plan,
                                                    int32_t* __restrict__ active) {
  const int32_t nsub3 = a.nsub * a.nsub * a.nsub;
  const int64_t w = blockIdx.x;
  const int32_t t = (int32_t)(w / nsub3), gsub = (int32_t)(w % nsub3);
  if (t >= n_targets) return;
  int32_t bt[3], U0[3], goff[3];
  target_block(a, a.tgt_elin[t], bt);
  sub_tile_origin(a, bt, gsub, U0, goff);
  int64_t U = box_count(a, 0, U0) + box_count(a, 1, U0);
  U = wave_sum_i64(U);
  if (threadIdx.x == 0) {
    int32_t parts = 0, win = 0;
    if (U > 0) {
      const double est = (double)U * frac / (double)a.budget;
      parts = (int32_t)fmin(fmax(ceil(est), 1.0), 65536.0);
      win = (int32_t)((U + parts - 1) / parts);
      atomicOr(&active[t], 1);
    }
    plan[w] = make_int4(parts, win, -1, 0);
  }
}

__global__ void k_map_lookup(MapDev m, GatherArgs a, int32_t n_targets,
                             const int32_t* __restrict__ active, int32_t* __restrict__ tgt_slot,
                             int32_t* __restrict__ is_new, uint32_t* __restrict__ err) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_targets) return;
  if (!active[t]) {
    tgt_slot[t] = -1;
    is_new[t] = 0;
    return;
  }
  int32_t bt[3];
  target_block(a, a.tgt_elin[t], bt);
  const uint64_t key = smki_block_key(bt[0], bt[1], bt[2]);
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

__global__ void k_assign_new(MapDev m, GatherArgs a, int32_t n_targets,
                             const int32_t* __restrict__ is_new, const int32_t* __restrict__ rank,
                             int64_t n_old, int32_t* __restrict__ tgt_slot,
                             uint32_t* __restrict__ err) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_targets || !is_new[t]) return;
  int32_t bt[3];
  target_block(a, a.tgt_elin[t], bt);
  const uint64_t key = smki_block_key(bt[0], bt[1], bt[2]);
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

__global__ void k_plan_counts(const int4* __restrict__ plan, int64_t n, int32_t* __restrict__ np,
                              int32_t* __restrict__ ns) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t p = plan[i].x;
  np[i] = p;
  ns[i] = p > 1 ? p : 0;
}

__global__ void k_units(int4* __restrict__ plan, const int32_t* __restrict__ unit_off,
                        const int32_t* __restrict__ split_off, int64_t n, int32_t nsub3,
                        int4* __restrict__ units) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int4 p = plan[i];
  if (p.x <= 0) return;
  p.z = p.x > 1 ? split_off[i] : -1;
  plan[i] = p;
  const int32_t t = (int32_t)(i / nsub3), gsub = (int32_t)(i % nsub3);
  for (int32_t part = 0; part < p.x; ++part) units[unit_off[i] + part] = make_int4(t, gsub, part, 0);
}

// sigma0 f(r) from s = 1 - r: s^5 * (sigma0 Q)(s^2)
__device__ __forceinline__ float kernel_weight(const float* c, float s) {
  const float u = s * s;
  float q = c[0];
#pragma unroll
  for (int i = 1; i < SMKI_POLY_N; ++i) q = fmaf(q, u, c[i]);
  return (u * u) * (s * q);
}

// Walk one point set for this lane's voxel inside the window [wlo, whi) of its
// candidate sequence; pos carries the running candidate count across sets.
template <bool HITS>
__device__ __forceinline__ void walk_set(const GatherArgs& a, int set, const int32_t* cs,
                                         const int32_t* ce, const int32_t U0[3],
                                         const int32_t bt[3], const int32_t vl[3],
                                         const int32_t bl[3], int64_t wlo, int64_t whi,
                                         int64_t& pos, float& acc, int32_t& cnt, float* hacc) {
  const int32_t D = a.D, R = a.R, B = a.g.B;
  const float4* __restrict__ pts = a.pts[set];
  const float res = a.g.res;
  const int lane = threadIdx.x;
  for (int c = 0; c < a.ncols; ++c) {
    if (__all(pos >= whi)) break;
    const StencilCol sc = a.cols[c];
    const int32_t cx = vl[0] + R + sc.dx, cy = vl[1] + R + sc.dy;
    // block offsets of this column relative to the target block
    const int32_t nbx = (U0[0] + cx) >> a.g.log2B, nby = (U0[1] + cy) >> a.g.log2B;
    // voxel centre relative to the centre of the point block holding the column
    const float ex = (float)(bl[0] + 0.5f - 0.5f * B - (float)((nbx - bt[0]) * B)) * res;
    const float ey = (float)(bl[1] + 0.5f - 0.5f * B - (float)((nby - bt[1]) * B)) * res;
    int32_t z = vl[2] + R - sc.h;
    const int32_t z1 = vl[2] + R + sc.h;
    const int32_t rowbase = (cx * D + cy) * D;
    while (z <= z1) {
      const int32_t nbz = (U0[2] + z) >> a.g.log2B;
      const int32_t ze = min(z1, (nbz + 1) * B - 1 - U0[2]);
      const int32_t S = cs[rowbase + z], E = ce[rowbase + ze];
      const float ez = (float)(bl[2] + 0.5f - 0.5f * B - (float)((nbz - bt[2]) * B)) * res;
      const int64_t n = (int64_t)(E - S);
      const int64_t lo = max((int64_t)0, wlo - pos), hi = min(n, whi - pos);
      for (int64_t q = S + lo; q < S + hi; ++q) {
        const float4 p = pts[q];
        const float dx = p.x - ex, dy = p.y - ey, dz = p.z - ez;
        const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        if (d2 < a.l2) {
          const float d = __builtin_sqrtf(d2);
          const float s = fmaxf(fmaf(-d, a.inv_l, 1.0f), 0.0f);
          const float wgt = kernel_weight(a.coef, s);
          if (HITS) {
            const int32_t y = __float_as_int(p.w);
            hacc[y * SMKI_WAVE + lane] += wgt;
          } else {
            acc += wgt;
          }
          ++cnt;
        }
      }
      pos += n;
      z = ze + 1;
    }
  }
}

// Stage (start, end) row ranges of every voxel cell of the box into LDS.
__device__ __forceinline__ void stage_box(const GatherArgs& a, int set, const int32_t U0[3],
                                          int32_t* cs, int32_t* ce) {
  const BucketGeom& g = a.g;
  const int32_t B = g.B, B3 = B * B * B, D = a.D;
  const int32_t* dense = a.dense[set];
  const int32_t* prefix = a.prefix[set];
  for (int c = threadIdx.x; c < D * D * D; c += SMKI_WAVE) {
    const int32_t vx = U0[0] + c / (D * D), vy = U0[1] + (c / D) % D, vz = U0[2] + c % D;
    const int32_t bx = vx >> g.log2B, by = vy >> g.log2B, bz = vz >> g.log2B;
    const int32_t slot = slot_of_block(g, dense, bx, by, bz);
    int32_t S = 0, E = 0;
    if (slot >= 0) {
      const int32_t loc = ((vx - bx * B) * B + (vy - by * B)) * B + (vz - bz * B);
      const int32_t* P = prefix + (int64_t)slot * (B3 + 1);
      S = P[loc];
      E = P[loc + 1];
    }
    cs[c] = S;
    ce[c] = E;
  }
}

__global__ void __launch_bounds__(SMKI_WAVE) k_gather(GatherArgs a) {
  extern __shared__ int32_t lds[];
  const int32_t D3 = a.D * a.D * a.D;
  int32_t* cs = lds;
  int32_t* ce = lds + D3;
  float* hacc = (float*)(lds + 2 * D3);
  const int lane = threadIdx.x;
  const int4 u = a.units[blockIdx.x];
  const int32_t t = u.x, gsub = u.y, part = u.z;
  const int32_t nsub3 = a.nsub * a.nsub * a.nsub;
  const int4 pl = a.plan[(int64_t)t * nsub3 + gsub];
  const int64_t wlo = (int64_t)part * pl.y, whi = wlo + pl.y;
  int32_t bt[3], U0[3], goff[3];
  target_block(a, a.tgt_elin[t], bt);
  sub_tile_origin(a, bt, gsub, U0, goff);
  const int32_t vl[3] = {lane >> 4, (lane >> 2) & 3, lane & 3};        // voxel in the sub-tile
  const int32_t bl[3] = {goff[0] + vl[0], goff[1] + vl[1], goff[2] + vl[2]};  // voxel in the block
  for (int k = 0; k < a.K; ++k) hacc[k * SMKI_WAVE + lane] = 0.0f;
  int64_t pos = 0;
  float acc = 0.0f;
  int32_t cnt = 0;
  stage_box(a, 0, U0, cs, ce);
  __syncthreads();
  walk_set<false>(a, 0, cs, ce, U0, bt, vl, bl, wlo, whi, pos, acc, cnt, hacc);
  __syncthreads();
  stage_box(a, 1, U0, cs, ce);
  __syncthreads();
  walk_set<true>(a, 1, cs, ce, U0, bt, vl, bl, wlo, whi, pos, acc, cnt, hacc);
  __syncthreads();
  hacc[a.free_class * SMKI_WAVE + lane] += acc;
  const int32_t B = a.g.B, B3 = B * B * B;
  if (pl.x == 1) {
    const int32_t slot = a.tgt_slot[t];
    float* A = a.alpha + (int64_t)slot * a.K * B3 + (bl[0] * B + bl[1]) * B + bl[2];
    for (int k = 0; k < a.K; ++k) {
      const float dk = hacc[k * SMKI_WAVE + lane];
      if (dk != 0.0f) A[(int64_t)k * B3] += dk;
    }
    const unsigned long long nz = __popcll(__ballot(cnt > 0));
    const int64_t tot = wave_sum_i64((int64_t)cnt);
    if (lane == 0) {
      atomicAdd(&a.stats[0], nz);
      atomicAdd(&a.stats[1], (unsigned long long)tot);
    }
  } else {
    const int64_t pidx = (int64_t)pl.z + part;
    float* P = a.part_acc + pidx * a.K * SMKI_WAVE;
    for (int k = 0; k < a.K; ++k) P[k * SMKI_WAVE + lane] = hacc[k * SMKI_WAVE + lane];
    a.part_cnt[pidx * SMKI_WAVE + lane] = cnt;
  }
}

__global__ void __launch_bounds__(SMKI_WAVE) k_merge(GatherArgs a, int64_t n_plan) {
  const int64_t w = blockIdx.x;
  if (w >= n_plan) return;
  const int4 pl = a.plan[w];
  if (pl.x <= 1) return;
  const int lane = threadIdx.x;
  const int32_t nsub3 = a.nsub * a.nsub * a.nsub;
  const int32_t t = (int32_t)(w / nsub3), gsub = (int32_t)(w % nsub3);
  int32_t bt[3], U0[3], goff[3];
  target_block(a, a.tgt_elin[t], bt);
  sub_tile_origin(a, bt, gsub, U0, goff);
  const int32_t bl[3] = {goff[0] + (lane >> 4), goff[1] + ((lane >> 2) & 3), goff[2] + (lane & 3)};
  const int32_t B = a.g.B, B3 = B * B * B;
  const int32_t slot = a.tgt_slot[t];
  float* A = a.alpha + (int64_t)slot * a.K * B3 + (bl[0] * B + bl[1]) * B + bl[2];
  for (int k = 0; k < a.K; ++k) {
    float s = 0.0f;
    for (int32_t p = 0; p < pl.x; ++p)
      s += a.part_acc[(((int64_t)pl.z + p) * a.K + k) * SMKI_WAVE + lane];
    if (s != 0.0f) A[(int64_t)k * B3] += s;
  }
  int64_t cnt = 0;
  for (int32_t p = 0; p < pl.x; ++p) cnt += a.part_cnt[((int64_t)pl.z + p) * SMKI_WAVE + lane];
  const unsigned long long nz = __popcll(__ballot(cnt > 0));
  const int64_t tot = wave_sum_i64(cnt);
  if (lane == 0) {
    atomicAdd(&a.stats[0], nz);
    atomicAdd(&a.stats[1], (unsigned long long)tot);
  }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)ceil_div_i64(n > 0 ? n : 1, t); }

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
                               int32_t* tgt_elin, hipStream_t st) {
  if (n_ext <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_list_targets, dim3(nblk(n_ext, 256)), dim3(256), 0, st, mark, mpos, n_ext,
                     tgt_elin);
  return hipGetLastError();
}

hipError_t launch_plan(const GatherArgs& a, int32_t n_targets, float frac, int4* plan,
                       int32_t* active, hipStream_t st) {
  const int64_t n = (int64_t)n_targets * a.nsub * a.nsub * a.nsub;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan, dim3((unsigned)n), dim3(SMKI_WAVE), 0, st, a, n_targets, frac, plan,
                     active);
  return hipGetLastError();
}

hipError_t launch_map_lookup(const MapDev& m, const GatherArgs& a, int32_t n_targets,
                             const int32_t* active, int32_t* tgt_slot, int32_t* is_new,
                             uint32_t* err, hipStream_t st) {
  if (n_targets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_map_lookup, dim3(nblk(n_targets, 256)), dim3(256), 0, st, m, a, n_targets,
                     active, tgt_slot, is_new, err);
  return hipGetLastError();
}

hipError_t launch_assign_new(const MapDev& m, const GatherArgs& a, int32_t n_targets,
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

hipError_t launch_plan_counts(const int4* plan, int64_t n, int32_t* nparts, int32_t* nsplit,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_counts, dim3(nblk(n, 256)), dim3(256), 0, st, plan, n, nparts, nsplit);
  return hipGetLastError();
}

hipError_t launch_units(int4* plan, const int32_t* unit_off, const int32_t* split_off, int64_t n,
                        int32_t nsub3, int4* units, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_units, dim3(nblk(n, 256)), dim3(256), 0, st, plan, unit_off, split_off, n,
                     nsub3, units);
  return hipGetLastError();
}

size_t gather_lds_bytes(const GatherArgs& a) {
  return sizeof(int32_t) * 2 * (size_t)a.D * a.D * a.D + sizeof(float) * (size_t)a.K * SMKI_WAVE;
}

hipError_t launch_gather(const GatherArgs& a, int64_t n_units, hipStream_t st) {
  if (n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)n_units), dim3(SMKI_WAVE), gather_lds_bytes(a), st,
                     a);
  return hipGetLastError();
}

hipError_t launch_merge(const GatherArgs& a, int64_t n_plan, hipStream_t st) {
  if (n_plan <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge, dim3((unsigned)n_plan), dim3(SMKI_WAVE), 0, st, a, n_plan);
  return hipGetLastError();
}
