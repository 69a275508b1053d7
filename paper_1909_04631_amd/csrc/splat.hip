// The S-BKI map update: Eq. (7) of Gan et al. (arXiv 1909.04631) at the
// centroid of every voxel near the scan, with the sparse kernel of Eq. (8):
//
//   alpha_v^k += sum over rows t with |x_t - c_v| < l of  sigma0 f(|x_t - c_v| / l) [y_t = k]
//
// Organisation (deterministic: no floating-point atomics across wavefronts):
//
//   splat   Rows are sorted by (class, block, voxel cell).  One wavefront takes
//           a chunk of at most `chunk` rows of one (class, block) and keeps,
//           in LDS, the partial sums of the region that those rows can reach:
//           the block grown by the stencil reach R on every side.  Rows are
//           taken 64 at a time, octant by octant of their position in their
//           cell, each octant's rows in sorted order; for each row (uniform
//           across the wavefront), lane i handles the voxel offsets i, i + 64,
//           ... of the list of voxels that can lie within l of a point of that
//           octant of the row's cell.  Lanes accumulate in registers while
//           consecutive rows share a cell and octant, and add to LDS when it
//           changes.  Every lane owns distinct LDS addresses and the LDS runs a
//           wavefront's adds in issue order, so the sum order of every voxel is
//           fixed: run-to-run identical.  The region is written out as the
//           chunk's partial sums.
//   merge   One workgroup per target block: for every class, add in double
//           the partial sums that the neighbouring (class, block) regions
//           covering a voxel hold for it (first chunks in a fixed neighbour
//           order, then the later chunks in chunk order), then add the total
//           to the voxel's concentration: one exclusive write per (voxel,
//           class).
//
// Kernel evaluation: with s = 1 - r, f(1 - s) = s^5 Q(s^2) exactly (the Taylor
// series of the sparse kernel about r = 1 has only odd powers from s^5 on);
// Q is a degree-6 polynomial fit (kernel_poly.py), which keeps f relatively
// accurate (about 1.3e-6 in binary32) up to the support edge, where the direct
// formula cancels.  The splat evaluates sigma0 Q, whose coefficients it forms
// once per work unit from Q divided by its leading coefficient (monic) and
// sigma0 times that coefficient.
#include "smki_gather.h"
#include "smki_pieces.h"

namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)ceil_div_i64(n > 0 ? n : 1, t); }

// Grid coordinates of a linear block index.  Every grid here has at most 2^30
// blocks (the insert refuses larger ones), so 32-bit arithmetic suffices.
__device__ __forceinline__ void unlin3(int32_t lin, const int32_t n[3], int32_t out[3]) {
  out[2] = lin % n[2];
  lin /= n[2];
  out[1] = lin % n[1];
  out[0] = lin / n[1];
}

// ---------------------------------------------------------------------------
// target blocks and work units
// ---------------------------------------------------------------------------
// The per-slot kernels that run before the slot count reaches the host take a
// grid of at most this many workgroups and stride over the count read on the
// device (a grid sized for the capacity would mostly start workgroups that exit).
constexpr int kSlotGrid = 1024;

__global__ void k_mark_targets(const int32_t* __restrict__ slot_lin,
                               const int32_t* __restrict__ d_nslots, int32_t max_slots,
                               BucketGeom g, int3 eblo, int3 enb, int32_t DB,
                               int32_t* __restrict__ mark) {
  const int32_t n = min(max_slots, *d_nslots);
  for (int32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    int32_t p[3];
    unlin3(slot_lin[s] % (int32_t)g.n_blocks, g.nb, p);
    const int32_t ex = p[0] + (g.blo[0] - eblo.x), ey = p[1] + (g.blo[1] - eblo.y),
                  ez = p[2] + (g.blo[2] - eblo.z);
    for (int dx = -DB; dx <= DB; ++dx)
      for (int dy = -DB; dy <= DB; ++dy)
        for (int dz = -DB; dz <= DB; ++dz)
          mark[((int64_t)(ex + dx) * enb.y + (ey + dy)) * enb.z + (ez + dz)] = 1;
  }
}

// entry i of the extended grid: its target index, and the target's grid index
__device__ __forceinline__ void list_target(const int32_t* __restrict__ mark,
                                            const int32_t* __restrict__ mpos, int64_t i,
                                            int32_t* __restrict__ tgt, int32_t* __restrict__ ext2t) {
  if (mark[i]) {
    tgt[mpos[i]] = (int32_t)i;
    ext2t[i] = mpos[i];
  } else {
    ext2t[i] = -1;
  }
}

__global__ void k_list_targets(const int32_t* __restrict__ mark, const int32_t* __restrict__ mpos,
                               int64_t n, int32_t* __restrict__ tgt, int32_t* __restrict__ ext2t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) list_target(mark, mpos, i, tgt, ext2t);
}

// chunks of every (class, block) slot (entries past the slot count are not
// written); cfirst (nullable): 1 + the first slot of each class with slots
// (slots are in class-major order)
__global__ void k_slot_units(const int32_t* __restrict__ head, const int32_t* __restrict__ d_nslots,
                             int32_t max_slots, int32_t chunk, int32_t* __restrict__ nunits,
                             const int32_t* __restrict__ slot_lin, int64_t n_blocks,
                             int32_t* __restrict__ cfirst) {
  const int32_t n = min(max_slots, *d_nslots);
  for (int32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    nunits[s] = max(0, (head[s + 1] - head[s] + chunk - 1) / chunk);
    if (cfirst) {
      const int32_t nb = (int32_t)n_blocks, c = slot_lin[s] / nb;
      if (s == 0 || slot_lin[s - 1] / nb != c) cfirst[c] = s + 1;
    }
  }
}

// Work units of every slot: (first row, end row, slot, class), chunk rows each.
// order (optional): the splat's launch order, longest first: the slots'
// full-chunk units (slot s's k-th at ustart[s] - s + k, since every slot before
// it has one last unit), then every slot's last unit (at F + s, F = units -
// slots).  A late long unit would leave the rest of the GPU idle at the end.
__global__ void k_unit_table(const int32_t* __restrict__ nunits, const int32_t* __restrict__ ustart,
                             const int32_t* __restrict__ head, const int32_t* __restrict__ slot_lin,
                             int64_t n_blocks, int32_t chunk, int32_t max_slots,
                             const int32_t* __restrict__ d_nslots,
                             const int32_t* __restrict__ d_nunits, int4* __restrict__ units,
                             int32_t* __restrict__ order, int32_t cap_units) {
  // eight threads per slot, taking its units k = j, j + 8, ...; the grid
  // strides over the slots (a multiple of eight threads)
  // (a captured insert whose slots or units outgrow their tables stores no
  // unit; its abort word is set and the map is left unchanged)
  if (*d_nslots > max_slots || *d_nunits > cap_units || *d_nunits < 0) return;
  const int32_t ns = *d_nslots;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; (t >> 3) < ns; t += stride) {
    const int32_t s = (int32_t)(t >> 3);
    const int32_t n = nunits[s];
    if (n == 0) continue;
    const int32_t b = ustart[s], h0 = head[s], h1 = head[s + 1];
    const int32_t plane = slot_lin[s] / (int32_t)n_blocks;
    for (int32_t k = (int32_t)(t & 7); k < n; k += 8) {
      const int32_t r0 = h0 + k * chunk;
      units[b + k] = make_int4(r0, min(h1, r0 + chunk), s, plane);
      if (order) order[k + 1 < n ? b - s + k : (*d_nunits - *d_nslots) + s] = b + k;
    }
  }
}

// ---------------------------------------------------------------------------
// splat
// ---------------------------------------------------------------------------
// NS: steps of 64 voxel offsets, enough for the first-octant stencil of any
// l / res with reach R (its size is largest at l / res -> R + 1/2: 1, 23, 90,
// 230, 471 offsets for R = 0..4).
template <int R>
struct Steps {
  static constexpr int MAXOFF = R == 0 ? 1 : R == 1 ? 23 : R == 2 ? 90 : R == 3 ? 230 : 471;
  static constexpr int NS = (MAXOFF + SMKI_WAVE - 1) / SMKI_WAVE;
  // fewest steps a reach-R stencil can need (its size at l / res -> R - 1/2)
  static constexpr int NSMIN = R <= 2 ? 1 : R == 3 ? 2 : 4;
};

// NS = ceil(stencil size / 64), the steps each row takes (compiled per value
// so that the steps of a row are independent straight-line code).  W: rows carry
// a weight (soft measurements) that scales their kernel values.  RPS: rows per
// step; 2 for a stencil of at most 32 offsets (one step), whose two halves of
// the wavefront then take two rows at once.
template <int B, int R, int NS, bool W, int RPS>
__global__ void __launch_bounds__(SMKI_WAVE) k_splat(SplatArgs a) {
  static_assert(RPS == 1 || (RPS == 2 && NS == 1), "two rows per step only for a one-step stencil");
  constexpr int DR = B + 2 * R;                 // region edge (voxels)
  constexpr int DR3 = DR * DR * DR;
  constexpr int NACC4 = (DR3 + 3) / 4;
  __shared__ float4 acc4[NACC4];   // the region
  // the batch being processed, its rows in octant-major order: (|u| per axis,
  // |u|^2), keys and (W) weights
  __shared__ float4 rowq[SMKI_WAVE];
  __shared__ int32_t keyq[SMKI_WAVE];
  __shared__ float wq[W ? SMKI_WAVE : 1];
  float* acc = (float*)acc4;
  const int lane = threadIdx.x;
  // the zero words that the merge reads for absent pieces
  if (blockIdx.x == 0 && lane < SMKI_PART_HEAD) a.part[lane] = 0.0f;
  if (a.dn_units && (int32_t)blockIdx.x >= *a.dn_units) return;   // capacity launch
  if (a.abort_word && *a.abort_word) return;   // (a failed captured insert: the units may be stale)
  const int32_t uid = a.uorder ? a.uorder[blockIdx.x] : (int32_t)blockIdx.x;
  const int4 u = a.units[uid];   // (first row, end row, slot, class)
  const int32_t r0 = u.x, r1 = u.y;
  const float4 kc = a.cls[u.w];         // the kernel of the unit's class
  const float l2 = kc.x, inv_l = kc.y, cscale = kc.z;
  // sigma0 Q (the class's scale times the monic fit), highest degree first: the
  // sums of kernel values go to LDS as they are
  float cq[SMKI_POLY_N];
  cq[0] = cscale;
#pragma unroll
  for (int i = 1; i < SMKI_POLY_N; ++i) cq[i] = cscale * a.mcoef[i];
  for (int i = lane; i < NACC4; i += SMKI_WAVE) acc4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // Per lane, for each step: one voxel offset o of the first-octant stencil
  // (offsets whose centre can lie within l of a point in the (+,+,+) octant of
  // its cell) as a centre offset in metres, and its region-index offset for
  // each of the 8 octants: a row in octant (sx, sy, sz) reaches voxel
  // cell + (sx ox, sy oy, sz oz), at the distance from |u| to o.
  // The squared distance is evaluated as |q|^2 + |w|^2 - 2 q.w (q: the row's
  // |u|, at most res sqrt(3)/2; w: the offset's centre): nw = -2 w, w2 = |w|^2.
  float nwx[NS], nwy[NS], nwz[NS], w2[NS];
  int32_t wl[8][NS];
  bool pad[NS];
  const double res = (double)a.g.res;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int o = s * SMKI_WAVE + (RPS == 2 ? (lane & 31) : lane);
    pad[s] = o >= a.noff;
    int4 off = a.offs[min(o, a.noff - 1)];   // unconditional load, pad lanes reset below
    if (pad[s]) off = make_int4(0, 0, 0, 0);
    {
      const double x = off.x * res, y = off.y * res, z = off.z * res;
      nwx[s] = (float)(-2.0 * x);
      nwy[s] = (float)(-2.0 * y);
      nwz[s] = (float)(-2.0 * z);
      w2[s] = pad[s] ? 1.0e30f : (float)(x * x + y * y + z * z);   // pad: never within l
    }
#pragma unroll
    for (int oc = 0; oc < 8; ++oc)
      wl[oc][s] = ((oc & 1) ? -off.x : off.x) * DR * DR + ((oc & 2) ? -off.y : off.y) * DR +
                  ((oc & 4) ? -off.z : off.z);
  }
  __syncthreads();
  const float4* __restrict__ pts = a.pts;
  uint32_t npair = 0;
  // The open group: rows of one (cell, octant), whose sums the lanes hold in
  // registers; its region index and the region-index offsets of its octant.
  int32_t gkey = -1, gcb = 0, goc = -1;
  int32_t cw[NS];
  float sum[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    sum[s] = 0.0f;
    cw[s] = 0;
  }
  const int xlane4 = (lane ^ 32) << 2;   // byte address of the other half's lane (RPS == 2)
  // Flush: every lane adds its group sum (0 included) to its voxel of the
  // region, all reads of a flush first, then all writes; pad lanes (no stencil
  // offset) touch nothing.  Within one flush the lanes' addresses are distinct;
  // the LDS executes one wavefront's reads and writes in issue order and the
  // compiler keeps flushes in program order (signal fence), so every voxel
  // sums its groups in processing order: run-to-run identical.
  auto flush = [&]() {
    if constexpr (RPS == 2) {
      // both halves hold sums of the same group for the same offsets: the
      // lower half adds their total
      const float tot =
          sum[0] + __int_as_float(__builtin_amdgcn_ds_bpermute(xlane4, __float_as_int(sum[0])));
      const int32_t fa0 = gcb + cw[0];
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (lane < 32 && !pad[0]) acc[fa0] = acc[fa0] + tot;
      sum[0] = 0.0f;
      return;
    }
    int32_t fa[NS];
    float fo[NS];
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      fa[s] = gcb + cw[s];
      // only the last step has pad lanes (NS = ceil(stencil size / 64))
      if (!(s == NS - 1 && pad[s])) fo[s] = acc[fa[s]];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!(s == NS - 1 && pad[s])) acc[fa[s]] = fo[s] + sum[s];
      sum[s] = 0.0f;
    }
  };
  // Rows are staged 64 at a time in registers (lane i holds row base + i); two
  // batches alternate so that one loads while the other is processed.
  // A batch: the rows' records and (W) their weights.
  struct Batch {
    float4 r;
    float w;
  };
  // A batch's rows are found through the permutation (sorted row -> record):
  // its indices are loaded one batch before its records.  Unconditional: lanes
  // past the end re-read row r1 - 1.
  auto load_index = [&](int32_t base) -> int32_t {
    const int32_t row = min(base + lane, r1 - 1);
    return a.perm ? (int32_t)a.perm[row] : row;
  };
  auto load_batch = [&](int32_t v) {
    Batch b;
    b.r = pts[v];
    b.w = W ? a.wts[v] : 1.0f;
    return b;
  };
  // A row's octant selects the mirrored region offsets; rows come octant by
  // octant, so this changes at most eight times per batch (the open group is
  // flushed first).
  auto octant = [&](int32_t key) {
    const int oc = key & 7;
    if (oc == goc) return;
    if (gkey >= 0) flush();
    gkey = -1;
    goc = oc;
    switch (oc) {
#define SMKI_OCT_CASE(OC)                                             \
  case OC:                                                            \
    _Pragma("unroll") for (int s = 0; s < NS; ++s) cw[s] = wl[OC][s]; \
    break;
      SMKI_OCT_CASE(0) SMKI_OCT_CASE(1) SMKI_OCT_CASE(2) SMKI_OCT_CASE(3)
      SMKI_OCT_CASE(4) SMKI_OCT_CASE(5) SMKI_OCT_CASE(6) SMKI_OCT_CASE(7)
#undef SMKI_OCT_CASE
    }
  };
  auto cell_base = [&](int32_t key) {
    const uint32_t c = (uint32_t)key >> 3;   // the cell: x, y, z of log2(B) bits each
    return (int32_t)(((c / (B * B) + R) * DR + ((c / B) % B + R)) * DR + (c % B + R));
  };
  // One row (j of the batch, its |u| and |u|^2 in q, read from LDS one row
  // earlier): octant and group change, the read of the next row (jn, into qn),
  // then the row's contribution to every stencil offset.  The wait for q sits
  // first, so that no wait for the next read stalls the arithmetic.
  auto row = [&](int32_t keyp, float wp, int j, const float4& q, int jn, float4& qn) {
    asm volatile("" ::"v"(q.x), "v"(q.y), "v"(q.z), "v"(q.w));
    const int32_t key = __builtin_amdgcn_readlane(keyp, j);
    const float wr = W ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wp), j)) : 1.0f;
    octant(key);
    if (key != gkey) {
      if (gkey >= 0) flush();
      gkey = key;
      gcb = cell_base(key);
    }
    qn = rowq[jn];
    // Branch-free: every lane evaluates its pair; s = 1 - d/l clamped to [0, 1]
    // (the clamp is free on the fused multiply-add) is 0 out of support, which
    // zeroes the weight s^5 Q(s^2).
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      // |d2| only guards rounding below 0 when the row sits on the voxel centre
      const float d2 = fmaf(q.z, nwz[s], fmaf(q.y, nwy[s], fmaf(q.x, nwx[s], q.w + w2[s])));
      const bool in = d2 < l2;
      const uint64_t inm = __ballot(in);
      npair += (uint32_t)__popcll(inm);
      // the last step holds the farthest offsets (the stencil is ordered by
      // distance): a row that reaches none of them skips it
      if (NS > 1 && s == NS - 1 && inm == 0) continue;
      const float d = __builtin_amdgcn_sqrtf(fabsf(d2));
      const float sv = __builtin_amdgcn_fmed3f(fmaf(-d, inv_l, 1.0f), 0.0f, 1.0f);
      const float uu = sv * sv;
      float qq = fmaf(uu, cq[0], cq[1]);
#pragma unroll
      for (int i = 2; i < SMKI_POLY_N; ++i) qq = fmaf(qq, uu, cq[i]);
      if (W)
        sum[s] = fmaf(uu * uu, (sv * wr) * qq, sum[s]);
      else
        sum[s] = fmaf(uu * uu, sv * qq, sum[s]);
    }
  };
  // Two rows at once (RPS == 2): j in the lower half of the wavefront, jh (-1:
  // none) in the upper, of one octant, keys klo and khi, their |u| and |u|^2 in
  // q (per half).  A half's sums join the open group when its row belongs to
  // it; a pair that spans two groups flushes in between.
  auto pair = [&](float wp, int j, int jh, int32_t klo, int32_t khi, const float4& q) {
    const bool hi = lane >= 32;
    const bool act = !hi || jh >= 0;   // this half has a row
    float wr = 1.0f;
    if (W) {
      const float wlo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wp), j));
      const float whi = jh >= 0 ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wp), jh)) : 0.0f;
      wr = hi ? whi : wlo;
    }
    const float d2 = fmaf(q.z, nwz[0], fmaf(q.y, nwy[0], fmaf(q.x, nwx[0], q.w + w2[0])));
    const bool in = act && d2 < l2;
    npair += (uint32_t)__popcll(__ballot(in));
    const float d = __builtin_amdgcn_sqrtf(fabsf(d2));
    const float sv = __builtin_amdgcn_fmed3f(fmaf(-d, inv_l, 1.0f), 0.0f, 1.0f);
    const float uu = sv * sv;
    float qq = fmaf(uu, cq[0], cq[1]);
#pragma unroll
    for (int i = 2; i < SMKI_POLY_N; ++i) qq = fmaf(qq, uu, cq[i]);
    float v = W ? (uu * uu) * ((sv * wr) * qq) : (uu * uu) * (sv * qq);
    if (!act) v = 0.0f;
    // (the value is complete before any flush's LDS traffic is issued)
    asm volatile("" ::"v"(v) : "memory");
    octant(klo);
    if (klo != gkey) {
      if (gkey >= 0) flush();
      gkey = klo;
      gcb = cell_base(klo);
    }
    if (khi == gkey) {
      sum[0] += v;
    } else {
      sum[0] += hi ? 0.0f : v;
      if (jh >= 0) {
        flush();
        gkey = khi;
        gcb = cell_base(khi);
        sum[0] = hi ? v : 0.0f;
      }
    }
  };
  // One batch: its rows go to LDS in octant-major order (each octant's rows in
  // sorted order) and are read back by every lane, one row (or pair) at a time.
  auto process = [&](const Batch& bt, int32_t base) {
    const int nb = min(SMKI_WAVE, r1 - base);
    const float4& cur = bt.r;
    // (consume the weights here, so that no wait for their load sits in the row loop)
    if (W) asm volatile("" ::"v"(bt.w));
    const float q2l = fmaf(cur.x, cur.x, fmaf(cur.y, cur.y, cur.z * cur.z));
    const int32_t keyl = __float_as_int(cur.w);
    const bool valid = lane < nb;
    // slot of each row: the rows of smaller octants, then its rank in its own
    // (lanes past the batch keep slots past it, never read)
    int slot = lane;
    uint32_t run = 0;
#pragma unroll
    for (int oc = 0; oc < 8; ++oc) {
      const bool mine = valid && (keyl & 7) == oc;
      const uint64_t m = __ballot(mine);
      if (mine)
        slot = (int)(run + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)));
      run += (uint32_t)__popcll(m);
    }
    // (the previous batch's reads of these arrays were issued before the writes)
    rowq[slot] = make_float4(cur.x, cur.y, cur.z, q2l);
    keyq[slot] = keyl;
    if (W) wq[slot] = bt.w;
    const int32_t keyp = keyq[lane];
    const float wp = W ? wq[lane] : 1.0f;
    if constexpr (RPS == 2) {
      // pairs of consecutive rows of one octant (a row whose successor lies in
      // another octant, or the last row, goes alone)
      int j = 0;
      while (j < nb) {
        const int32_t klo = __builtin_amdgcn_readlane(keyp, j);
        int jh = -1;
        int32_t khi = -1;
        if (j + 1 < nb) {
          const int32_t k1 = __builtin_amdgcn_readlane(keyp, j + 1);
          if (((k1 ^ klo) & 7) == 0) {
            jh = j + 1;
            khi = k1;
          }
        }
        const float4 q = rowq[(lane >= 32 && jh >= 0) ? jh : j];
        pair(wp, j, jh, klo, khi, q);
        j = (jh >= 0 ? jh : j) + 1;
      }
    } else {
      // rows in order, through two row registers: the next row is read while
      // this one is processed
      float4 qa = rowq[0], qb;
      for (int j = 0; j < nb; j += 2) {
        row(keyp, wp, j, qa, min(j + 1, nb - 1), qb);
        if (j + 1 >= nb) break;
        row(keyp, wp, j + 1, qb, min(j + 2, nb - 1), qa);
      }
    }
  };
  Batch ba = load_batch(load_index(r0));
  int32_t vb = load_index(r0 + SMKI_WAVE);
  for (int32_t base = r0; base < r1; base += 2 * SMKI_WAVE) {
    const Batch bb = load_batch(vb);
    const int32_t va = load_index(base + 2 * SMKI_WAVE);
    process(ba, base);
    if (base + SMKI_WAVE >= r1) break;
    ba = load_batch(va);
    vb = load_index(base + 3 * SMKI_WAVE);
    process(bb, base + SMKI_WAVE);
  }
  if (gkey >= 0) flush();
  __syncthreads();
  // Write out the pieces that received a contribution (and that the selection
  // keeps): per piece, every lane reads its elements into registers, the
  // wavefront votes on any non-zero value, and a non-zero piece is stored
  // contiguously.  Piece geometry is compile-time, so the index arithmetic
  // folds to constants.
  using PC = Pieces<B, R>;
  float* out = a.part + SMKI_PART_HEAD + (int64_t)uid * DR3;
  constexpr int MAXPER = (B * B * B + SMKI_WAVE - 1) / SMKI_WAVE;   // the largest piece is the block
  uint32_t touched = 0;
  if constexpr (MAXPER > 8) {
#pragma unroll
    for (int p = 0; p < 27; ++p) {
      if (!((a.piece_mask >> p) & 1u)) continue;
      const int ey = PC::ext((p / 3) % 3 - 1), ez = PC::ext(p % 3 - 1);
      const int sx = PC::rstart(p / 9 - 1), sy = PC::rstart((p / 3) % 3 - 1),
                sz = PC::rstart(p % 3 - 1);
      const int n = PC::size(p), b = PC::base(p);
      // large blocks: vote while reading, then read again to store (no
      // register copy of the piece)
      bool nz = false;
      for (int i = lane; i < n; i += SMKI_WAVE) {
        const int lx = i / (ey * ez), ly = (i / ez) % ey, lz = i % ez;
        nz = nz || acc[((sx + lx) * DR + (sy + ly)) * DR + (sz + lz)] != 0.0f;
      }
      if (__ballot(nz) == 0) continue;
      touched |= 1u << p;
      for (int i = lane; i < n; i += SMKI_WAVE) {
        const int lx = i / (ey * ez), ly = (i / ez) % ey, lz = i % ez;
        out[b + i] = acc[((sx + lx) * DR + (sy + ly)) * DR + (sz + lz)];
      }
    }
  } else {
    // Region index of element i = lane + 64 k of a piece, relative to the
    // piece's first voxel, for each pair of (y, z) extents in {R, B}: computed
    // once here (the x extent only bounds i).
    constexpr int KRR = (B * R * R + SMKI_WAVE - 1) / SMKI_WAVE,
                  KRB = (B * R * B + SMKI_WAVE - 1) / SMKI_WAVE;
    int32_t lRR[KRR > 0 ? KRR : 1], lRB[KRB > 0 ? KRB : 1], lBR[KRB > 0 ? KRB : 1], lBB[MAXPER];
    auto rel = [&](int ey, int ez, int i) { return ((i / (ey * ez)) * DR + (i / ez) % ey) * DR + i % ez; };
#pragma unroll
    for (int k = 0; k < MAXPER; ++k) {
      const int i = lane + k * SMKI_WAVE;
      if (k < KRR) lRR[k] = rel(R, R, i);
      if (k < KRB) {
        lRB[k] = rel(R, B, i);
        lBR[k] = rel(B, R, i);
      }
      lBB[k] = rel(B, B, i);
    }
#pragma unroll
    for (int p = 0; p < 27; ++p) {
      if (!((a.piece_mask >> p) & 1u)) continue;
      const bool yr = (p / 3) % 3 != 1, zr = p % 3 != 1;   // y / z extent R (else B)
      const int sx = PC::rstart(p / 9 - 1), sy = PC::rstart((p / 3) % 3 - 1),
                sz = PC::rstart(p % 3 - 1);
      const int n = PC::size(p), b = PC::base(p);
      const int per = (n + SMKI_WAVE - 1) / SMKI_WAVE;
      const int S = (sx * DR + sy) * DR + sz;
      float v[MAXPER];
      bool nz = false;
#pragma unroll
      for (int k = 0; k < MAXPER; ++k) {
        v[k] = 0.0f;
        if (k < per && lane + k * SMKI_WAVE < n) {
          const int r = yr ? (zr ? lRR[k < KRR ? k : 0] : lRB[k < KRB ? k : 0])
                           : (zr ? lBR[k < KRB ? k : 0] : lBB[k]);
          v[k] = acc[S + r];
          nz = nz || v[k] != 0.0f;
        }
      }
      if (__ballot(nz) == 0) continue;
      touched |= 1u << p;
      float* ob = out + b;
#pragma unroll
      for (int k = 0; k < MAXPER; ++k)
        if (k < per && lane + k * SMKI_WAVE < n) ob[lane + k * SMKI_WAVE] = v[k];
    }
  }
  if (lane == 0) a.umask[uid] = touched;
  if (lane == 0)
    atomicAdd(&a.stats[(blockIdx.x % SMKI_STAT_COPIES) * 4 + 1], (unsigned long long)npair);
}

// ---------------------------------------------------------------------------
// merge
// ---------------------------------------------------------------------------
// Per slot: its units, the union of their non-zero pieces, and the first
// unit's own pieces.
// Eight threads per slot (one 8-lane group of a wavefront, active or exited
// together) OR the masks of units j, j + 8, ...
__device__ __forceinline__ void slot_info(const SplatArgs& a, int64_t t) {
  const int32_t s = (int32_t)(t >> 3), j = (int32_t)(t & 7);
  if (s >= (a.dn_slots ? min(a.n_slots, *a.dn_slots) : a.n_slots)) return;
  if (a.abort_word && *a.abort_word) return;   // (the unit tables may be stale)
  const int32_t u0 = a.ustart[s], nu = a.nunits[s];
  uint32_t m = 0;
  for (int32_t w = u0 + j; w < u0 + nu; w += 8) m |= a.umask[w];
  m |= __shfl_xor(m, 1, 8);
  m |= __shfl_xor(m, 2, 8);
  m |= __shfl_xor(m, 4, 8);
  if (j == 0) a.sinfo[s] = make_int4(u0, nu, (int32_t)m, nu > 0 ? (int32_t)a.umask[u0] : 0);
}

__global__ void k_slot_info(SplatArgs a) {
  slot_info(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// After the splat of an ordinary insert, three independent steps in one
// launch: workgroups [0, gc) clear nclear words from clr (the allocation's
// counts and flags), [gc, gc + gl) list the targets (k_list_targets), the rest
// summarise the slots' pieces (k_slot_info).  (Whole workgroups take one step.)
__global__ void k_after_splat(SplatArgs a, int32_t* __restrict__ clr, int64_t nclear, int64_t gc,
                              const int32_t* __restrict__ mark, const int32_t* __restrict__ mpos,
                              int64_t n_ext, int64_t gl, int32_t* __restrict__ tgt,
                              int32_t* __restrict__ ext2t) {
  const int64_t b = blockIdx.x;
  if (b < gc) {
    for (int64_t i = b * blockDim.x + threadIdx.x; i < nclear; i += gc * blockDim.x) clr[i] = 0;
  } else if (b < gc + gl) {
    const int64_t i = (b - gc) * blockDim.x + threadIdx.x;
    if (i < n_ext) list_target(mark, mpos, i, tgt, ext2t);
  } else {
    slot_info(a, (b - gc - gl) * blockDim.x + threadIdx.x);
  }
}

// Partial sum at element off of unit w's region; unit w < 0 reads the zero
// word at the head of the buffer.  Below 4 GiB of partial sums (WIDE false) the
// address is a 32-bit byte offset from the buffer base (unit times region size
// in a 24-bit multiply: fewer than 2^24 units fit there), so that a load takes
// one address register instead of two.
template <int DR3, bool WIDE>
__device__ __forceinline__ float part_at(const float* part, int32_t w, int32_t off) {
  if (WIDE) return part[w < 0 ? (int64_t)0 : SMKI_PART_HEAD + (int64_t)w * DR3 + off];
  const uint32_t e = ((uint32_t)SMKI_PART_HEAD + __umul24((uint32_t)w & 0xffffffu, (uint32_t)DR3) +
                      (uint32_t)off) * 4u;
  return *(const float*)((const char*)part + (w < 0 ? 0u : e));
}

// (B = 8 up to reach 3: at most 64 registers, eight wavefronts per SIMD)
// One workgroup per active target block, one thread per voxel (blocks of more
// than 1024 voxels: several voxels per thread).  Each thread first lists the
// neighbours whose regions cover its voxel and the offset of its voxel in the
// corresponding piece.  For a group of classes, the workgroup lists the classes
// whose rows reach this block and looks up the slots of the 27 neighbouring
// blocks into LDS (for all classes of the group at once when one round of
// lookups covers them, else for the listed classes), keeping for each neighbour
// only whether its units wrote the piece that lies in this block.  For every listed class, each thread adds, in double, the pieces that
// cover its voxel: the first chunks of all its candidates (loads issued
// together, in the fixed neighbour order; an absent one reads a zero word),
// then the later chunks of multi-chunk slots eight at a time; blocks allocated
// by this insert are written alpha0 + sum, older blocks updated in place where
// the sum is non-zero.  The per-thread state is kept small (packed candidates,
// slot entries re-read from LDS) so that 8 wavefronts fit per SIMD.
template <int B, int R, bool WIDE>
__global__ void __launch_bounds__((B * B * B < 1024 ? B * B * B : 1024), (B == 8 && R <= 3 && !WIDE) ? 8 : 1)
k_merge(SplatArgs a, int32_t n_targets) {
  using S = MergeShape<B, R>;
  constexpr int DR = B + 2 * R;
  constexpr int DR3 = DR * DR * DR;
  constexpr int B3 = S::B3, NT = S::NT, CPG = S::CPG, MAXC = S::MAXC, VPT = S::VPT;
  // [class (or listed class)][neighbour d]: (first unit, units) of the
  // neighbour's slot if some unit of it wrote piece 26 - d (the part of its
  // region inside this block), else (0, 0); units negated when the first unit
  // did not write it
  __shared__ int2 ent[CPG * 27];
  __shared__ int32_t cflag[CPG], clist[CPG], cblk[CPG], ncls_s;
  __shared__ int32_t red[(NT + SMKI_WAVE - 1) / SMKI_WAVE];
  const int32_t t = blockIdx.x;
  if (a.dn_targets) n_targets = min(n_targets, *a.dn_targets);
  if (t >= n_targets || !a.tgt_active[t]) return;
  if (a.abort_word && *a.abort_word) return;   // nothing is written to the map
  const int64_t n_cold = a.dn_targets ? a.map.counts[1] : a.n_cold;
  const int tid = threadIdx.x;
  const int32_t mslot = a.tgt_slot[t];
  int32_t bt[3];
  unlin3(a.tgt_elin[t], a.enb, bt);
  int32_t pt[3];   // target block on the point grid
  for (int q = 0; q < 3; ++q) pt[q] = bt[q] + a.eblo[q] - a.g.blo[q];
  // Thread tid serves voxels tid + i NT, i < VPT (one voxel up to B = 8);
  // its candidates (a fixed order) are kept for one voxel and recomputed
  // per voxel otherwise.
  int pk[MAXC];
  auto candidates = [&](int vox) {
    const int vv[3] = {vox / (B * B), (vox / B) % B, vox % B};
#pragma unroll
    for (int k = 0; k < MAXC; ++k) pk[k] = merge_candidate<B, R>(vv, k);
  };
  if (VPT == 1) candidates(tid);
  uint32_t upd = 0;   // bit i: voxel tid + i NT received a non-zero sum
  for (int y0 = 0; y0 < a.K; y0 += CPG) {
    const int ny = min(CPG, a.K - y0);
    // Slots of the 27 neighbouring blocks, entry i = class * 27 + neighbour,
    // two per thread and round, their loads in flight together: for every
    // class of the group when that takes one round (issued with the class
    // flags), else only for the classes listed as reaching this block.
    // (compile-time: one round covers a whole group for blocks of 8^3 and more)
    constexpr bool all = 27 * CPG <= 2 * NT;
    auto list_classes = [&]() {   // the classes with contributions, in class order
      if (tid < SMKI_WAVE) {
        const bool f = tid < ny && cflag[tid] != 0;
        const uint64_t m = __ballot(f);
        if (f) clist[__popcll(m & ((1ull << tid) - 1ull))] = tid;
        if (tid == 0) ncls_s = __popcll(m);
      }
    };
    // classes whose rows reach this block, and their class blocks
    if (tid < ny) {
      cflag[tid] = a.contrib[(int64_t)t * a.K + y0 + tid];
      cblk[tid] = a.map.cslot[(int64_t)mslot * a.K + y0 + tid];
    }
    if constexpr (!all) {
      __syncthreads();
      list_classes();
      __syncthreads();
      if (ncls_s == 0) continue;   // (uniform; nothing below reads this group's tables)
    }
    // lookup i of this round: class yc, neighbour d
    auto lookup = [&](int yc, int d) {
      const int px = pt[0] + d / 9 - 1, py = pt[1] + (d / 3) % 3 - 1, pz = pt[2] + d % 3 - 1;
      if (px >= 0 && py >= 0 && pz >= 0 && px < a.g.nb[0] && py < a.g.nb[1] && pz < a.g.nb[2])
        return a.dense[(((int64_t)px * a.g.nb[1] + py) * a.g.nb[2] + pz) * a.K + y0 + yc];
      return -1;
    };
    auto entry = [&](int32_t sl, int d) {
      int2 e2 = make_int2(0, 0);
      if (sl >= 0) {
        const int4 e = a.sinfo[sl];
        if ((e.z >> (26 - d)) & 1) e2 = make_int2(e.x, ((e.w >> (26 - d)) & 1) ? e.y : -e.y);
      }
      return e2;
    };
    const int nl = all ? ny : ncls_s;
    for (int i0 = tid; i0 < 27 * nl; i0 += 2 * NT) {
      int32_t sl[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int i = i0 + j * NT;
        sl[j] = -1;
        if (i < 27 * nl) {
          if constexpr (all) {   // i = d * ny + class
            const int d = i / ny;
            sl[j] = lookup(i - d * ny, d);
          } else {               // i = listed class * 27 + d
            const int c = i / 27;
            sl[j] = lookup(clist[c], i - 27 * c);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int i = i0 + j * NT;
        if (i >= 27 * nl) continue;
        if constexpr (all) {
          const int d = i / ny, yc = i - d * ny;
          ent[yc * 27 + d] = entry(sl[j], d);
        } else {
          ent[i] = entry(sl[j], i % 27);
        }
      }
    }
    __syncthreads();
    if constexpr (all) {
      list_classes();
      __syncthreads();
    }
    const int ncls = ncls_s;
    for (int ic = 0; ic < ncls; ++ic) {
     const int yc = clist[ic];
     const int2* E = ent + (all ? yc : ic) * 27;
     for (int vi = 0; vi < VPT; ++vi) {
      const int vox = tid + vi * NT;
      if (VPT > 1) candidates(vox);
      // Branch-free over the candidates (up to 27 when 2R > B): every candidate
      // loads (an absent one reads a zero word) and the sum is kept in double;
      // then the later units of multi-unit slots, eight at a time (their masks,
      // then their pieces, each set of loads in flight together).
      float first[MAXC];
      bool more = false;
#pragma unroll
      for (int k = 0; k < MAXC; ++k) {
        const int pkk = pk[k];
        const int2 e = E[pkk >= 0 ? (pkk >> 16) : 13];
        const bool ld = pkk >= 0 && e.y > 0;
        first[k] = part_at<DR3, WIDE>(a.part, ld ? e.x : -1, pkk & 0xffff);
        more = more || (pkk >= 0 && (e.y > 1 || e.y < -1));
      }
      double sd = 0.0;
#pragma unroll
      for (int k = 0; k < MAXC; ++k) sd += (double)first[k];
      if (more) {
        // (up to 27 candidates: a runtime loop, the candidates recomputed, so
        // that this path adds no registers to the common one)
        const int vv[3] = {vox / (B * B), (vox / B) % B, vox % B};
        constexpr int MU = MAXC > 8 ? 1 : MAXC;
#pragma unroll MU
        for (int k = 0; k < MAXC; ++k) {
          const int pkk = MAXC > 8 ? merge_candidate<B, R>(vv, k) : pk[k];
          if (pkk < 0) continue;
          const int ci = pkk >> 16;
          const int2 e = E[ci];
          const int32_t w1 = e.x + abs(e.y);
          for (int32_t w0 = e.x + 1; w0 < w1; w0 += 8) {
            uint32_t mk[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) mk[j] = w0 + j < w1 ? a.umask[w0 + j] : 0u;
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const bool has = (mk[j] >> (26 - ci)) & 1u;
              v[j] = part_at<DR3, WIDE>(a.part, has ? w0 + j : -1, pkk & 0xffff);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) sd += (double)v[j];
          }
        }
      }
      const float sm = (float)sd;
      const int32_t cb = cblk[yc];   // allocated for every class with rows reaching here
      float* dst = a.map.calpha + (int64_t)cb * B3 + vox;
      if (cb >= n_cold) {
        *dst = a.alpha0 + sm;   // class block allocated by this insert: written whole
      } else if (sm != 0.0f) {
        *dst += sm;
      }
      if (sm != 0.0f) upd |= 1u << vi;
     }
    }
    __syncthreads();
  }
  int32_t wsum = __popc(upd);
#pragma unroll
  for (int o = S::RW / 2; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, S::RW);
  if ((tid & (SMKI_WAVE - 1)) == 0) red[tid / SMKI_WAVE] = wsum;
  __syncthreads();
  if (tid == 0) {
    int32_t tot = 0;
    for (int i = 0; i < (NT + SMKI_WAVE - 1) / SMKI_WAVE; ++i) tot += red[i];
    atomicAdd(&a.stats[(blockIdx.x % SMKI_STAT_COPIES) * 4], (unsigned long long)tot);
  }
}

// (target, class) pairs that receive rows: from each slot's non-zero pieces (or
// the slot's own block for the counting model); idempotent flag stores.  One
// thread per slot: its block's coordinates once, then the targets of its
// pieces (their lookups in flight together).
__global__ void k_contrib(SplatArgs a, int32_t own_block_only, int32_t* __restrict__ contrib) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (a.dn_slots ? min(a.n_slots, *a.dn_slots) : a.n_slots)) return;
  if (a.abort_word && *a.abort_word) return;
  const uint32_t mk = own_block_only ? (1u << 13) : (uint32_t)a.sinfo[s].z;
  if (mk == 0) return;
  const int32_t plane_lin = a.slot_lin[s];
  const int32_t nb = (int32_t)a.g.n_blocks, y = plane_lin / nb;
  int32_t pb[3];
  unlin3(plane_lin - y * nb, a.g.nb, pb);
  const int32_t e0 = ((pb[0] + a.g.blo[0] - a.eblo[0]) * a.enb[1] + (pb[1] + a.g.blo[1] - a.eblo[1])) *
                         a.enb[2] + (pb[2] + a.g.blo[2] - a.eblo[2]);
  int32_t tt[27];
#pragma unroll
  for (int p = 0; p < 27; ++p) {
    const int dx = p / 9 - 1, dy = (p / 3) % 3 - 1, dz = p % 3 - 1;
    tt[p] = ((mk >> p) & 1u) ? a.ext2t[e0 + (dx * a.enb[1] + dy) * a.enb[2] + dz] : -1;
  }
#pragma unroll
  for (int p = 0; p < 27; ++p) {
    if (tt[p] < 0) continue;
    contrib[(int64_t)tt[p] * a.K + y] = 1;
    a.tgt_active[tt[p]] = 1;   // some row reaches the block
  }
}

// Per target: for each class, whether it needs a class block (rows reach the
// block and it has none yet) as need = 1 + its rank among the target's classes
// that do (0: no), and the target's number of them in need_t, whose exclusive
// scan places the target's class blocks.  G lanes per target (G >= K, a power
// of two up to 64; the ranks from a wave ballot), else one thread per target.
// (dnt: the device count of targets, n_targets then a capacity whose tail is
// written 0 for the scan that follows)
template <int G>
__global__ void k_need(MapDev m, int32_t n_targets, const int32_t* __restrict__ contrib,
                       const int32_t* __restrict__ is_new, const int32_t* __restrict__ tgt_slot,
                       int32_t* __restrict__ need, int32_t* __restrict__ need_t,
                       const int32_t* __restrict__ dnt) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t t = (int32_t)(gi / G), k = (int32_t)(gi % G);
  const bool in = t < n_targets;                      // (uniform per group of G lanes)
  const bool live = in && (!dnt || t < *dnt);
  const bool fresh = live && is_new[t] != 0;
  const int64_t base = (int64_t)t * m.K;
  if (G == 1) {
    if (!in) return;
    int32_t r = 0;
    for (int32_t c = 0; c < m.K; ++c) {
      int32_t v = 0;
      if (live && contrib[base + c])
        v = (fresh || m.cslot[(int64_t)tgt_slot[t] * m.K + c] < 0) ? 1 : 0;
      need[base + c] = v ? r + 1 : 0;
      r += v;
    }
    need_t[t] = r;
    return;
  }
  bool v = false;
  if (live && k < m.K && contrib[base + k])
    v = fresh || m.cslot[(int64_t)tgt_slot[t] * m.K + k] < 0;
  const int lane = threadIdx.x & (SMKI_WAVE - 1);
  const uint64_t grp = (G == SMKI_WAVE ? ~0ull : ((1ull << G) - 1ull)) << (lane & ~(G - 1));
  const uint64_t mk = __ballot(v) & grp;
  if (!in) return;
  if (k < m.K) need[base + k] = v ? __popcll(mk & ((1ull << lane) - 1ull)) + 1 : 0;
  if (k == 0) need_t[t] = __popcll(mk);
}

// map-slot lookup of the active targets; new blocks are marked for allocation
__global__ void k_map_lookup(MapDev m, SplatArgs a, int32_t n_targets,
                             int32_t* __restrict__ tgt_slot, int32_t* __restrict__ is_new) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_targets) return;
  if ((a.dn_targets && t >= *a.dn_targets) || !a.tgt_active[t]) {
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

// Allocation, one thread per (target, class): a new target block takes map
// slot n_old + its rank (the class-0 thread records its key and inserts it in
// the hash), and its class slots start empty; a (target, class) pair that
// needs a class block takes class block n_cold + cpos[t] + its rank among the
// target's (cpos: the exclusive scan of the per-target counts).
__global__ void k_assign(MapDev m, SplatArgs a, int32_t n_targets,
                         const int32_t* __restrict__ is_new, const int32_t* __restrict__ rank,
                         int64_t n_old, int32_t* __restrict__ tgt_slot,
                         const int32_t* __restrict__ need, const int32_t* __restrict__ cpos,
                         int64_t n_cold, uint32_t* __restrict__ err,
                         const int32_t* __restrict__ cnt, int32_t* __restrict__ cnt_copy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a.dn_targets) n_targets = min(n_targets, *a.dn_targets);
  if (i >= (int64_t)n_targets * m.K) return;
  if (a.abort_word && *a.abort_word) return;   // nothing is written to the map
  if (cnt && i == 0) {   // an ordinary insert: the map's counts after it, on the device
    m.counts[0] = n_old + cnt[0];
    m.counts[1] = n_cold + cnt[1];
    cnt_copy[0] = cnt[0];
    cnt_copy[1] = cnt[1];
  }
  if (a.dn_targets) {   // the map's counts before this insert, from the device
    n_old = m.counts[0];
    n_cold = m.counts[1];
  }
  const int32_t t = (int32_t)(i / m.K), k = (int32_t)(i % m.K);
  const bool fresh = is_new[t] != 0;
  const int32_t slot = fresh ? (int32_t)(n_old + rank[t]) : tgt_slot[t];
  const int32_t nd = need[i];   // 1 + rank among the target's new class blocks, 0: none
  if (fresh || nd)
    m.cslot[(int64_t)slot * m.K + k] = nd ? (int32_t)(n_cold + cpos[t] + nd - 1) : -1;
  if (!fresh || k != 0) return;
  int32_t bt[3];
  unlin3(a.tgt_elin[t], a.enb, bt);
  const uint64_t key = smki_block_key(bt[0] + a.eblo[0], bt[1] + a.eblo[1], bt[2] + a.eblo[2]);
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

template <int B, int R, int NSV>
hipError_t launch_splat_ns(const SplatArgs& a, int64_t n_units, int ns, hipStream_t st) {
  if constexpr (NSV >= Steps<R>::NSMIN) {
    if (ns == NSV) {
      const dim3 grid((unsigned)n_units), block(SMKI_WAVE);
      if constexpr (NSV == 1) {
        if (a.noff <= 32) {   // two rows per step
          if (a.wts)
            hipLaunchKernelGGL((k_splat<B, R, 1, true, 2>), grid, block, 0, st, a);
          else
            hipLaunchKernelGGL((k_splat<B, R, 1, false, 2>), grid, block, 0, st, a);
          return hipGetLastError();
        }
      }
      if (a.wts)
        hipLaunchKernelGGL((k_splat<B, R, NSV, true, 1>), grid, block, 0, st, a);
      else
        hipLaunchKernelGGL((k_splat<B, R, NSV, false, 1>), grid, block, 0, st, a);
      return hipGetLastError();
    }
    return launch_splat_ns<B, R, NSV - 1>(a, n_units, ns, st);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int B, int R>
hipError_t launch_splat_br(const SplatArgs& a, int64_t n_units, int32_t n_targets, bool merge,
                           hipStream_t st) {
  if (!merge) {
    if (n_units > 0)
      return launch_splat_ns<B, R, Steps<R>::NS>(a, n_units, (a.noff + SMKI_WAVE - 1) / SMKI_WAVE,
                                                 st);
  } else {
    if (n_targets > 0) {
      constexpr int64_t DR3 = (int64_t)(B + 2 * R) * (B + 2 * R) * (B + 2 * R);
      if (!a.wide && a.part_elems * sizeof(float) <= (int64_t(1) << 32) &&
          (a.part_elems - SMKI_PART_HEAD) / DR3 < (int64_t(1) << 24))
        hipLaunchKernelGGL((k_merge<B, R, false>), dim3((unsigned)n_targets),
                           dim3(MergeShape<B, R>::NT), 0, st, a, n_targets);
      else
        hipLaunchKernelGGL((k_merge<B, R, true>), dim3((unsigned)n_targets),
                           dim3(MergeShape<B, R>::NT), 0, st, a, n_targets);
    }
  }
  return hipGetLastError();
}

// reach R <= B (a row's region covers its own block and the 26 around it)
template <int B>
hipError_t launch_splat_b(const SplatArgs& a, int64_t n_units, int32_t n_targets, bool merge,
                          hipStream_t st) {
  if (a.R > B) return hipErrorInvalidValue;
  switch (a.R) {
    case 0: return launch_splat_br<B, 0>(a, n_units, n_targets, merge, st);
    case 1: return launch_splat_br<B, (B >= 1 ? 1 : 0)>(a, n_units, n_targets, merge, st);
    case 2: return launch_splat_br<B, (B >= 2 ? 2 : 0)>(a, n_units, n_targets, merge, st);
    case 3: return launch_splat_br<B, (B >= 3 ? 3 : 0)>(a, n_units, n_targets, merge, st);
    case 4: return launch_splat_br<B, (B >= 4 ? 4 : 0)>(a, n_units, n_targets, merge, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_splat_any(const SplatArgs& a, int64_t n_units, int32_t n_targets, bool merge,
                            hipStream_t st) {
  static const int kMaxOff[SMKI_MAX_REACH + 1] = {Steps<0>::MAXOFF, Steps<1>::MAXOFF,
                                                  Steps<2>::MAXOFF, Steps<3>::MAXOFF,
                                                  Steps<4>::MAXOFF};
  if (a.R < 0 || a.R > SMKI_MAX_REACH || a.noff < 1 || a.noff > kMaxOff[a.R])
    return hipErrorInvalidValue;
  switch (a.g.B) {
    case 2: return launch_splat_b<2>(a, n_units, n_targets, merge, st);
    case 4: return launch_splat_b<4>(a, n_units, n_targets, merge, st);
    case 8: return launch_splat_b<8>(a, n_units, n_targets, merge, st);
    case 16: return launch_splat_b<16>(a, n_units, n_targets, merge, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_mark_targets(const int32_t* slot_lin, const int32_t* d_nslots, int32_t max_slots,
                               const BucketGeom& g, const int32_t eblo[3], const int32_t enb[3],
                               int32_t DB, int32_t* mark, hipStream_t st) {
  if (max_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_targets, dim3(std::min<unsigned>(nblk(max_slots, 256), kSlotGrid)),
                     dim3(256), 0, st, slot_lin,
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

hipError_t launch_slot_units(const int32_t* head, const int32_t* d_nslots, int32_t max_slots,
                             int32_t chunk, int32_t* nunits, hipStream_t st,
                             const int32_t* slot_lin, int64_t n_blocks, int32_t* cfirst) {
  if (max_slots <= 0) return hipSuccess;
  if (chunk <= 0 || n_blocks <= 0 || (cfirst && !slot_lin)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_slot_units, dim3(std::min<unsigned>(nblk(max_slots, 256), kSlotGrid)),
                     dim3(256), 0, st, head, d_nslots, max_slots, chunk, nunits, slot_lin,
                     n_blocks, cfirst);
  return hipGetLastError();
}

hipError_t launch_unit_table(const int32_t* nunits, const int32_t* ustart, const int32_t* head,
                             const int32_t* slot_lin, int64_t n_blocks, int32_t chunk,
                             int32_t max_slots, const int32_t* d_nslots, const int32_t* d_nunits,
                             int4* units, int32_t* order, hipStream_t st, int32_t cap_units) {
  if (max_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_table,
                     dim3(std::min<unsigned>(nblk((int64_t)max_slots * 8, 256), 8 * kSlotGrid)),
                     dim3(256), 0, st,
                     nunits, ustart, head, slot_lin, n_blocks, chunk, max_slots, d_nslots, d_nunits,
                     units, order, cap_units);
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

hipError_t launch_assign(const MapDev& m, const SplatArgs& a, int32_t n_targets,
                         const int32_t* is_new, const int32_t* new_rank, int64_t n_old,
                         int32_t* tgt_slot, const int32_t* need, const int32_t* cpos,
                         int64_t n_cold, uint32_t* err, hipStream_t st, const int32_t* cnt,
                         int32_t* cnt_copy) {
  const int64_t n = (int64_t)n_targets * m.K;
  if (n <= 0)
    return cnt ? launch_commit_counts(cnt, m.counts, n_old, n_cold, cnt_copy, st) : hipSuccess;
  hipLaunchKernelGGL(k_assign, dim3(nblk(n, 256)), dim3(256), 0, st, m, a, n_targets, is_new,
                     new_rank, n_old, tgt_slot, need, cpos, n_cold, err, cnt, cnt_copy);
  return hipGetLastError();
}

hipError_t launch_after_splat(const SplatArgs& a, int32_t* clr, int64_t nclear,
                              const int32_t* mark, const int32_t* mpos, int64_t n_ext,
                              int32_t* tgt_elin, int32_t* ext2t, hipStream_t st) {
  const int64_t gc = std::min<int64_t>(nblk(nclear, 256), 2048);
  const int64_t gl = n_ext > 0 ? nblk(n_ext, 256) : 0;
  const int64_t gs = a.n_slots > 0 ? nblk((int64_t)a.n_slots * 8, 256) : 0;
  hipLaunchKernelGGL(k_after_splat, dim3((unsigned)(gc + gl + gs)), dim3(256), 0, st, a, clr,
                     nclear, gc, mark, mpos, n_ext, gl, tgt_elin, ext2t);
  return hipGetLastError();
}

hipError_t launch_slot_info(const SplatArgs& a, hipStream_t st) {
  if (a.n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_info, dim3(nblk((int64_t)a.n_slots * 8, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_contrib(const SplatArgs& a, bool own_block_only, int32_t* contrib,
                          hipStream_t st) {
  if (a.n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_contrib, dim3(nblk(a.n_slots, 256)), dim3(256), 0, st, a,
                     own_block_only ? 1 : 0, contrib);
  return hipGetLastError();
}

hipError_t launch_need(const MapDev& m, int32_t n_targets, const int32_t* contrib,
                       const int32_t* is_new, const int32_t* tgt_slot, int32_t* need,
                       int32_t* need_t, hipStream_t st, const int32_t* dn_targets) {
  if (n_targets <= 0 || m.K <= 0) return hipSuccess;
  if (m.K <= 32)
    hipLaunchKernelGGL(k_need<32>, dim3(nblk((int64_t)n_targets * 32, 256)), dim3(256), 0, st, m,
                       n_targets, contrib, is_new, tgt_slot, need, need_t, dn_targets);
  else if (m.K <= 64)
    hipLaunchKernelGGL(k_need<64>, dim3(nblk((int64_t)n_targets * 64, 256)), dim3(256), 0, st, m,
                       n_targets, contrib, is_new, tgt_slot, need, need_t, dn_targets);
  else
    hipLaunchKernelGGL(k_need<1>, dim3(nblk(n_targets, 256)), dim3(256), 0, st, m, n_targets,
                       contrib, is_new, tgt_slot, need, need_t, dn_targets);
  return hipGetLastError();
}

