// The semantic counting sensor model (S-CSM, Eq. (2) of Gan et al., arXiv
// 1909.04631): a voxel's concentration is the prior plus the number of
// training rows of each class that fall inside it,
//
//   alpha_v^k = alpha0 + #{ rows t in voxel v with y_t = k }.
//
// Rows arrive bucketed by (class, block, voxel cell), so the rows of one
// (class, voxel) are a run of equal cells inside their slot.  One wavefront per
// slot finds the runs and adds each run's length to its voxel: every
// (voxel, class) is written by exactly one lane, and the counts are integers,
// so the result is exact and order-free.
#include "smki_gather.h"

namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)ceil_div_i64(n > 0 ? n : 1, t); }

__device__ __forceinline__ int32_t cell_of_row(const float4* __restrict__ pts, int32_t r) {
  return __float_as_int(pts[r].w) >> 3;
}

template <int B>
__global__ void __launch_bounds__(SMKI_WAVE) k_csm_counts(SplatArgs a, uint32_t* __restrict__ vbits) {
  constexpr int B3 = B * B * B;
  const int32_t s = blockIdx.x;
  if (s >= a.n_slots) return;
  const int32_t r0 = a.head[s], r1 = a.head[s + 1];
  const int32_t plane_lin = a.slot_lin[s];
  const int32_t y = (int32_t)(plane_lin / a.g.n_blocks);
  const int64_t blin = plane_lin % a.g.n_blocks;
  const int32_t pz = (int32_t)(blin % a.g.nb[2]);
  const int32_t py = (int32_t)((blin / a.g.nb[2]) % a.g.nb[1]);
  const int32_t px = (int32_t)(blin / ((int64_t)a.g.nb[2] * a.g.nb[1]));
  const int64_t e = ((int64_t)(px + a.g.blo[0] - a.eblo[0]) * a.enb[1] +
                     (py + a.g.blo[1] - a.eblo[1])) * a.enb[2] + (pz + a.g.blo[2] - a.eblo[2]);
  const int32_t t = a.ext2t[e];
  const int32_t mslot = a.tgt_slot[t];
  float* A = a.alpha + ((int64_t)mslot * a.K + y) * B3;
  const float4* __restrict__ pts = a.pts;
  for (int32_t r = r0 + (int32_t)threadIdx.x; r < r1; r += SMKI_WAVE) {
    const int32_t c = cell_of_row(pts, r);
    if (r > r0 && cell_of_row(pts, r - 1) == c) continue;   // not the first row of its run
    int32_t lo = r, hi = r1 - 1;                             // last row of the run
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (cell_of_row(pts, mid) == c) lo = mid; else hi = mid - 1;
    }
    A[c] += (float)(lo - r + 1);
    atomicOr(&vbits[(int64_t)t * (B3 / 32) + (c >> 5)], 1u << (c & 31));
  }
}

// voxels with at least one row: popcount of the per-target voxel bits
__global__ void k_csm_voxels(const uint32_t* __restrict__ vbits, int64_t nwords,
                             unsigned long long* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = i < nwords ? __popc(vbits[i]) : 0;
  int v = c;
#pragma unroll
  for (int o = SMKI_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SMKI_WAVE);
  if ((threadIdx.x & (SMKI_WAVE - 1)) == 0 && v) atomicAdd(out, (unsigned long long)v);
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_csm_counts(const SplatArgs& a, uint32_t* vbits, int64_t n_targets,
                             hipStream_t st) {
  if (a.n_slots <= 0) return hipSuccess;
  switch (a.g.B) {
    case 4:
      hipLaunchKernelGGL(k_csm_counts<4>, dim3((unsigned)a.n_slots), dim3(SMKI_WAVE), 0, st, a,
                         vbits);
      break;
    case 8:
      hipLaunchKernelGGL(k_csm_counts<8>, dim3((unsigned)a.n_slots), dim3(SMKI_WAVE), 0, st, a,
                         vbits);
      break;
    default:
      return hipErrorInvalidValue;
  }
  const int64_t nwords = n_targets * (int64_t)(a.g.B * a.g.B * a.g.B / 32);
  hipLaunchKernelGGL(k_csm_voxels, dim3(nblk(nwords, 256)), dim3(256), 0, st, vbits, nwords,
                     &a.stats[0]);
  return hipGetLastError();
}

hipError_t launch_fill_alpha0(const MapDev& m, int64_t slot0, int64_t nslots, hipStream_t st) {
  const int64_t per = (int64_t)m.K * m.B * m.B * m.B;
  const int64_t n = nslots * per;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n, 256)), dim3(256), 0, st, m.alpha + slot0 * per, n,
                     m.alpha0);
  return hipGetLastError();
}
