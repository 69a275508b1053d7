// The semantic counting sensor model (S-CSM, Eq. (2) of Gan et al., arXiv
// 1909.04631): a voxel's concentration is the prior plus the number of
// training rows of each class that fall inside it,
//
//   alpha_v^k = alpha0 + #{ rows t in voxel v with y_t = k }.
//
// Rows arrive sorted by (class, block, voxel cell), so the rows of one
// (class, voxel) are a run of equal keys.  The last row of each run adds the
// run's length to its voxel: every (voxel, class) is written by exactly one
// thread, and the counts are integers, so the result is exact and order-free.
// With soft measurements (Sec. VI) a row counts its class weight instead of 1.
#include "smki_gather.h"

namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)ceil_div_i64(n > 0 ? n : 1, t); }

// One thread per row; the last row of each run of equal keys (one class in one
// voxel: keys are sorted by (class, block, voxel)) finds the run's first row by
// binary search and adds the run length to that voxel's class.
// Words of voxel bits per target block.
constexpr int vbit_words(int B) { return (B * B * B + 31) / 32; }

template <typename KeyT, int B>
__global__ void k_csm_counts(SplatArgs a, const KeyT* __restrict__ keys, int64_t n,
                             uint32_t* __restrict__ vbits) {
  constexpr int B3 = B * B * B;
  constexpr int L3 = B == 1 ? 0 : B == 2 ? 3 : B == 4 ? 6 : B == 8 ? 9 : B == 16 ? 12 : 15;   // cell bits
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const KeyT k = keys[i];
  if (i + 1 < n && keys[i + 1] == k) return;   // not the last row of its run
  int64_t lo = 0, hi = i;                      // first row with this key
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < k) lo = mid + 1; else hi = mid;
  }
  const int32_t c = (int32_t)((uint64_t)k & (uint64_t)(B3 - 1));
  const int64_t plane_lin = (int64_t)((uint64_t)k >> L3);
  const int32_t y = (int32_t)(plane_lin / a.g.n_blocks);
  const int64_t blin = plane_lin % a.g.n_blocks;
  const int32_t pz = (int32_t)(blin % a.g.nb[2]);
  const int32_t py = (int32_t)((blin / a.g.nb[2]) % a.g.nb[1]);
  const int32_t px = (int32_t)(blin / ((int64_t)a.g.nb[2] * a.g.nb[1]));
  const int64_t e = ((int64_t)(px + a.g.blo[0] - a.eblo[0]) * a.enb[1] +
                     (py + a.g.blo[1] - a.eblo[1])) * a.enb[2] + (pz + a.g.blo[2] - a.eblo[2]);
  const int32_t t = a.ext2t[e];
  const int32_t mslot = a.tgt_slot[t];
  const int32_t cb = a.map.cslot[(int64_t)mslot * a.K + y];   // allocated: the class has rows here
  float add = (float)(i - lo + 1);
  if (a.wts) {   // soft measurements: the run's weights, summed in row order in double
    double sw = 0.0;
    for (int64_t r = lo; r <= i; ++r) sw += (double)a.wts[a.perm ? a.perm[r] : r];
    add = (float)sw;
  }
  a.map.calpha[(int64_t)cb * B3 + c] += add;
  atomicOr(&vbits[(int64_t)t * vbit_words(B) + (c >> 5)], 1u << (c & 31));
}

// voxels with at least one row: popcount of the per-target voxel bits
__global__ void k_csm_voxels(const uint32_t* __restrict__ vbits, int64_t nwords,
                             unsigned long long* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = i < nwords ? __popc(vbits[i]) : 0;
  int v = c;
#pragma unroll
  for (int o = SMKI_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, SMKI_WAVE);
  if ((threadIdx.x & (SMKI_WAVE - 1)) == 0 && v)
    atomicAdd(&out[(blockIdx.x % SMKI_STAT_COPIES) * 4], (unsigned long long)v);
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_csm_counts(const SplatArgs& a, const void* keys, bool wide_keys, int64_t n,
                             uint32_t* vbits, int64_t n_targets, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(nblk(n, 256)), block(256);
#define SMKI_CSM_CASE(BB)                                                                    \
  case BB:                                                                                  \
    if (wide_keys)                                                                          \
      hipLaunchKernelGGL((k_csm_counts<uint64_t, BB>), grid, block, 0, st, a,               \
                         (const uint64_t*)keys, n, vbits);                                  \
    else                                                                                    \
      hipLaunchKernelGGL((k_csm_counts<uint32_t, BB>), grid, block, 0, st, a,               \
                         (const uint32_t*)keys, n, vbits);                                  \
    break;
  switch (a.g.B) {
    SMKI_CSM_CASE(1) SMKI_CSM_CASE(2) SMKI_CSM_CASE(4) SMKI_CSM_CASE(8) SMKI_CSM_CASE(16)
    SMKI_CSM_CASE(32)
    default: return hipErrorInvalidValue;
  }
#undef SMKI_CSM_CASE
  const int64_t nwords = n_targets * (int64_t)((a.g.B * a.g.B * a.g.B + 31) / 32);
  hipLaunchKernelGGL(k_csm_voxels, dim3(nblk(nwords, 256)), dim3(256), 0, st, vbits, nwords,
                     &a.stats[0]);
  return hipGetLastError();
}

hipError_t launch_fill_calpha0(const MapDev& m, int64_t c0, int64_t nc, hipStream_t st) {
  const int64_t per = (int64_t)m.B * m.B * m.B;
  const int64_t n = nc * per;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n, 256)), dim3(256), 0, st, m.calpha + c0 * per, n,
                     m.alpha0);
  return hipGetLastError();
}
