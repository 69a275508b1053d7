// Device-wide exclusive prefix sum (reduce, scan the tile sums, scan again).
// Deterministic: integer sums only.
#include <algorithm>

#include "smki_internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & (SMKI_WAVE - 1);
#pragma unroll
  for (int o = 1; o < SMKI_WAVE; o <<= 1) {
    T u = __shfl_up(v, o, SMKI_WAVE);
    if (lane >= o) v += u;
  }
  return v;
}

// exclusive scan of one value per thread across the workgroup; returns the
// exclusive prefix, *block_total the sum.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* block_total) {
  __shared__ T wsum[SCAN_THREADS / SMKI_WAVE];
  const int lane = threadIdx.x & (SMKI_WAVE - 1);
  const int w = threadIdx.x / SMKI_WAVE;
  T inc = wave_incl_scan(v);
  if (lane == SMKI_WAVE - 1) wsum[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_THREADS / SMKI_WAVE; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *block_total = tot;
  return off + inc - v;
}

// Elements of an array of capacity n whose count (dn, nullable) is read on
// the device: tiles past the count read and write nothing, and add zero.
__device__ __forceinline__ int64_t count_of(int64_t n, const int32_t* dn) {
  return dn ? min(n, (int64_t)max(*dn, 0)) : n;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_sums(const T* __restrict__ in, int64_t n,
                                                            T* __restrict__ sums,
                                                            const int32_t* dn) {
  n = count_of(n, dn);
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) s += in[base + i];
  T tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_scan(const T* in, T* out, int64_t n,
                                                            const T* __restrict__ tile_off,
                                                            T* total, const int32_t* dn) {
  n = count_of(n, dn);
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = (base + i < n) ? in[base + i] : (T)0;
    s += v[i];
  }
  T tot;
  T run = block_excl_scan(s, &tot) + (tile_off ? tile_off[blockIdx.x] : (T)0);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) *total = run;
}

// The same with each tile's offset computed by the workgroup itself as the sum
// of the preceding tile sums (for few tiles: saves the launch that scans them).
template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_scan_direct(const T* in, T* out, int64_t n,
                                                                   const T* __restrict__ sums,
                                                                   T* total, const int32_t* dn) {
  n = count_of(n, dn);
  __shared__ T part[SCAN_THREADS / SMKI_WAVE];
  T pre = 0;
  for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += SCAN_THREADS) pre += sums[i];
#pragma unroll
  for (int o = SMKI_WAVE / 2; o > 0; o >>= 1) pre += __shfl_xor(pre, o, SMKI_WAVE);
  if ((threadIdx.x & (SMKI_WAVE - 1)) == 0) part[threadIdx.x / SMKI_WAVE] = pre;
  __syncthreads();
  T off = 0;
#pragma unroll
  for (int i = 0; i < SCAN_THREADS / SMKI_WAVE; ++i) off += part[i];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = (base + i < n) ? in[base + i] : (T)0;
    s += v[i];
  }
  T tot;
  T run = block_excl_scan(s, &tot) + off;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_THREADS - 1) *total = run;
}

// Two independent scans in the same two launches (each of at most 512 tiles):
// workgroups [0, ta) take the first array's tiles, the rest the second's.
template <typename T>
__device__ __forceinline__ void tile_sum(const T* __restrict__ in, int64_t n, T* __restrict__ sums,
                                         int64_t tile) {
  const int64_t base = tile * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) s += in[base + i];
  T tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) sums[tile] = tot;
}

template <typename T>
__device__ __forceinline__ void tile_scan_direct(const T* in, T* out, int64_t n,
                                                 const T* __restrict__ sums, T* total,
                                                 int64_t tile, int64_t ntiles) {
  __shared__ T part[SCAN_THREADS / SMKI_WAVE];
  T pre = 0;
  for (int64_t i = threadIdx.x; i < tile; i += SCAN_THREADS) pre += sums[i];
#pragma unroll
  for (int o = SMKI_WAVE / 2; o > 0; o >>= 1) pre += __shfl_xor(pre, o, SMKI_WAVE);
  if ((threadIdx.x & (SMKI_WAVE - 1)) == 0) part[threadIdx.x / SMKI_WAVE] = pre;
  __syncthreads();
  T off = 0;
#pragma unroll
  for (int i = 0; i < SCAN_THREADS / SMKI_WAVE; ++i) off += part[i];
  const int64_t base = tile * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = (base + i < n) ? in[base + i] : (T)0;
    s += v[i];
  }
  T tot;
  T run = block_excl_scan(s, &tot) + off;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (total && tile == ntiles - 1 && threadIdx.x == SCAN_THREADS - 1) *total = run;
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_sums_pair(const TA* __restrict__ ina,
                                                                 int64_t na, TA* __restrict__ sa,
                                                                 int64_t ta,
                                                                 const TB* __restrict__ inb,
                                                                 int64_t nb, TB* __restrict__ sb,
                                                                 const int32_t* dnb) {
  if ((int64_t)blockIdx.x < ta)
    tile_sum<TA>(ina, na, sa, blockIdx.x);
  else
    tile_sum<TB>(inb, count_of(nb, dnb), sb, (int64_t)blockIdx.x - ta);
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_scan_direct_pair(
    const TA* ina, TA* outa, int64_t na, const TA* __restrict__ sa, TA* tota, int64_t ta,
    const TB* inb, TB* outb, int64_t nb, const TB* __restrict__ sb, TB* totb, int64_t tb,
    const int32_t* dnb) {
  if ((int64_t)blockIdx.x < ta)
    tile_scan_direct<TA>(ina, outa, na, sa, tota, blockIdx.x, ta);
  else
    tile_scan_direct<TB>(inb, outb, count_of(nb, dnb), sb, totb, (int64_t)blockIdx.x - ta, tb);
}

template <typename T>
__global__ void k_zero_total(T* total) { *total = 0; }

template <typename T>
size_t tmp_elems(int64_t n) {
  size_t e = 0;
  int64_t m = n;
  while (m > SCAN_TILE) {
    m = ceil_div_i64(m, SCAN_TILE);
    e += (size_t)m + 1;
  }
  return e + 1;
}

// dn (device, nullable): the element count, n then being the capacity
template <typename T>
hipError_t scan_impl(const T* in, T* out, int64_t n, T* total, T* tmp, hipStream_t st,
                     const int32_t* dn = nullptr) {
  if (n <= 0) {
    if (total) hipLaunchKernelGGL(k_zero_total<T>, dim3(1), dim3(1), 0, st, total);
    return hipGetLastError();
  }
  const int64_t tiles = ceil_div_i64(n, SCAN_TILE);
  if (tiles == 1) {
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(SCAN_THREADS), 0, st, in, out, n,
                       (const T*)nullptr, total, dn);
    return hipGetLastError();
  }
  T* sums = tmp;
  T* rest = tmp + tiles + 1;
  hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, st, in, n,
                     sums, dn);
  if (tiles <= 512) {   // up to 512 tile sums: every workgroup adds its predecessors' itself
    hipLaunchKernelGGL(k_tile_scan_direct<T>, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, st, in,
                       out, n, (const T*)sums, total, dn);
    return hipGetLastError();
  }
  hipError_t e = scan_impl<T>(sums, sums, tiles, (T*)nullptr, rest, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, st, in, out,
                     n, (const T*)sums, total, dn);
  return hipGetLastError();
}

constexpr int64_t kPairTiles = 512;   // per array, for the two-launch pair scan

template <typename TA, typename TB>
hipError_t scan_pair_impl(const TA* ina, TA* outa, int64_t na, TA* tota, const TB* inb, TB* outb,
                          int64_t nb, TB* totb, void* tmp, hipStream_t st, const int32_t* dnb) {
  const int64_t ta = ceil_div_i64(na, SCAN_TILE), tb = ceil_div_i64(nb, SCAN_TILE);
  if (na <= 0 || nb <= 0 || ta > kPairTiles || tb > kPairTiles) {
    hipError_t e = scan_impl<TA>(ina, outa, na, tota, (TA*)tmp, st);
    if (e != hipSuccess) return e;
    return scan_impl<TB>(inb, outb, nb, totb, (TB*)tmp, st, dnb);
  }
  TA* sa = (TA*)tmp;
  TB* sb = (TB*)((char*)tmp + kPairTiles * sizeof(int64_t));
  hipLaunchKernelGGL((k_tile_sums_pair<TA, TB>), dim3((unsigned)(ta + tb)), dim3(SCAN_THREADS), 0,
                     st, ina, na, sa, ta, inb, nb, sb, dnb);
  hipLaunchKernelGGL((k_tile_scan_direct_pair<TA, TB>), dim3((unsigned)(ta + tb)),
                     dim3(SCAN_THREADS), 0, st, ina, outa, na, (const TA*)sa, tota, ta, inb, outb,
                     nb, (const TB*)sb, totb, tb, dnb);
  return hipGetLastError();
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) {
  return std::max<size_t>(tmp_elems<int64_t>(n), 2 * kPairTiles) * sizeof(int64_t) + 256;
}

hipError_t scan_excl_pair_i64_i32(const int64_t* ina, int64_t* outa, int64_t na, int64_t* tota,
                                  const int32_t* inb, int32_t* outb, int64_t nb, int32_t* totb,
                                  void* tmp, hipStream_t st) {
  return scan_pair_impl<int64_t, int32_t>(ina, outa, na, tota, inb, outb, nb, totb, tmp, st,
                                          nullptr);
}

hipError_t scan_excl_pair_i32(const int32_t* ina, int32_t* outa, int64_t na, int32_t* tota,
                              const int32_t* inb, int32_t* outb, int64_t nb, int32_t* totb,
                              void* tmp, hipStream_t st, const int32_t* dnb) {
  return scan_pair_impl<int32_t, int32_t>(ina, outa, na, tota, inb, outb, nb, totb, tmp, st, dnb);
}

hipError_t scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total, void* tmp,
                         hipStream_t st) {
  return scan_impl<int64_t>(in, out, n, total, (int64_t*)tmp, st);
}

hipError_t scan_excl_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* tmp,
                         hipStream_t st) {
  return scan_impl<int32_t>(in, out, n, total, (int32_t*)tmp, st);
}
