// Stable least-significant-digit radix sort of (key, u32 value) pairs.
//
// One pass per digit of up to 8 bits: (1) per-tile digit histograms in LDS,
// (2) an exclusive scan of the digit-major histogram table, (3) a stable
// scatter in which each element's rank among equal digits inside its tile is
// found with wave ballots (the peers of a lane are the lanes whose digit
// agrees on every bit), then combined across the tile's waves and rounds in
// element order.  Integer work only: bit-exact and run-to-run deterministic.
#include "smki_internal.h"

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / SMKI_WAVE;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;  // 4096 elements per tile
constexpr int RS_BINS = 256;

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
  return (uint32_t)(key >> shift) & mask;
}

template <typename K>
__global__ void __launch_bounds__(RS_THREADS) k_hist(const K* __restrict__ keys, int64_t n,
                                                     int shift, uint32_t mask, int64_t ntiles,
                                                     uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[RS_BINS];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t i = base + (int64_t)r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[digit_of(keys[i], shift, mask)], 1u);
  }
  __syncthreads();
  // digit-major layout: all tiles of digit 0, then digit 1, ...
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile (RS_TILE elements, one workgroup):
//   1. the tile's digit counts come from the scanned histogram table (entry
//      (digit, tile) minus the next entry), their exclusive scan gives each
//      digit's first index inside the tile, and the table entry itself the
//      digit's first global position;
//   2. every thread loads its RS_ROUNDS elements, and the rounds rank them in
//      element order (wave ballots over the digit bits, per-wave counts in LDS);
//   3. the elements are placed in LDS in digit order, then written out by
//      consecutive threads, so the stores of each digit's run are contiguous.
// pl.rec_in (last pass only, optional): also gather the records by value.
template <typename K>
__global__ void __launch_bounds__(RS_THREADS) k_scatter(const K* __restrict__ keys,
                                                        const uint32_t* __restrict__ vals,
                                                        K* __restrict__ okeys,
                                                        uint32_t* __restrict__ ovals, int64_t n,
                                                        int shift, uint32_t mask, int64_t ntiles,
                                                        const uint32_t* __restrict__ offs,
                                                        SortPayload pl) {
  __shared__ uint32_t gbase[RS_BINS];    // first global position of the tile's digit-d elements
  __shared__ uint32_t lstart[RS_BINS];   // first index of digit d inside the tile
  __shared__ uint32_t run_of[RS_BINS];   // digit-d elements ranked so far
  __shared__ uint32_t wcnt[2][RS_WAVES][RS_BINS];
  __shared__ uint32_t wsum[RS_WAVES];
  __shared__ K skey[RS_TILE];
  __shared__ uint32_t sval[RS_TILE];
  const int tid = threadIdx.x;
  const int lane = tid & (SMKI_WAVE - 1);
  const int w = tid / SMKI_WAVE;
  const int64_t tile_base = (int64_t)blockIdx.x * RS_TILE;
  // 1. digit counts of the tile and their exclusive scan (bin tid)
  {
    const int64_t e = (int64_t)tid * ntiles + blockIdx.x;
    const uint32_t g0 = offs[e];
    const uint32_t g1 = e + 1 < (int64_t)RS_BINS * ntiles ? offs[e + 1] : (uint32_t)n;
    const uint32_t c = g1 - g0;
    gbase[tid] = g0;
    uint32_t inc = c;
#pragma unroll
    for (int o = 1; o < SMKI_WAVE; o <<= 1) {
      const uint32_t u = __shfl_up(inc, o, SMKI_WAVE);
      if (lane >= o) inc += u;
    }
    if (lane == SMKI_WAVE - 1) wsum[w] = inc;
    run_of[tid] = 0;
#pragma unroll
    for (int q = 0; q < RS_WAVES; ++q) {
      wcnt[0][q][tid] = 0;
      wcnt[1][q][tid] = 0;
    }
    __syncthreads();
    uint32_t pre = 0;
    for (int q = 0; q < w; ++q) pre += wsum[q];
    lstart[tid] = pre + inc - c;
  }
  // 2. load and rank
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (SMKI_WAVE - lane));
  K key[RS_ROUNDS];
  uint32_t val[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = tile_base + (int64_t)r * RS_THREADS + tid;
    key[r] = i < n ? keys[i] : (K)0;
    val[r] = i < n ? vals[i] : 0u;
  }
  __syncthreads();
  uint32_t lidx[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int b = r & 1;
    const bool valid = tile_base + (int64_t)r * RS_THREADS + tid < n;
    const uint32_t d = digit_of(key[r], shift, mask);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit_i = 0; bit_i < 8; ++bit_i) {
      const bool bit = (d >> bit_i) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    const bool leader = valid && ((peers & lt_mask) == 0);
    if (leader) wcnt[b][w][d] = cnt;
    __syncthreads();
    lidx[r] = 0;
    if (valid) {
      uint32_t pre = lstart[d] + run_of[d];
      for (int q = 0; q < w; ++q) pre += wcnt[b][q][d];
      lidx[r] = pre + rank;
    }
    __syncthreads();
    // bin tid: advance past this round's elements, clear this round's counts
    uint32_t add = 0;
#pragma unroll
    for (int q = 0; q < RS_WAVES; ++q) {
      add += wcnt[b][q][tid];
      wcnt[b][q][tid] = 0;
    }
    run_of[tid] += add;
  }
  // 3. place in digit order, then write out contiguously
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    if (tile_base + (int64_t)r * RS_THREADS + tid < n) {
      skey[lidx[r]] = key[r];
      sval[lidx[r]] = val[r];
    }
  }
  __syncthreads();
  const int tile_n = (int)min((int64_t)RS_TILE, n - tile_base);
  for (int j = tid; j < tile_n; j += RS_THREADS) {
    const K k = skey[j];
    const uint32_t v = sval[j];
    const uint32_t d = digit_of(k, shift, mask);
    const uint32_t pos = gbase[d] + ((uint32_t)j - lstart[d]);
    okeys[pos] = k;
    ovals[pos] = v;
    if (pl.rec_in) {
      pl.rec_out[pos] = pl.rec_in[v];
      if (pl.w_in) pl.w_out[pos] = pl.w_in[v];
    }
  }
}

template <typename K>
hipError_t sort_impl(K* keys, uint32_t* vals, K* akeys, uint32_t* avals, int64_t n, int bits,
                     void* tmp, hipStream_t st, const SortPayload* pl) {
  if (n <= 1 || bits <= 0) return hipSuccess;
  const int64_t ntiles = ceil_div_i64(n, RS_TILE);
  uint32_t* hist = (uint32_t*)tmp;
  void* scan_tmp = (void*)(hist + RS_BINS * ntiles + 64);
  const int passes = (bits + 7) / 8;
  const int dbits = (bits + passes - 1) / passes;
  const uint32_t mask = (1u << dbits) - 1u;
  K* src_k = keys;
  uint32_t* src_v = vals;
  K* dst_k = akeys;
  uint32_t* dst_v = avals;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * dbits;
    hipLaunchKernelGGL(k_hist<K>, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, st, src_k, n,
                       shift, mask, ntiles, hist);
    hipError_t e = scan_excl_i32((const int32_t*)hist, (int32_t*)hist, RS_BINS * ntiles,
                                 (int32_t*)nullptr, scan_tmp, st);
    if (e != hipSuccess) return e;
    const SortPayload none{};
    hipLaunchKernelGGL(k_scatter<K>, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, st, src_k,
                       src_v, dst_k, dst_v, n, shift, mask, ntiles, (const uint32_t*)hist,
                       (p == passes - 1 && pl) ? *pl : none);
    K* tk = src_k; src_k = dst_k; dst_k = tk;
    uint32_t* tv = src_v; src_v = dst_v; dst_v = tv;
  }
  if (src_k != keys) {
    hipError_t e = hipMemcpyAsync(keys, src_k, sizeof(K) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vals, src_v, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace

size_t radix_tmp_bytes(int64_t n) {
  const int64_t ntiles = ceil_div_i64(n > 0 ? n : 1, RS_TILE);
  return sizeof(uint32_t) * (RS_BINS * ntiles + 64) + scan_tmp_bytes(RS_BINS * ntiles) + 256;
}

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* ak, uint32_t* av, int64_t n,
                          int bits, void* tmp, hipStream_t st, const SortPayload* pl) {
  return sort_impl<uint32_t>(keys, vals, ak, av, n, bits, tmp, st, pl);
}

hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* ak, uint32_t* av, int64_t n,
                          int bits, void* tmp, hipStream_t st, const SortPayload* pl) {
  return sort_impl<uint64_t>(keys, vals, ak, av, n, bits, tmp, st, pl);
}
