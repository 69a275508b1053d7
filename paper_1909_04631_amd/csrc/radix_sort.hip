// Stable least-significant-digit radix sort of (key, u32 value) pairs.
//
// One pass per digit of up to 9 bits: (1) per-tile digit histograms, (2) per
// digit, an exclusive scan of its tile counts and its total, (3) a stable
// scatter, which adds the totals of the smaller digits itself.  In the
// scatter a wavefront takes 1024 consecutive elements of its tile and groups
// equal digits with wave ballots (the peers of a lane are the lanes whose
// digit agrees on every bit); its running digit counts live in its own LDS
// row, so rounds need no barrier.  Integer work only: bit-exact and
// run-to-run deterministic.
#include "smki_internal.h"

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / SMKI_WAVE;
constexpr int RS_ROUNDS = 16;
constexpr int RS_SPAN = RS_ROUNDS * SMKI_WAVE;   // 1024 consecutive elements per wavefront
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;  // 4096 elements per tile
constexpr int RS_MAXBITS = 9;                   // digits of up to 9 bits
constexpr int RS_MAXBINS = 1 << RS_MAXBITS;

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask) {
  return (uint32_t)(key >> shift) & mask;
}

// Lanes of the wavefront that hold a valid element with digit d (dbits bits).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid, int dbits) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < dbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Element layout of a tile: wavefront w holds elements [w RS_SPAN, (w+1) RS_SPAN),
// round r of it the 64 elements from w RS_SPAN + 64 r, lane i the i-th of them;
// so (wavefront, round, lane) is element order.
__device__ __forceinline__ int64_t elem_index(int64_t tile_base, int w, int r, int lane) {
  return tile_base + (int64_t)w * RS_SPAN + (int64_t)r * SMKI_WAVE + lane;
}

// Per-tile digit counts: every element adds 1 to its digit's counter with an
// LDS atomic (integer counts: the order of the adds does not matter).  Lane l
// uses copy l % NC of the counters, rows padded by one word, so that the lanes
// of one wavefront with equal digits neither hit one address nor one bank;
// the copies are summed at the end.
template <typename K, int NB>
__global__ void __launch_bounds__(RS_THREADS) k_hist(const K* __restrict__ keys, int64_t ncap,
                                                     const int64_t* __restrict__ dn, int shift,
                                                     int dbits, int64_t ntiles,
                                                     uint32_t* __restrict__ hist) {
  const int64_t n = eff_n(ncap, dn);   // tiles past the count contribute zero counts
  constexpr int NC = 16;         // counter copies
  constexpr int STR = NB + 1;    // padded row of one copy
  constexpr int DPT = NB / RS_THREADS;   // digits per thread
  __shared__ uint32_t h[NC * STR];
  const int tid = threadIdx.x, lane = tid & (SMKI_WAVE - 1), w = tid / SMKI_WAVE;
  const uint32_t mask = (1u << dbits) - 1u;
  const int64_t tile_base = (int64_t)blockIdx.x * RS_TILE;
  for (int i = tid; i < NC * STR; i += RS_THREADS) h[i] = 0;
  K key[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = elem_index(tile_base, w, r, lane);
    key[r] = i < n ? keys[i] : (K)0;
  }
  __syncthreads();
  uint32_t* hc = h + (lane % NC) * STR;
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r)
    if (elem_index(tile_base, w, r, lane) < n) atomicAdd(&hc[digit_of(key[r], shift, mask)], 1u);
  __syncthreads();
  // digit-major layout: all tiles of digit 0, then digit 1, ...
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int d = tid * DPT + j;
    if (d > (int)mask) continue;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < NC; ++q) c += h[q * STR + d];
    hist[(int64_t)d * ntiles + blockIdx.x] = c;
  }
}

// Per digit (one workgroup each): exclusive scan, in place, of the digit's
// row of the digit-major table (its count in every tile), and the digit's
// total.
__global__ void __launch_bounds__(RS_THREADS) k_digit_scan(uint32_t* __restrict__ hist,
                                                           int64_t ntiles,
                                                           uint32_t* __restrict__ total) {
  // The digit's row of tile counts, scanned in chunks of RS_THREADS * 4 counts
  // (thread t takes four consecutive ones): per chunk a workgroup scan, carried
  // into the next chunk, whose counts are loaded while this one is scanned.
  constexpr int V = 4, CH = RS_THREADS * V;
  __shared__ uint32_t wsum[2][RS_WAVES];
  const int tid = threadIdx.x, lane = tid & (SMKI_WAVE - 1), w = tid / SMKI_WAVE;
  uint32_t* row = hist + (int64_t)blockIdx.x * ntiles;
  auto load = [&](int64_t c0, uint32_t* v) {
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t i = c0 + (int64_t)tid * V + j;
      v[j] = i < ntiles ? row[i] : 0u;
    }
  };
  uint32_t cur[V], nxt[V];
  load(0, cur);
  uint32_t carry = 0;
  int par = 0;
  for (int64_t c0 = 0; c0 < ntiles; c0 += CH, par ^= 1) {
    load(c0 + CH, nxt);
    const uint32_t s = cur[0] + cur[1] + cur[2] + cur[3];
    uint32_t inc = s;
#pragma unroll
    for (int o = 1; o < SMKI_WAVE; o <<= 1) {
      const uint32_t u = __shfl_up(inc, o, SMKI_WAVE);
      if (lane >= o) inc += u;
    }
    if (lane == SMKI_WAVE - 1) wsum[par][w] = inc;
    __syncthreads();   // (two copies of wsum: a chunk's writes never meet the previous chunk's reads)
    uint32_t run = carry + inc - s;
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < RS_WAVES; ++q) {
      run += q < w ? wsum[par][q] : 0u;
      tot += wsum[par][q];
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t i = c0 + (int64_t)tid * V + j;
      if (i < ntiles) row[i] = run;
      run += cur[j];
    }
    carry += tot;
#pragma unroll
    for (int j = 0; j < V; ++j) cur[j] = nxt[j];
  }
  if (tid == 0) total[blockIdx.x] = carry;
}

// Last pass with records: a thread gathers the records (and weights) of eight
// of the tile's sorted elements before storing any of them.
template <typename K, bool WT>
__device__ __forceinline__ void write_records(const K* skey, const uint32_t* sval,
                                              const uint32_t* gbase, const uint32_t* lstart,
                                              int tile_n, int shift, uint32_t mask,
                                              K* __restrict__ okeys, uint32_t* __restrict__ ovals,
                                              const SortPayload& pl) {
  constexpr int G = 8;
  const int tid = threadIdx.x;
#pragma unroll
  for (int j0 = 0; j0 < RS_TILE; j0 += G * RS_THREADS) {
    // Unconditional: a thread past the tile's end takes its last element again
    // and stores the same values to the same place.
    float rx[G], ry[G], rz[G], rw[G], wv[G];   // (component arrays stay in registers)
    K kk[G];
    uint32_t vv[G], pos[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = min(j0 + g * RS_THREADS + tid, tile_n - 1);
      kk[g] = skey[j];
      vv[g] = sval[j];
      const float4 r = pl.rec_in[vv[g]];
      rx[g] = r.x;
      ry[g] = r.y;
      rz[g] = r.z;
      rw[g] = r.w;
      wv[g] = WT ? pl.w_in[vv[g]] : 0.0f;
      const uint32_t d = digit_of(kk[g], shift, mask);
      pos[g] = gbase[d] + ((uint32_t)j - lstart[d]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      okeys[pos[g]] = kk[g];
      ovals[pos[g]] = vv[g];
      pl.rec_out[pos[g]] = make_float4(rx[g], ry[g], rz[g], rw[g]);
      if (WT) pl.w_out[pos[g]] = wv[g];
    }
  }
}

// Stable scatter of one tile (RS_TILE elements, one workgroup):
//   1. every wavefront loads its span and ranks each element among the equal
//      digits of its span (wave ballots; per-wavefront running counts in LDS,
//      no barrier between rounds);
//   2. per digit, the tile's count and each wavefront's first index inside the
//      tile (exclusive scans over wavefronts, then over digits); the scanned
//      histogram table gives the digit's first global position;
//   3. the elements are placed in LDS in digit order, then written out by
//      consecutive threads, so the stores of each digit's run are contiguous.
// pl.rec_in (last pass only, optional): also gather the records by value.
template <typename K, int NB>
__global__ void __launch_bounds__(RS_THREADS) k_scatter(const K* __restrict__ keys,
                                                        const uint32_t* __restrict__ vals,
                                                        K* __restrict__ okeys,
                                                        uint32_t* __restrict__ ovals, int64_t ncap,
                                                        const int64_t* __restrict__ dn, int shift,
                                                        int dbits, int64_t ntiles,
                                                        const uint32_t* __restrict__ offs,
                                                        const uint32_t* __restrict__ total,
                                                        SortPayload pl, int vals_iota) {
  const int64_t n = eff_n(ncap, dn);
  if ((int64_t)blockIdx.x * RS_TILE >= n) return;   // a tile past the count (capacity launch)
  constexpr int DPT = NB / RS_THREADS;   // digits per thread: tid * DPT + j
  __shared__ uint32_t gbase[NB];    // first global position of the tile's digit-d elements
  __shared__ uint32_t lstart[NB];   // first index of digit d inside the tile
  __shared__ uint32_t wh[RS_WAVES][NB];   // per wavefront: digit counts, then first index
  __shared__ uint32_t wsum[2][RS_WAVES];
  __shared__ K skey[RS_TILE];
  __shared__ uint32_t sval[RS_TILE];
  const int tid = threadIdx.x, lane = tid & (SMKI_WAVE - 1), w = tid / SMKI_WAVE;
  const uint32_t mask = (1u << dbits) - 1u;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (SMKI_WAVE - lane));
  const int64_t tile_base = (int64_t)blockIdx.x * RS_TILE;
  uint32_t in_digit[DPT], dtot[DPT];   // earlier tiles' count of the digit, its total
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int d = tid * DPT + j;
    const bool real = d <= (int)mask;
    in_digit[j] = real ? offs[(int64_t)d * ntiles + blockIdx.x] : 0u;
    dtot[j] = real ? total[d] : 0u;
  }
#pragma unroll
  for (int q = 0; q < RS_WAVES; ++q)
#pragma unroll
    for (int j = 0; j < DPT; ++j) wh[q][tid * DPT + j] = 0;
  K key[RS_ROUNDS];
  uint32_t val[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = elem_index(tile_base, w, r, lane);
    key[r] = i < n ? keys[i] : (K)0;
    val[r] = vals_iota ? (uint32_t)i : (i < n ? vals[i] : 0u);
  }
  __syncthreads();
  // 1. rank inside the wavefront's span
  uint32_t lrank[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const bool valid = elem_index(tile_base, w, r, lane) < n;
    const uint32_t d = digit_of(key[r], shift, mask);
    const uint64_t peers = digit_peers(d, valid, dbits);
    const uint32_t before = wh[w][d];
    lrank[r] = before + (uint32_t)__popcll(peers & lt_mask);
    if (valid && (peers & lt_mask) == 0) wh[w][d] = before + (uint32_t)__popcll(peers);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  __syncthreads();
  // 2. digits of thread tid: the wavefronts' counts, the tile's count and its
  //    first index inside the tile; the digit's first global position (the
  //    totals of the smaller digits plus the digit's count in earlier tiles)
  {
    uint32_t pw[DPT][RS_WAVES], c[DPT];
    uint32_t csum = 0, gsum = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      c[j] = 0;
#pragma unroll
      for (int q = 0; q < RS_WAVES; ++q) {
        pw[j][q] = c[j];
        c[j] += wh[q][tid * DPT + j];
      }
      csum += c[j];
      gsum += dtot[j];
    }
    uint32_t inc = csum, incg = gsum;
#pragma unroll
    for (int o = 1; o < SMKI_WAVE; o <<= 1) {
      const uint32_t u = __shfl_up(inc, o, SMKI_WAVE);
      const uint32_t ug = __shfl_up(incg, o, SMKI_WAVE);
      if (lane >= o) {
        inc += u;
        incg += ug;
      }
    }
    if (lane == SMKI_WAVE - 1) {
      wsum[0][w] = inc;
      wsum[1][w] = incg;
    }
    __syncthreads();
    uint32_t ls = inc - csum, lg = incg - gsum;
    for (int q = 0; q < w; ++q) {
      ls += wsum[0][q];
      lg += wsum[1][q];
    }
    // the digits of thread tid are read and rewritten by thread tid only
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int d = tid * DPT + j;
      lstart[d] = ls;
      gbase[d] = lg + in_digit[j];
#pragma unroll
      for (int q = 0; q < RS_WAVES; ++q) wh[q][d] = ls + pw[j][q];
      ls += c[j];
      lg += dtot[j];
    }
  }
  __syncthreads();
  // 3. place in digit order, then write out contiguously
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    if (elem_index(tile_base, w, r, lane) < n) {
      const uint32_t p = wh[w][digit_of(key[r], shift, mask)] + lrank[r];
      skey[p] = key[r];
      sval[p] = val[r];
    }
  }
  __syncthreads();
  const int tile_n = (int)min((int64_t)RS_TILE, n - tile_base);
  if (!pl.rec_in) {
#pragma unroll 4
    for (int j = tid; j < tile_n; j += RS_THREADS) {
      const K k = skey[j];
      const uint32_t d = digit_of(k, shift, mask);
      const uint32_t pos = gbase[d] + ((uint32_t)j - lstart[d]);
      okeys[pos] = k;
      ovals[pos] = sval[j];
    }
    return;
  }
  if (pl.w_in)
    write_records<K, true>(skey, sval, gbase, lstart, tile_n, shift, mask, okeys, ovals, pl);
  else
    write_records<K, false>(skey, sval, gbase, lstart, tile_n, shift, mask, okeys, ovals, pl);
}

template <typename K, int NB>
void launch_pass(const K* sk, const uint32_t* sv, K* dk, uint32_t* dv, int64_t n,
                 const int64_t* dn, int shift, int dbits, int64_t ntiles, uint32_t* hist,
                 uint32_t* total, const SortPayload& pl, int vals_iota, hipStream_t st) {
  hipLaunchKernelGGL((k_hist<K, NB>), dim3((unsigned)ntiles), dim3(RS_THREADS), 0, st, sk, n, dn,
                     shift, dbits, ntiles, hist);
  hipLaunchKernelGGL(k_digit_scan, dim3(1u << dbits), dim3(RS_THREADS), 0, st, hist, ntiles,
                     total);
  hipLaunchKernelGGL((k_scatter<K, NB>), dim3((unsigned)ntiles), dim3(RS_THREADS), 0, st, sk, sv,
                     dk, dv, n, dn, shift, dbits, ntiles, (const uint32_t*)hist,
                     (const uint32_t*)total, pl, vals_iota);
}

template <typename K>
hipError_t sort_impl(K* keys, uint32_t* vals, K* akeys, uint32_t* avals, int64_t n, int bits,
                     void* tmp, hipStream_t st, const SortPayload* pl, bool vals_iota,
                     const int64_t* dn) {
  // with a device count the passes always run (the count is not known here);
  // without one, one element or none needs no pass
  if (n <= 0 || (!dn && n <= 1)) return hipSuccess;
  if (bits <= 0) bits = 1;
  const int64_t ntiles = ceil_div_i64(n, RS_TILE);
  uint32_t* hist = (uint32_t*)tmp;
  uint32_t* total = hist + RS_MAXBINS * ntiles;   // digit totals
  // fewest passes of at most 9 bits, the bits spread evenly over them; digits
  // of 8 bits or fewer use the 256-bin kernels (smaller LDS footprint)
  const int passes = (bits + RS_MAXBITS - 1) / RS_MAXBITS;
  const int dbits = (bits + passes - 1) / passes;
  K* src_k = keys;
  uint32_t* src_v = vals;
  K* dst_k = akeys;
  uint32_t* dst_v = avals;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * dbits;
    const SortPayload none{};
    const SortPayload& pp = (p == passes - 1 && pl) ? *pl : none;
    const int iota = (p == 0 && vals_iota) ? 1 : 0;
    if (dbits <= 8)
      launch_pass<K, 256>(src_k, src_v, dst_k, dst_v, n, dn, shift, dbits, ntiles, hist, total,
                          pp, iota, st);
    else
      launch_pass<K, 512>(src_k, src_v, dst_k, dst_v, n, dn, shift, dbits, ntiles, hist, total,
                          pp, iota, st);
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
  return sizeof(uint32_t) * RS_MAXBINS * (ntiles + 1) + 256;   // tile counts, digit totals
}

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* ak, uint32_t* av, int64_t n,
                          int bits, void* tmp, hipStream_t st, const SortPayload* pl,
                          bool vals_iota, const int64_t* dn) {
  return sort_impl<uint32_t>(keys, vals, ak, av, n, bits, tmp, st, pl, vals_iota, dn);
}

hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* ak, uint32_t* av, int64_t n,
                          int bits, void* tmp, hipStream_t st, const SortPayload* pl,
                          bool vals_iota, const int64_t* dn) {
  return sort_impl<uint64_t>(keys, vals, ak, av, n, bits, tmp, st, pl, vals_iota, dn);
}
