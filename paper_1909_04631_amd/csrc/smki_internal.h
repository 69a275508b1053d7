// Internal declarations shared by the HIP translation units of libsmki.
// Not part of the public C ABI (that is include/smki.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#define SMKI_WAVE 64

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
#define SMKI_HIP_TRY(expr)                                   \
  do {                                                       \
    hipError_t e__ = (expr);                                 \
    if (e__ != hipSuccess) return smki_hip_error(e__);       \
  } while (0)

int32_t smki_hip_error(hipError_t e);

// device error bits (sticky flag, OR-ed by kernels)
enum : uint32_t {
  DEVERR_LABEL = 1u << 0,      // label outside {-1, 0..K-1}
  DEVERR_NONFINITE = 1u << 1,  // non-finite coordinate
  DEVERR_RAY = 1u << 2,        // more than 2^20 free samples on one beam
  DEVERR_RANGE = 1u << 3,      // voxel index outside [-2^20, 2^20)
  DEVERR_HASH = 1u << 4,       // block hash full
  DEVERR_DUP = 1u << 5,        // the same block twice in an import
  DEVERR_CAPACITY = 1u << 6,   // a captured insert outgrew a capacity fixed at capture
};

// ---------------------------------------------------------------------------
// scan / sort primitives (scan.hip, radix_sort.hip)
// ---------------------------------------------------------------------------
// exclusive prefix sum of n elements (in may equal out); *total (device,
// nullable) receives the sum.  tmp must hold scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
hipError_t scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total, void* tmp,
                         hipStream_t st);
hipError_t scan_excl_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* tmp,
                         hipStream_t st);
// two independent exclusive scans (the same contract each) sharing two launches
// when each array has at most 512 tiles of 2048 elements; tmp as for the larger
hipError_t scan_excl_pair_i64_i32(const int64_t* ina, int64_t* outa, int64_t na, int64_t* tota,
                                  const int32_t* inb, int32_t* outb, int64_t nb, int32_t* totb,
                                  void* tmp, hipStream_t st);
// dnb (device, nullable): the second array's element count, nb then being its
// capacity; entries past the count are neither read nor written
hipError_t scan_excl_pair_i32(const int32_t* ina, int32_t* outa, int64_t na, int32_t* tota,
                              const int32_t* inb, int32_t* outb, int64_t nb, int32_t* totb,
                              void* tmp, hipStream_t st, const int32_t* dnb = nullptr);

// stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys.  keys/vals are sorted in place; alt_* are scratch of the same size.
// With a payload (n > 1), the last pass also writes rec_out[i] = rec_in[value
// of sorted element i] (and w_out alike when w_in is set).
struct SortPayload {
  const float4* rec_in;
  float4* rec_out;
  const float* w_in;
  float* w_out;
};
size_t radix_tmp_bytes(int64_t n);
// vals_iota: vals holds nothing on entry; element i's value is i.
// dn (device, nullable): the element count, read by the kernels; n is then a
// capacity (buffers, tiles and launches are sized for n elements).
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* alt_keys, uint32_t* alt_vals,
                          int64_t n, int bits, void* tmp, hipStream_t st,
                          const SortPayload* payload = nullptr, bool vals_iota = false,
                          const int64_t* dn = nullptr);
hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* alt_keys, uint32_t* alt_vals,
                          int64_t n, int bits, void* tmp, hipStream_t st,
                          const SortPayload* payload = nullptr, bool vals_iota = false,
                          const int64_t* dn = nullptr);

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
// Element count of a launch sized for capacity n: the device count *dn when
// given (the launch does not know it when it is enqueued), else n.
__device__ __forceinline__ int64_t eff_n(int64_t n, const int64_t* dn) {
  return dn ? min(n, *dn) : n;
}

__device__ __forceinline__ int64_t floordiv_i64(int64_t a, int64_t b) {
  int64_t q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

static inline int64_t ceil_div_i64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Wait until the stream's work is done, polling (blocking after 2 ms).
hipError_t stream_wait(hipStream_t q);
