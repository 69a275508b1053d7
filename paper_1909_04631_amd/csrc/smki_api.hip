// Host side of the C ABI declared in include/smki.h: the map object, argument
// validation, workspace management and the per-insert launch sequence.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "../../include/smki.h"
#include "smki_gather.h"


int32_t smki_hip_error(hipError_t e) {
  return e == hipErrorOutOfMemory ? SMKI_E_OOM : SMKI_E_DEVICE;
}

// Wait for the stream by polling its status: the insert's waits are short,
// and a blocking wait resumes the host only after an interrupt.  Waits longer
// than 2 ms fall back to the blocking wait.
hipError_t stream_wait(hipStream_t q) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipStreamQuery(q);
    if (e != hipErrorNotReady) return e;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2))
      return hipStreamSynchronize(q);
  }
}

namespace {

constexpr size_t kAlign = 256;

// Device memory of a map's growable buffers: the caller's allocator
// (smki_set_allocator) or hipMalloc / hipFree.  Every buffer is released by
// the allocator that made it.
struct Allocator {
  smki_alloc_fn alloc = nullptr;
  smki_release_fn release = nullptr;
  void* ctx = nullptr;
};

hipError_t dev_alloc(const Allocator& A, void** p, size_t bytes) {
  if (!A.alloc) return hipMalloc(p, bytes);
  *p = A.alloc(bytes, A.ctx);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_release(const Allocator& A, void* p) {
  if (!p) return;
  if (A.release)
    A.release(p, A.ctx);
  else
    (void)hipFree(p);
}

// A growable device region carved into aligned sub-buffers per phase.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  Allocator by;   // the allocator of base
  hipError_t reserve(size_t bytes, const Allocator& now = Allocator{}) {
    used = 0;
    if (bytes <= cap) return hipSuccess;
    if (base) {
      // work queued on any stream may still read the old region
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return e;
      dev_release(by, base);
      base = nullptr;
      cap = 0;
    }
    const size_t want = bytes + bytes / 4 + (1 << 20);
    hipError_t e = dev_alloc(now, (void**)&base, want);
    if (e != hipSuccess) return e;
    by = now;
    cap = want;
    return hipSuccess;
  }
  template <typename T>
  T* take(size_t n) {
    size_t off = (used + kAlign - 1) / kAlign * kAlign;
    used = off + std::max<size_t>(n, 1) * sizeof(T);
    return (T*)(base + off);
  }
  void release() {
    dev_release(by, base);
    base = nullptr;
    cap = used = 0;
  }
};

// Size of a sequence of aligned sub-buffers.
struct Sizer {
  size_t total = 0;
  template <typename T>
  void add(size_t n) {
    total = (total + kAlign - 1) / kAlign * kAlign + std::max<size_t>(n, 1) * sizeof(T);
  }
};

int ilog2(int32_t x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

int bits_for(int64_t n) {  // bits to represent values 0..n-1
  int b = 0;
  while (b < 62 && (int64_t(1) << b) < n) ++b;
  return b;
}

bool finite_pos(float x) { return isfinite(x) && x > 0.0f; }

// Bounding-box accumulators of k_count: initial values of every copy, and the
// reduction of the copies read back (min xyz, max xyz).
void bbox_init(int32_t* h) {
  for (int c = 0; c < SMKI_BBOX_COPIES; ++c)
    for (int a = 0; a < 8; ++a) h[c * 8 + a] = a < 3 ? INT32_MAX : (a < 6 ? INT32_MIN : 0);
}
void bbox_reduce(const int32_t* h, int32_t out[6]) {
  for (int a = 0; a < 3; ++a) {
    out[a] = INT32_MAX;
    out[3 + a] = INT32_MIN;
  }
  for (int c = 0; c < SMKI_BBOX_COPIES; ++c)
    for (int a = 0; a < 3; ++a) {
      out[a] = std::min(out[a], h[c * 8 + a]);
      out[3 + a] = std::max(out[3 + a], h[c * 8 + 3 + a]);
    }
}
constexpr size_t kBboxInts = 8 * SMKI_BBOX_COPIES;
constexpr size_t kStatBytes = sizeof(unsigned long long) * 4 * SMKI_STAT_COPIES;
// The device's insert counters (d_stats) are followed by one word holding an
// insert's new block and class block counts (two int32); both stay on the
// device until smki_last_scan_stats reads them (the next insert clears them).
constexpr size_t kStatAlloc = kStatBytes + sizeof(int64_t);
// pinned staging (h_pin, 8 KiB, int64 words): [20] the counting model's row
// count, [256, 512) the insert counters and [512] the new block counts (one
// copy of d_stats), [704, 706) the map's block counts read back with an
// insert's first copy
constexpr int kPinNew = 512, kPinCounts = 704;

}  // namespace

// Voxel offsets that a row of a cell can reach (first octant of the cell:
// mirrored per octant by the splat), nearest first, and their reach R.
struct Stencil {
  int32_t R = 0;
  std::vector<StencilOff> offs;
};

struct smki_map {
  float res, l, sigma0, alpha0;
  int32_t K, B, log2B, free_class;
  int32_t chunk;  // rows per splat work unit
  int32_t model;      // SMKI_MODEL_SBKI or SMKI_MODEL_SCSM
  int32_t selection;  // SMKI_SELECT_EXACT or SMKI_SELECT_FACE_BLOCKS
  int32_t flags;      // SMKI_FLAG_*
  int device = 0;
  hipStream_t stream = nullptr;
  // persistent device state
  MapDev dev{};
  int64_t pool_cap = 0;      // blocks
  int64_t n_blocks = 0;
  int64_t cpool_cap = 0;     // class blocks
  int64_t n_cblocks = 0;
  uint32_t* d_err = nullptr;
  unsigned long long* d_stats = nullptr;
  StencilOff* d_offs = nullptr;
  std::vector<StencilOff> dev_offs;      // the stencil now in d_offs
  int32_t dev_R = -1;
  // the last insert's stencil and the (l / res, rounding margin) it was built for
  Stencil sten_cache;
  double sten_lv = -1.0, sten_margin = -1.0;
  // kernel of each class (l_k, sigma0_k; all l and sigma0 unless set per class)
  std::vector<float> lk, s0k;
  float4* d_cls = nullptr;  // [K] (l^2, 1/l, sigma0 * Q's leading coefficient, l)
  // workspaces
  Arena a_hits, a_sets, a_tgts, a_misc;
  // pinned host staging
  int64_t* h_pin = nullptr;
  char* h_hdr = nullptr;   // pinned staging of an insert's first-phase header
  size_t h_hdr_cap = 0;
  smki_scan_stats last{};
  bool stats_pending = false;
  // per insert: events around the splat [0, 1] and the allocation + merge [2, 3],
  // kept for the last SMKI_TIMING_RING inserts; ev points at the current set
  hipEvent_t evr[SMKI_TIMING_RING][4] = {};
  hipEvent_t* ev = evr[0];
  int64_t n_timed = 0;    // inserts that recorded a set
  bool timing = true;     // inserts record the events (smki_set_kernel_timing)
  bool last_timed = false;   // the last insert recorded a set
  // Captured inserts (smki_batch_*): the device copy of the block counts
  // (dev.counts) is current after a replay, the host's (n_blocks, n_cblocks)
  // until then; epoch changes whenever the map's storage moves (a captured
  // graph holds its addresses).
  bool host_counts_valid = true;
  bool new_pending = false;   // the last insert's new (class) block counts are in h_pin[kPinNew]
  int64_t epoch = 0;
  smki_batch* stats_batch = nullptr;   // the replay whose counters smki_last_scan_stats reports
  // allocator of new growable buffers, and the one that made each current buffer
  Allocator alloc_now, by_hash, by_pool, by_cpool;
  int32_t last_vlo[3] = {0, 0, 0}, last_vhi[3] = {0, 0, 0};   // voxel box of the last insert
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
namespace {

smki_status status_of_err(uint32_t e) {
  if (e & (DEVERR_LABEL | DEVERR_NONFINITE | DEVERR_DUP)) return SMKI_E_BAD_INPUT;
  if (e & (DEVERR_RANGE | DEVERR_RAY)) return SMKI_E_RANGE;
  if (e & (DEVERR_HASH | DEVERR_CAPACITY)) return SMKI_E_CAPACITY;
  return SMKI_E_DEVICE;
}

// First-octant stencil: voxel offsets o (relative to a cell) whose centroid can
// lie within l of some point in the (+,+,+) octant of that cell, i.e. with the
// point at u in [0, 1/2]^3 (voxel units, relative to the cell centre):
// sum_a dist(o_a, [0, 1/2])^2 < (l/res + margin)^2.  The margin covers a point
// assigned to the neighbouring cell by the rounding of floor(x / res).  A point
// in another octant uses the mirrored offsets.  Ordered by that distance.
Stencil make_stencil(double lv, double margin) {
  Stencil s;
  const double L = lv + margin;
  s.R = std::max(0, (int32_t)ceil(lv + 0.5 + margin) - 1);
  auto dist = [](int o) { return o >= 1 ? o - 0.5 : (o == 0 ? 0.0 : -(double)o); };
  for (int dx = -s.R; dx <= s.R; ++dx)
    for (int dy = -s.R; dy <= s.R; ++dy)
      for (int dz = -s.R; dz <= s.R; ++dz) {
        const double ax = dist(dx), ay = dist(dy), az = dist(dz);
        if (ax * ax + ay * ay + az * az < L * L) s.offs.push_back(StencilOff{dx, dy, dz, 0});
      }
  // nearest first: the splat's last step then holds the offsets that a row can
  // reach least often, and is skipped for rows that reach none of them
  auto key = [&](const StencilOff& o) {
    const double ax = dist(o.dx), ay = dist(o.dy), az = dist(o.dz);
    return ax * ax + ay * ay + az * az;
  };
  std::stable_sort(s.offs.begin(), s.offs.end(),
                   [&](const StencilOff& a, const StencilOff& b) { return key(a) < key(b); });
  return s;
}

// Block sizes and reaches the S-BKI kernels serve: B in {2, 4, 8, 16}, reach
// R <= B (a row's region covers its own block and the 26 around it) and at
// most SMKI_MAX_REACH; the splat's LDS region (B + 2R)^3 floats stays under
// 64 KiB for all of them.
bool sbki_shape_ok(int32_t B, int32_t R) {
  return (B == 2 || B == 4 || B == 8 || B == 16) && R <= B && R <= SMKI_MAX_REACH;
}

hipError_t sync_read(smki_map* m, const void* dev, size_t bytes, void* host) {
  hipError_t e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, m->stream);
  if (e != hipSuccess) return e;
  return stream_wait(m->stream);
}

// Grow the block arrays (keys, class-block table) to hold `need` blocks.
smki_status ensure_pool(smki_map* m, int64_t need) {
  if (need <= m->pool_cap) return SMKI_OK;
  const int64_t cap = std::max<int64_t>(need, m->pool_cap * 2);
  int32_t* ncs = nullptr;
  uint64_t* nk = nullptr;
  SMKI_HIP_TRY(dev_alloc(m->alloc_now, (void**)&ncs, sizeof(int32_t) * m->K * cap));
  hipError_t e = dev_alloc(m->alloc_now, (void**)&nk, sizeof(uint64_t) * cap);
  if (e != hipSuccess) {
    dev_release(m->alloc_now, ncs);
    return smki_hip_error(e);
  }
  if (m->n_blocks > 0) {
    SMKI_HIP_TRY(hipMemcpyAsync(ncs, m->dev.cslot, sizeof(int32_t) * m->K * m->n_blocks,
                                hipMemcpyDeviceToDevice, m->stream));
    SMKI_HIP_TRY(hipMemcpyAsync(nk, m->dev.bkeys, sizeof(uint64_t) * m->n_blocks,
                                hipMemcpyDeviceToDevice, m->stream));
  }
  SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
  dev_release(m->by_pool, m->dev.cslot);
  dev_release(m->by_pool, m->dev.bkeys);
  m->by_pool = m->alloc_now;
  m->dev.cslot = ncs;
  m->dev.bkeys = nk;
  m->pool_cap = cap;
  ++m->epoch;
  return SMKI_OK;
}

// Grow the class-block pool (B^3 floats each) to hold `need` class blocks.
smki_status ensure_cpool(smki_map* m, int64_t need) {
  if (need <= m->cpool_cap) return SMKI_OK;
  const int64_t cap = std::max<int64_t>(need, m->cpool_cap * 2);
  const size_t per = (size_t)m->B * m->B * m->B;
  float* na = nullptr;
  SMKI_HIP_TRY(dev_alloc(m->alloc_now, (void**)&na, sizeof(float) * per * cap));
  if (m->n_cblocks > 0)
    SMKI_HIP_TRY(hipMemcpyAsync(na, m->dev.calpha, sizeof(float) * per * m->n_cblocks,
                                hipMemcpyDeviceToDevice, m->stream));
  SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
  dev_release(m->by_cpool, m->dev.calpha);
  m->by_cpool = m->alloc_now;
  m->dev.calpha = na;
  m->cpool_cap = cap;
  ++m->epoch;
  return SMKI_OK;
}

// Keep the block hash at most half full; rebuild it from the slot keys on growth.
smki_status ensure_hash(smki_map* m, int64_t blocks) {
  if (m->dev.hcap >= 2 * blocks && m->dev.hkeys) return SMKI_OK;
  int64_t cap = std::max<int64_t>(m->dev.hcap, 1 << 14);
  while (cap < 2 * blocks) cap *= 2;
  uint64_t* hk = nullptr;
  int32_t* hv = nullptr;
  SMKI_HIP_TRY(dev_alloc(m->alloc_now, (void**)&hk, sizeof(uint64_t) * cap));
  hipError_t e = dev_alloc(m->alloc_now, (void**)&hv, sizeof(int32_t) * cap);
  if (e != hipSuccess) {
    dev_release(m->alloc_now, hk);
    return smki_hip_error(e);
  }
  SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
  dev_release(m->by_hash, m->dev.hkeys);
  dev_release(m->by_hash, m->dev.hvals);
  m->by_hash = m->alloc_now;
  m->dev.hkeys = hk;
  m->dev.hvals = hv;
  m->dev.hcap = cap;
  ++m->epoch;
  SMKI_HIP_TRY(launch_hash_clear(m->dev, m->stream));
  SMKI_HIP_TRY(launch_hash_insert_slots(m->dev, 0, m->n_blocks, m->d_err, m->stream));
  return SMKI_OK;
}

// Device table of the class kernels (synchronous: no insert in flight reads it).
smki_status upload_class_params(smki_map* m) {
  std::vector<float4> t(m->K);
  for (int32_t k = 0; k < m->K; ++k) {
    const float l = m->lk[k];
    t[k] = make_float4(l * l, 1.0f / l, (float)(kSmkiQ[0] * (double)m->s0k[k]), l);
  }
  SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
  SMKI_HIP_TRY(hipMemcpy(m->d_cls, t.data(), sizeof(float4) * m->K, hipMemcpyHostToDevice));
  return SMKI_OK;
}

float max_class_l(const smki_map* m) {
  float l = 0.0f;
  for (float v : m->lk) l = std::max(l, v);
  return l;
}

// The block counts on the host, read back from the device after a replay of a
// captured insert (synchronises the map's stream then).
smki_status refresh_counts(smki_map* m) {
  if (m->host_counts_valid) return SMKI_OK;
  int64_t c[2];
  SMKI_HIP_TRY(sync_read(m, m->dev.counts, sizeof(c), c));
  m->n_blocks = c[0];
  m->n_cblocks = c[1];
  m->host_counts_valid = true;
  return SMKI_OK;
}

// The HIP events around an insert's splat [0, 1] and allocation + merge [2, 3],
// when the map records them: begin takes the next set of the ring and marks 0.
hipError_t timing_begin(smki_map* m, hipStream_t q) {
  if (!m->timing) return hipSuccess;
  m->ev = m->evr[m->n_timed++ % SMKI_TIMING_RING];
  m->last_timed = true;
  return hipEventRecord(m->ev[0], q);
}

hipError_t timing_mark(smki_map* m, int i, hipStream_t q) {
  return m->last_timed ? hipEventRecord(m->ev[i], q) : hipSuccess;
}

smki_status take_device_error(smki_map* m) {
  uint32_t e = 0;
  SMKI_HIP_TRY(sync_read(m, m->d_err, sizeof(uint32_t), &e));
  if (e) {
    SMKI_HIP_TRY(hipMemsetAsync(m->d_err, 0, sizeof(uint32_t), m->stream));
    SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
    return status_of_err(e);
  }
  return SMKI_OK;
}

// Grid of blocks covering voxel box [vlo, vhi].
BucketGeom make_geom(const smki_map* m, const int32_t vlo[3], const int32_t vhi[3], int32_t planes) {
  BucketGeom g{};
  g.planes = planes;
  g.res = m->res;
  g.B = m->B;
  g.log2B = m->log2B;
  g.n_blocks = 1;
  for (int a = 0; a < 3; ++a) {
    const int32_t lo = vlo[a] >> m->log2B, hi = vhi[a] >> m->log2B;
    g.blo[a] = lo;
    g.nb[a] = hi - lo + 1;
    g.n_blocks *= g.nb[a];
  }
  g.key_bits = std::max(1, bits_for(g.n_blocks * planes) + 3 * m->log2B);
  return g;
}

// ---------------------------------------------------------------------------
// counting-model insert (S-CSM): rows already bucketed; allocate the row blocks,
// then add each (class, voxel) run length to alpha
// ---------------------------------------------------------------------------
smki_status insert_csm(smki_map* m, const BucketGeom& g, const PointSet& ps,
                       const float* wts_unsorted, const void* keys,
                       int32_t n_slots, int32_t n_t, int64_t n_ext, const int32_t eblo[3],
                       const int32_t enb[3], const int32_t* d_mark, const int32_t* d_mpos,
                       int32_t* d_ext2t, hipStream_t q) {
  const int32_t B3 = m->B * m->B * m->B;
  const int64_t ntk = (int64_t)n_t * m->K;
  SplatArgs sa{};
  sa.g = g;
  sa.K = m->K;
  sa.pts = nullptr;   // the counting model reads no records
  sa.wts = wts_unsorted;
  sa.perm = ps.perm;
  sa.dense = ps.dense;
  sa.head = ps.head;
  sa.slot_lin = ps.slot_lin;
  sa.n_slots = n_slots;
  for (int q2 = 0; q2 < 3; ++q2) {
    sa.eblo[q2] = eblo[q2];
    sa.enb[q2] = enb[q2];
  }
  sa.ext2t = d_ext2t;
  sa.stats = m->d_stats;
  Sizer zc;
  for (int i = 0; i < 5; ++i) zc.add<int32_t>(n_t);
  zc.add<int32_t>(8);
  zc.add<char>(scan_tmp_bytes(std::max<int64_t>(ntk, 1)));
  const int64_t vwords = (B3 + 31) / 32;   // voxel bits per target block
  zc.add<uint32_t>((size_t)n_t * vwords);
  for (int i = 0; i < 3; ++i) zc.add<int32_t>(ntk);
  SMKI_HIP_TRY(m->a_tgts.reserve(zc.total, m->alloc_now));
  Arena& C = m->a_tgts;
  // cleared together: counts, voxel bits, contribution flags
  int32_t* d_cnt = C.take<int32_t>(8);
  uint32_t* d_vbits = C.take<uint32_t>((size_t)n_t * vwords);
  int32_t* d_contrib = C.take<int32_t>(ntk);
  int32_t* d_tgt = C.take<int32_t>(n_t);
  int32_t* d_active = C.take<int32_t>(n_t);
  int32_t* d_tslot = C.take<int32_t>(n_t);
  int32_t* d_isnew = C.take<int32_t>(n_t);
  int32_t* d_rank = C.take<int32_t>(n_t);
  void* d_ctmp = C.take<char>(scan_tmp_bytes(std::max<int64_t>(ntk, 1)));
  int32_t* d_need = C.take<int32_t>(ntk);
  int32_t* d_cpos = C.take<int32_t>(ntk);
  sa.tgt_elin = d_tgt;
  sa.tgt_active = d_active;
  sa.tgt_slot = d_tslot;
  sa.contrib = d_contrib;
  SMKI_HIP_TRY(hipMemsetAsync(d_cnt, 0,
                              (size_t)((char*)(d_contrib + std::max<int64_t>(ntk, 1)) - (char*)d_cnt),
                              q));
  SMKI_HIP_TRY(hipMemsetAsync(m->d_stats, 0, kStatBytes, q));
  SMKI_HIP_TRY(launch_list_targets(d_mark, d_mpos, n_ext, d_tgt, d_ext2t, q));
  SMKI_HIP_TRY(launch_fill_i32(d_active, n_t, 1, q));   // every row block is updated
  SMKI_HIP_TRY(launch_contrib(sa, true, d_contrib, q));
  SMKI_HIP_TRY(timing_begin(m, q));
  SMKI_HIP_TRY(timing_mark(m, 1, q));
  SMKI_HIP_TRY(launch_map_lookup(m->dev, sa, n_t, d_tslot, d_isnew, q));
  SMKI_HIP_TRY(launch_need(m->dev, n_t, d_contrib, d_isnew, d_tslot, d_need, d_cpos, q));
  SMKI_HIP_TRY(scan_excl_pair_i32(d_isnew, d_rank, n_t, d_cnt, d_cpos, d_cpos, n_t, d_cnt + 1,
                                  d_ctmp, q));
  int32_t cnt[2];
  SMKI_HIP_TRY(sync_read(m, d_cnt, sizeof(cnt), cnt));
  const int64_t n_new = cnt[0], n_cnew = cnt[1];
  m->last.n_new_blocks = n_new;
  smki_status rc = ensure_pool(m, m->n_blocks + n_new);
  if (rc != SMKI_OK) return rc;
  rc = ensure_hash(m, m->n_blocks + n_new);
  if (rc != SMKI_OK) return rc;
  rc = ensure_cpool(m, m->n_cblocks + n_cnew);
  if (rc != SMKI_OK) return rc;
  SMKI_HIP_TRY(timing_mark(m, 2, q));
  SMKI_HIP_TRY(launch_assign(m->dev, sa, n_t, d_isnew, d_rank, m->n_blocks, d_tslot, d_need,
                             d_cpos, m->n_cblocks, m->d_err, q));
  SMKI_HIP_TRY(launch_fill_calpha0(m->dev, m->n_cblocks, n_cnew, q));
  sa.map = m->dev;
  SMKI_HIP_TRY(launch_csm_counts(sa, keys, g.key_bits > 32, ps.n, d_vbits, n_t, q));
  SMKI_HIP_TRY(timing_mark(m, 3, q));
  // in-support pairs of the counting model: every row counts once (staged in
  // pinned memory, which no later insert touches before this one has synchronised)
  unsigned long long* h_rows = (unsigned long long*)(m->h_pin + 20);
  *h_rows = (unsigned long long)ps.n;
  SMKI_HIP_TRY(hipMemcpyAsync(m->d_stats + 1, h_rows, sizeof(*h_rows), hipMemcpyHostToDevice, q));
  m->n_blocks += n_new;
  m->n_cblocks += n_cnew;
  m->last.n_new_class_blocks = n_cnew;
  m->stats_pending = true;
  return SMKI_OK;
}

// ---------------------------------------------------------------------------
// the insert (one or several scans)
// ---------------------------------------------------------------------------
// label (one class per hit) or probs (soft: [n][K] class weights per hit), not both
smki_status insert_impl(smki_map* m, const float* xyz, const int32_t* label, const float* probs,
                        int64_t n, const int64_t* offsets, const float* origins, int32_t S,
                        float step) {
  // host-side validation
  if (!m || S < 1 || !offsets || !origins || n < 0 ||
      (n > 0 && (!xyz || (label == nullptr) == (probs == nullptr))))
    return SMKI_E_INVALID_ARG;
  if (!isfinite(step)) return SMKI_E_INVALID_ARG;
  if (offsets[0] != 0 || offsets[S] != n) return SMKI_E_INVALID_ARG;
  for (int32_t s = 0; s < S; ++s)
    if (offsets[s + 1] < offsets[s]) return SMKI_E_INVALID_ARG;
  for (int32_t s = 0; s < 3 * S; ++s) {
    if (!isfinite(origins[s])) return SMKI_E_INVALID_ARG;
    const float q = floorf((float)((double)origins[s] / (double)m->res));
    if (!(q >= -(float)SMKI_COORD_LIM && q < (float)SMKI_COORD_LIM)) return SMKI_E_RANGE;
  }
  if (n > (int64_t)INT32_MAX / 2) return SMKI_E_CAPACITY;
  // soft: up to K hit rows per hit, counted in int32
  if (probs && n * (int64_t)m->K > (int64_t)INT32_MAX / 2) return SMKI_E_CAPACITY;
  SMKI_HIP_TRY(hipSetDevice(m->device));
  // block counts still on the device (after an insert or a replay) come back
  // with this insert's first copy
  const bool counts_on_device = !m->host_counts_valid;
  smki_scan_stats st{};
  m->last = st;
  m->stats_pending = false;
  m->new_pending = false;
  m->last_timed = false;
  m->stats_batch = nullptr;
  if (n == 0) return SMKI_OK;
  hipStream_t q = m->stream;

  // ---- phase A: per-hit validation, free-sample counts, bounding box ----
  // A header, uploaded in one copy from pinned memory and read back in one:
  // [0, 32) counts (zeroed), [32, 36) error word of this phase (zeroed),
  // [64, 64 + 4 kBboxInts) bounding-box copies, then the scan offsets and origins.
  constexpr size_t kHdrBox = 64, kHdrTail = 64 + sizeof(int32_t) * kBboxInts;
  const size_t hdr_bytes = kHdrTail + sizeof(int64_t) * (S + 1) + sizeof(float) * 3 * S;
  if (hdr_bytes > m->h_hdr_cap) {
    SMKI_HIP_TRY(hipStreamSynchronize(q));   // the old staging may still be read
    if (m->h_hdr) (void)hipHostFree(m->h_hdr);
    m->h_hdr = nullptr;
    m->h_hdr_cap = 0;
    SMKI_HIP_TRY(hipHostMalloc((void**)&m->h_hdr, hdr_bytes, hipHostMallocDefault));
    m->h_hdr_cap = hdr_bytes;
  }
  char* hh = m->h_hdr;
  memset(hh, 0, kHdrBox);
  bbox_init((int32_t*)(hh + kHdrBox));
  memcpy(hh + kHdrTail, offsets, sizeof(int64_t) * (S + 1));
  memcpy(hh + kHdrTail + sizeof(int64_t) * (S + 1), origins, sizeof(float) * 3 * S);
  Sizer za;
  za.add<char>(hdr_bytes);
  za.add<int64_t>(n);        // nfree
  za.add<int64_t>(n);        // off
  za.add<int32_t>(n);        // kept
  za.add<int32_t>(n);        // kpos
  za.add<char>(scan_tmp_bytes(n));
  SMKI_HIP_TRY(m->a_hits.reserve(za.total, m->alloc_now));
  Arena& A = m->a_hits;
  char* d_hdr = A.take<char>(hdr_bytes);
  int64_t* d_sc = (int64_t*)d_hdr;
  uint32_t* d_err0 = (uint32_t*)(d_hdr + 32);
  int32_t* d_bbox = (int32_t*)(d_hdr + kHdrBox);
  int64_t* d_soff = (int64_t*)(d_hdr + kHdrTail);
  float* d_org = (float*)(d_hdr + kHdrTail + sizeof(int64_t) * (S + 1));
  int64_t* d_nfree = A.take<int64_t>(n);
  int64_t* d_off = A.take<int64_t>(n);
  int32_t* d_kept = A.take<int32_t>(n);
  int32_t* d_kpos = A.take<int32_t>(n);
  void* d_stmp = A.take<char>(scan_tmp_bytes(n));
  SMKI_HIP_TRY(hipMemcpyAsync(d_hdr, hh, hdr_bytes, hipMemcpyHostToDevice, q));
  SMKI_HIP_TRY(launch_count(xyz, label, probs, n, d_soff, d_org, S, m->res, step, m->K, d_nfree,
                            d_kept, d_bbox, d_err0, q));
  SMKI_HIP_TRY(scan_excl_pair_i64_i32(d_nfree, d_off, n, d_sc, d_kept, d_kpos, n,
                                      (int32_t*)(d_sc + 1), d_stmp, q));
  // sync 1: counts, error word and box in one copy (and the map's block counts)
  SMKI_HIP_TRY(hipMemcpyAsync(hh, d_hdr, kHdrTail, hipMemcpyDeviceToHost, q));
  if (counts_on_device)
    SMKI_HIP_TRY(hipMemcpyAsync(m->h_pin + kPinCounts, m->dev.counts, 2 * sizeof(int64_t),
                                hipMemcpyDeviceToHost, q));
  SMKI_HIP_TRY(stream_wait(q));
  if (counts_on_device) {
    m->n_blocks = m->h_pin[kPinCounts];
    m->n_cblocks = m->h_pin[kPinCounts + 1];
    m->host_counts_valid = true;
  }
  const int64_t nf = ((const int64_t*)hh)[0];
  const int64_t nk = (int64_t)((const int32_t*)hh)[2];
  int32_t bb[6];
  bbox_reduce((const int32_t*)(hh + kHdrBox), bb);
  const uint32_t derr = *(const uint32_t*)(hh + 32);
  if (derr) return status_of_err(derr);
  m->last.n_hits = nk;
  m->last.n_free = nf;
  if (nk == 0) return SMKI_OK;
  if (nk + nf > (int64_t)INT32_MAX - 1) return SMKI_E_CAPACITY;

  // ---- geometry of this insert ----
  int32_t vlo[3], vhi[3];
  int64_t maxabs = 0;
  for (int q2 = 0; q2 < 3; ++q2) {
    vlo[q2] = std::max(bb[q2] - 1, -SMKI_COORD_LIM);
    vhi[q2] = std::min(bb[3 + q2] + 1, SMKI_COORD_LIM - 1);
    maxabs = std::max<int64_t>(maxabs, std::max(std::abs((int64_t)vlo[q2]), std::abs((int64_t)vhi[q2])));
  }
  const BucketGeom g = make_geom(m, vlo, vhi, m->K);
  for (int q2 = 0; q2 < 3; ++q2) {
    m->last_vlo[q2] = vlo[q2];
    m->last_vhi[q2] = vhi[q2];
  }
  if (g.n_blocks * m->K > (int64_t(1) << 30)) return SMKI_E_CAPACITY;
  if ((int64_t)(g.nb[0] + 2) * (g.nb[1] + 2) * (g.nb[2] + 2) > (int64_t(1) << 30))
    return SMKI_E_CAPACITY;
  const bool csm = m->model == SMKI_MODEL_SCSM;
  const double lv = (double)max_class_l(m) / (double)m->res;   // the stencil of the widest kernel
  const double margin = std::max(1e-4, 4.0 * ldexp((double)maxabs + 1.0, -23));
  if (!csm && (lv != m->sten_lv || margin != m->sten_margin)) {   // (rebuilt when they change)
    m->sten_cache = make_stencil(lv, margin);
    m->sten_lv = lv;
    m->sten_margin = margin;
  }
  const Stencil empty_sten{};
  const Stencil& sten = csm ? empty_sten : m->sten_cache;
  if (!csm && !sbki_shape_ok(m->B, sten.R)) return SMKI_E_CAPACITY;
  // target blocks: the row blocks and their neighbours (S-BKI), the row blocks (S-CSM)
  const int32_t DB = csm ? 0 : 1;
  int32_t eblo[3], enb[3];
  int64_t n_ext = 1;
  for (int q2 = 0; q2 < 3; ++q2) {
    eblo[q2] = g.blo[q2] - DB;
    enb[q2] = g.nb[q2] + 2 * DB;
    n_ext *= enb[q2];
  }
  const int32_t DR = m->B + 2 * sten.R;
  const int64_t DR3 = (int64_t)DR * DR * DR;

  // ---- phase B: bucket all rows (class-major keys), mark target blocks ----
  const int64_t nt = nk + nf;
  const int64_t max_slots = std::min<int64_t>(nt, g.n_blocks * m->K);
  Sizer zb;
  zb.add<int32_t>(g.n_blocks * m->K);
  zb.add<int32_t>(max_slots);
  zb.add<int32_t>(8);
  zb.add<int32_t>(m->K);
  zb.add<uint64_t>(nt);
  zb.add<uint64_t>(nt);
  zb.add<uint32_t>(nt);
  zb.add<uint32_t>(nt);
  zb.add<float4>(nt);
  zb.add<int32_t>(nt);
  zb.add<int32_t>(nt);
  zb.add<int32_t>(max_slots + 1);
  zb.add<char>(radix_tmp_bytes(nt));
  zb.add<char>(scan_tmp_bytes(std::max(nt, n_ext)));
  zb.add<int32_t>(n_ext);
  zb.add<int32_t>(n_ext);
  zb.add<int32_t>(n_ext);
  zb.add<int32_t>(max_slots);
  zb.add<int32_t>(max_slots);
  if (probs) zb.add<float>(nt);   // row weights (read through the permutation)
  zb.add<int32_t>(free_sample_workgroups(nf));
  SMKI_HIP_TRY(m->a_sets.reserve(zb.total, m->alloc_now));
  Arena& Bz = m->a_sets;
  PointSet ps{};
  ps.n = nt;
  ps.pts = nullptr;   // records stay unsorted: the splat reads them through the permutation
  ps.dense = Bz.take<int32_t>(g.n_blocks * m->K);
  ps.slot_lin = Bz.take<int32_t>(max_slots);
  ps.prefix = nullptr;   // the splat needs only the slot ranges
  ps.head = Bz.take<int32_t>(max_slots + 1);
  BucketScratch scr{};
  scr.keys = Bz.take<uint64_t>(nt);
  scr.akeys = Bz.take<uint64_t>(nt);
  scr.idx = Bz.take<uint32_t>(nt);
  scr.aidx = Bz.take<uint32_t>(nt);
  scr.rec = Bz.take<float4>(nt);
  scr.flag = Bz.take<int32_t>(nt);
  scr.slot_excl = Bz.take<int32_t>(nt);
  scr.sort_tmp = Bz.take<char>(radix_tmp_bytes(nt));
  scr.scan_tmp = Bz.take<char>(scan_tmp_bytes(std::max(nt, n_ext)));
  int32_t* d_si = Bz.take<int32_t>(8);   // counts; cleared with the target marks below
  int32_t* d_cfirst = Bz.take<int32_t>(m->K);   // first slot of each class (cleared too)
  ps.d_nslots = d_si;
  int32_t* d_ntgt = d_si + 1;
  int32_t* d_nunits = d_si + 2;
  int32_t* d_mark = Bz.take<int32_t>(n_ext);
  int32_t* d_mpos = Bz.take<int32_t>(n_ext);
  int32_t* d_ext2t = Bz.take<int32_t>(n_ext);
  int32_t* d_nun = Bz.take<int32_t>(max_slots);
  int32_t* d_ust = Bz.take<int32_t>(max_slots);
  ps.wts = nullptr;
  scr.wt = probs ? Bz.take<float>(nt) : nullptr;
  int32_t* d_wgbeam = Bz.take<int32_t>(free_sample_workgroups(nf));
  // one launch clears the counts and target marks, the insert counters, and the
  // dense slot table
  SMKI_HIP_TRY(launch_clear3(d_si, (int64_t)(d_mark + n_ext - d_si), (int32_t*)m->d_stats,
                             (int64_t)(kStatBytes / sizeof(int32_t)), ps.dense,
                             g.n_blocks * m->K, -1, q));
  // errors of the bucketing (a row's voxel index out of range) go to d_si[3],
  // read with the counts below, before any concentration is written
  SMKI_HIP_TRY(bucket_scan(xyz, label, probs, m->K, n, d_kept, d_kpos, nk, d_off, nf, d_wgbeam,
                           d_soff, d_org, S, step, m->free_class, g, ps, scr,
                           (uint32_t*)(d_si + 3), q));
  SMKI_HIP_TRY(launch_mark_targets(ps.slot_lin, ps.d_nslots, (int32_t)max_slots, g, eblo, enb, DB,
                                   d_mark, q));
  SMKI_HIP_TRY(launch_slot_units(ps.head, ps.d_nslots, (int32_t)max_slots, m->chunk, d_nun, q,
                                 ps.slot_lin, g.n_blocks, d_cfirst));
  SMKI_HIP_TRY(scan_excl_pair_i32(d_mark, d_mpos, n_ext, d_ntgt, d_nun, d_ust, max_slots, d_nunits,
                                  scr.scan_tmp, q, ps.d_nslots));
  // sync 2: slots, targets, work units, the bucketing's error word, each
  // class's first slot
  std::vector<int32_t> sih((size_t)(d_cfirst + m->K - d_si));
  SMKI_HIP_TRY(sync_read(m, d_si, sizeof(int32_t) * sih.size(), sih.data()));
  const int32_t* si = sih.data();
  const int32_t* cfirst = si + (d_cfirst - d_si);
  if (si[3]) return status_of_err((uint32_t)si[3]);
  const int32_t n_slots = si[0], n_t = si[1];
  const int64_t n_units = si[2];
  m->last.n_point_blocks = n_slots;
  m->last.n_target_blocks = n_t;
  m->last.n_units = n_units;
  if ((double)n_units * (double)DR3 * sizeof(float) > 64.0 * (1ull << 30)) return SMKI_E_CAPACITY;
  m->last.n_candidates = nt * (int64_t)sten.offs.size();
  m->last.n_lane_slots = nt * (int64_t)SMKI_WAVE * ((int64_t)(sten.offs.size() + SMKI_WAVE - 1) / SMKI_WAVE);

  // ---- phase C: splat, allocate, merge ----
  if (csm)
    return insert_csm(m, g, ps, scr.wt, scr.keys, n_slots, n_t, n_ext, eblo, enb, d_mark, d_mpos,
                      d_ext2t, q);
  // Room in the map for what this insert can allocate, by bounds known now, so
  // that the allocation needs no further synchronisation: at most one new block
  // per target, and per class at most min(targets, 27 x its slots) new class
  // blocks (a slot's rows reach its own block and the 26 around it).
  {
    int64_t new_cb = 0, prev = -1, prev_first = 0;
    for (int32_t c = 0; c < m->K; ++c) {
      if (cfirst[c] <= 0) continue;
      if (prev >= 0) new_cb += std::min<int64_t>(n_t, 27 * (int64_t)(cfirst[c] - 1 - prev_first));
      prev = c;
      prev_first = cfirst[c] - 1;
    }
    if (prev >= 0) new_cb += std::min<int64_t>(n_t, 27 * (int64_t)(n_slots - prev_first));
    smki_status rc = ensure_pool(m, m->n_blocks + n_t);
    if (rc == SMKI_OK) rc = ensure_hash(m, m->n_blocks + n_t);
    if (rc == SMKI_OK) rc = ensure_cpool(m, m->n_cblocks + new_cb);
    if (rc != SMKI_OK) return rc;
  }
  SplatArgs sa{};
  sa.g = g;
  sa.R = sten.R;
  sa.noff = (int32_t)sten.offs.size();
  // the stencil changes only with l / res (or the rounding margin)
  if (sten.R != m->dev_R || sten.offs.size() != m->dev_offs.size() ||
      memcmp(sten.offs.data(), m->dev_offs.data(), sizeof(StencilOff) * sten.offs.size()) != 0) {
    SMKI_HIP_TRY(hipStreamSynchronize(q));   // no insert in flight reads the old stencil
    SMKI_HIP_TRY(hipMemcpy(m->d_offs, sten.offs.data(), sizeof(StencilOff) * sten.offs.size(),
                           hipMemcpyHostToDevice));
    m->dev_offs = sten.offs;
    m->dev_R = sten.R;
  }
  sa.offs = (const int4*)m->d_offs;
  sa.cls = m->d_cls;
  for (int i = 0; i < SMKI_POLY_N; ++i) sa.mcoef[i] = (float)(kSmkiQ[i] / kSmkiQ[0]);
  sa.K = m->K;
  sa.chunk = m->chunk;
  // piece p = (dx+1)*9 + (dy+1)*3 + (dz+1): all 27, or those with at most one dx, dy, dz != 0
  sa.piece_mask = 0;
  for (int p = 0; p < 27; ++p) {
    const int nz = (p / 9 != 1) + ((p / 3) % 3 != 1) + (p % 3 != 1);
    if (m->selection == SMKI_SELECT_EXACT || nz <= 1) sa.piece_mask |= 1u << p;
  }
  sa.pts = scr.rec;   // unsorted records and weights, read through the permutation
  sa.wts = scr.wt;
  sa.perm = ps.perm;
  sa.dense = ps.dense;
  sa.head = ps.head;
  sa.slot_lin = ps.slot_lin;
  sa.nunits = d_nun;
  sa.ustart = d_ust;
  for (int q2 = 0; q2 < 3; ++q2) {
    sa.eblo[q2] = eblo[q2];
    sa.enb[q2] = enb[q2];
  }
  sa.ext2t = d_ext2t;
  sa.stats = m->d_stats;
  Sizer zc;
  zc.add<int32_t>(n_t);   // tgt_elin
  zc.add<int32_t>(n_t);   // active
  zc.add<int32_t>(n_t);   // tgt_slot
  zc.add<int32_t>(n_t);   // is_new
  zc.add<int32_t>(n_t);   // new_rank
  zc.add<int32_t>(8);
  const int64_t ntk = (int64_t)n_t * m->K;
  zc.add<char>(scan_tmp_bytes(std::max<int64_t>(ntk, 1)));
  zc.add<int4>(n_units);
  zc.add<float>(SMKI_PART_HEAD + (size_t)n_units * DR3);
  zc.add<uint32_t>(n_units);
  zc.add<int32_t>(n_units);   // splat launch order
  zc.add<int4>(n_slots);
  for (int i = 0; i < 3; ++i) zc.add<int32_t>(ntk);
  SMKI_HIP_TRY(m->a_tgts.reserve(zc.total, m->alloc_now));
  Arena& C = m->a_tgts;
  // cleared together: counts, active flags, contribution flags
  int32_t* d_cnt = C.take<int32_t>(8);
  int32_t* d_active = C.take<int32_t>(n_t);
  int32_t* d_contrib = C.take<int32_t>(ntk);
  int32_t* d_tgt = C.take<int32_t>(n_t);
  int32_t* d_tslot = C.take<int32_t>(n_t);
  int32_t* d_isnew = C.take<int32_t>(n_t);
  int32_t* d_rank = C.take<int32_t>(n_t);
  void* d_ctmp = C.take<char>(scan_tmp_bytes(std::max<int64_t>(ntk, 1)));
  int4* d_units = C.take<int4>(n_units);
  float* d_part = C.take<float>(SMKI_PART_HEAD + (size_t)n_units * DR3);
  uint32_t* d_umask = C.take<uint32_t>(n_units);
  int32_t* d_uorder = C.take<int32_t>(n_units);
  int4* d_sinfo = C.take<int4>(n_slots);
  int32_t* d_need = C.take<int32_t>(ntk);
  int32_t* d_cpos = C.take<int32_t>(ntk);
  sa.tgt_elin = d_tgt;
  sa.tgt_active = d_active;
  sa.tgt_slot = d_tslot;
  sa.units = d_units;
  sa.uorder = d_uorder;
  sa.part = d_part;
  sa.part_elems = SMKI_PART_HEAD + n_units * DR3;
  sa.wide = (m->flags & SMKI_FLAG_WIDE_OFFSETS) ? 1 : 0;
  sa.umask = d_umask;
  sa.sinfo = d_sinfo;
  sa.n_slots = n_slots;
  sa.contrib = d_contrib;
  // the splat first (its counters were cleared before the bucketing); what
  // only the later kernels read is prepared while it runs
  SMKI_HIP_TRY(launch_unit_table(d_nun, d_ust, ps.head, ps.slot_lin, g.n_blocks, m->chunk, n_slots,
                                 ps.d_nslots, d_nunits, d_units, d_uorder, q));
  SMKI_HIP_TRY(timing_begin(m, q));
  SMKI_HIP_TRY(launch_splat(sa, n_units, q));
  SMKI_HIP_TRY(timing_mark(m, 1, q));
  // the counts, active flags and contribution flags cleared, the targets
  // listed and the slots summarised, in one launch
  SMKI_HIP_TRY(launch_after_splat(sa, d_cnt, (int64_t)(d_contrib + std::max<int64_t>(ntk, 1) - d_cnt),
                                  d_mark, d_mpos, n_ext, d_tgt, d_ext2t, q));
  SMKI_HIP_TRY(launch_contrib(sa, false, d_contrib, q));
  SMKI_HIP_TRY(launch_map_lookup(m->dev, sa, n_t, d_tslot, d_isnew, q));
  SMKI_HIP_TRY(launch_need(m->dev, n_t, d_contrib, d_isnew, d_tslot, d_need, d_cpos, q));
  SMKI_HIP_TRY(scan_excl_pair_i32(d_isnew, d_rank, n_t, d_cnt, d_cpos, d_cpos, n_t, d_cnt + 1,
                                  d_ctmp, q));
  // no synchronisation here: the map has room for the bounds above; the
  // numbers of new blocks and class blocks stay on the device, which updates
  // the map's counts there (the host reads them back at its next synchronisation)
  SMKI_HIP_TRY(timing_mark(m, 2, q));
  SMKI_HIP_TRY(launch_assign(m->dev, sa, n_t, d_isnew, d_rank, m->n_blocks, d_tslot, d_need,
                             d_cpos, m->n_cblocks, m->d_err, q, d_cnt,
                             (int32_t*)((char*)m->d_stats + kStatBytes)));
  sa.map = m->dev;
  sa.n_cold = m->n_cblocks;
  sa.alpha0 = m->alpha0;
  SMKI_HIP_TRY(launch_merge(sa, n_t, q));
  SMKI_HIP_TRY(timing_mark(m, 3, q));
  m->host_counts_valid = false;
  m->new_pending = true;
  m->stats_pending = true;
  return SMKI_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// captured batched insert: every launch sized for capacities fixed at capture,
// every count read on the device, no host synchronisation (a HIP graph)
// ---------------------------------------------------------------------------
namespace {

// Input header of a replay (pinned on the host, copied by the graph's first
// node): [0, 32) int64 install-counts flag, blocks, class blocks; [32, 48) the
// first phase's totals (zeroed); [48, 52) error word (zeroed); [64, ...) the
// bounding-box copies; then the scan offsets and origins.
constexpr size_t kBSc = 32, kBErr = 48, kBBox = 64;
constexpr size_t kBTail = kBBox + sizeof(int32_t) * kBboxInts;
constexpr int kBOut = 16;   // int64 results ahead of the counter copies in the output

struct BatchBufs {
  char* hdr;
  int64_t *sc, *soff, *pc, *out;
  uint32_t* err;
  int32_t* bbox;
  float* org;
  unsigned long long* stats;
  int64_t *nfree, *off;
  int32_t *kept, *kpos, *wgbeam;
  void *stmp_a, *sort_tmp, *scan_tmp, *ctmp;
  int32_t *si, *mark, *mpos, *ext2t, *dense, *slot_lin, *head, *nun, *ust;
  void *keys, *akeys;
  uint32_t *idx, *aidx;
  float4* rec;
  int32_t *flag, *slot_excl;
  int32_t *cnt, *active, *contrib, *tgt, *tslot, *isnew, *rank, *need, *cpos, *uorder;
  int4 *units, *sinfo;
  float* part;
  uint32_t* umask;
};

}  // namespace

struct smki_batch {
  smki_map* m = nullptr;
  int64_t epoch = -1;        // the map's storage epoch the graph was recorded for
  const float* xyz = nullptr;
  const int32_t* label = nullptr;
  int64_t n = 0;
  int32_t S = 0;
  float step = 0.0f;
  BucketGeom g{};            // the window: the sizing insert's voxel box, grown
  int32_t eblo[3] = {0, 0, 0}, enb[3] = {0, 0, 0};
  int64_t n_ext = 0;
  Stencil sten;
  int64_t cap_rows = 0, cap_slots = 0, cap_units = 0;
  int64_t pool_cap = 0, cpool_cap = 0, hcap = 0;
  size_t in_bytes = 0;
  char* dbuf = nullptr;
  Allocator by;              // the allocator of dbuf
  char* h_in = nullptr;      // pinned input header
  int64_t* h_out = nullptr;  // pinned results: kBOut int64, then the counter copies
  StencilOff* d_offs = nullptr;
  BatchBufs d{};
  hipStream_t cs = nullptr;  // stream the graph is recorded on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool launched = false;
};

namespace {

// Aligned sub-buffers carved from base (nullptr: sizes only).
struct Carver {
  char* base;
  size_t used = 0;
  template <typename T>
  T* take(size_t k) {
    size_t off = (used + kAlign - 1) / kAlign * kAlign;
    used = off + std::max<size_t>(k, 1) * sizeof(T);
    return base ? (T*)(base + off) : nullptr;
  }
};

// Carve the batch's device buffers from base (nullptr: size only).
size_t carve_batch(smki_batch* b, char* base) {
  smki_map* m = b->m;
  const int64_t n = std::max<int64_t>(b->n, 1), ne = b->n_ext, ntk = ne * m->K;
  const int64_t R = b->cap_rows, NS = b->cap_slots, NU = b->cap_units;
  const int64_t DR = m->B + 2 * b->sten.R, DR3 = DR * DR * DR;
  const size_t kw = b->g.key_bits <= 32 ? 4 : 8;
  Carver c{base};
  BatchBufs& d = b->d;
  d.hdr = c.take<char>(b->in_bytes);
  d.sc = (int64_t*)(d.hdr ? d.hdr + kBSc : nullptr);
  d.err = (uint32_t*)(d.hdr ? d.hdr + kBErr : nullptr);
  d.bbox = (int32_t*)(d.hdr ? d.hdr + kBBox : nullptr);
  d.soff = (int64_t*)(d.hdr ? d.hdr + kBTail : nullptr);
  d.org = (float*)(d.hdr ? d.hdr + kBTail + sizeof(int64_t) * (b->S + 1) : nullptr);
  d.pc = c.take<int64_t>(4);
  d.out = c.take<int64_t>(kBOut + 4 * SMKI_STAT_COPIES);   // results, then the counter copies
  d.stats = (unsigned long long*)(d.out ? d.out + kBOut : nullptr);
  d.nfree = c.take<int64_t>(n);
  d.off = c.take<int64_t>(n);
  d.kept = c.take<int32_t>(n);
  d.kpos = c.take<int32_t>(n);
  d.stmp_a = c.take<char>(scan_tmp_bytes(n));
  d.si = c.take<int32_t>(8);        // slots, targets, units; cleared with the marks
  d.mark = c.take<int32_t>(ne);
  d.mpos = c.take<int32_t>(ne);
  d.ext2t = c.take<int32_t>(ne);
  d.dense = c.take<int32_t>(b->g.n_blocks * m->K);
  d.slot_lin = c.take<int32_t>(NS);
  d.head = c.take<int32_t>(NS + 1);
  d.nun = c.take<int32_t>(NS);
  d.ust = c.take<int32_t>(NS);
  d.keys = c.take<char>(kw * R);
  d.akeys = c.take<char>(kw * R);
  d.idx = c.take<uint32_t>(R);
  d.aidx = c.take<uint32_t>(R);
  d.rec = c.take<float4>(R);
  d.flag = c.take<int32_t>(R);
  d.slot_excl = c.take<int32_t>(R);
  d.sort_tmp = c.take<char>(radix_tmp_bytes(R));
  d.scan_tmp = c.take<char>(scan_tmp_bytes(std::max(std::max(R, ne), NS)));
  d.wgbeam = c.take<int32_t>(free_sample_workgroups(R));
  d.cnt = c.take<int32_t>(8);       // cnt, active, contrib: cleared together
  d.active = c.take<int32_t>(ne);
  d.contrib = c.take<int32_t>(ntk);
  d.tgt = c.take<int32_t>(ne);
  d.tslot = c.take<int32_t>(ne);
  d.isnew = c.take<int32_t>(ne);
  d.rank = c.take<int32_t>(ne);
  d.ctmp = c.take<char>(scan_tmp_bytes(std::max<int64_t>(ntk, 1)));
  d.units = c.take<int4>(NU);
  d.part = c.take<float>(SMKI_PART_HEAD + (size_t)NU * DR3);
  d.umask = c.take<uint32_t>(NU);
  d.uorder = c.take<int32_t>(NU);
  d.sinfo = c.take<int4>(NS);
  d.need = c.take<int32_t>(ntk);
  d.cpos = c.take<int32_t>(ntk);
  return c.used;
}

// Fill the pinned input header of a replay.
void batch_header(smki_batch* b, const int64_t* offsets, const float* origins) {
  smki_map* m = b->m;
  char* h = b->h_in;
  memset(h, 0, kBBox);
  int64_t* f = (int64_t*)h;
  f[0] = m->host_counts_valid ? 1 : 0;   // else the device's counts are the current ones
  f[1] = m->n_blocks;
  f[2] = m->n_cblocks;
  bbox_init((int32_t*)(h + kBBox));
  memcpy(h + kBTail, offsets, sizeof(int64_t) * (b->S + 1));
  memcpy(h + kBTail + sizeof(int64_t) * (b->S + 1), origins, sizeof(float) * 3 * b->S);
}

// The whole insert with device-resident counts (recorded into the graph).
smki_status batch_enqueue(smki_batch* b, hipStream_t q) {
  smki_map* m = b->m;
  const BucketGeom& g = b->g;
  BatchBufs& d = b->d;
  const int64_t n = b->n, ne = b->n_ext, ntk = ne * m->K;
  SMKI_HIP_TRY(hipMemcpyAsync(d.hdr, b->h_in, b->in_bytes, hipMemcpyHostToDevice, q));
  SMKI_HIP_TRY(launch_batch_start((const int64_t*)d.hdr, m->dev.counts, d.stats, q));
  SMKI_HIP_TRY(launch_clear3(d.si, (int64_t)(d.mark + ne - d.si), d.cnt,
                             (int64_t)(d.contrib + ntk - d.cnt), d.dense, g.n_blocks * m->K, -1,
                             q));
  // first phase: validation, free-sample counts, their offsets
  SMKI_HIP_TRY(launch_count(b->xyz, b->label, nullptr, n, d.soff, d.org, b->S, m->res, b->step,
                            m->K, d.nfree, d.kept, d.bbox, d.err, q));
  SMKI_HIP_TRY(scan_excl_pair_i64_i32(d.nfree, d.off, n, d.sc, d.kept, d.kpos, n,
                                      (int32_t*)(d.sc + 1), d.stmp_a, q));
  SMKI_HIP_TRY(launch_batch_rows(d.sc, b->cap_rows, d.pc, d.err, q));
  // bucketing over the window's grid (rows outside it: SMKI_E_RANGE)
  PointSet ps{};
  ps.n = b->cap_rows;
  ps.dense = d.dense;
  ps.slot_lin = d.slot_lin;
  ps.head = d.head;
  ps.d_nslots = d.si;
  BucketScratch scr{};
  scr.keys = d.keys;
  scr.akeys = d.akeys;
  scr.idx = d.idx;
  scr.aidx = d.aidx;
  scr.rec = d.rec;
  scr.flag = d.flag;
  scr.slot_excl = d.slot_excl;
  scr.sort_tmp = d.sort_tmp;
  scr.scan_tmp = d.scan_tmp;
  SMKI_HIP_TRY(bucket_scan(b->xyz, b->label, nullptr, m->K, n, d.kept, d.kpos, n, d.off,
                           b->cap_rows, d.wgbeam, d.soff, d.org, b->S, b->step, m->free_class, g,
                           ps, scr, d.err, q, d.pc, (int32_t)b->cap_slots));
  SMKI_HIP_TRY(launch_mark_targets(ps.slot_lin, ps.d_nslots, (int32_t)b->cap_slots, g, b->eblo,
                                   b->enb, 1, d.mark, q));
  SMKI_HIP_TRY(launch_slot_units(ps.head, ps.d_nslots, (int32_t)b->cap_slots, m->chunk, d.nun, q));
  SMKI_HIP_TRY(scan_excl_pair_i32(d.mark, d.mpos, ne, d.si + 1, d.nun, d.ust, b->cap_slots,
                                  d.si + 2, d.scan_tmp, q, ps.d_nslots));
  SMKI_HIP_TRY(launch_batch_units(d.si, b->cap_slots, b->cap_units, d.err, q));
  // splat, allocation, merge
  const Stencil& sten = b->sten;
  const int64_t DR = m->B + 2 * sten.R;
  SplatArgs sa{};
  sa.g = g;
  sa.R = sten.R;
  sa.noff = (int32_t)sten.offs.size();
  sa.offs = (const int4*)b->d_offs;
  sa.cls = m->d_cls;
  for (int i = 0; i < SMKI_POLY_N; ++i) sa.mcoef[i] = (float)(kSmkiQ[i] / kSmkiQ[0]);
  sa.K = m->K;
  sa.chunk = m->chunk;
  sa.piece_mask = 0;
  for (int p = 0; p < 27; ++p) {
    const int nz = (p / 9 != 1) + ((p / 3) % 3 != 1) + (p % 3 != 1);
    if (m->selection == SMKI_SELECT_EXACT || nz <= 1) sa.piece_mask |= 1u << p;
  }
  sa.pts = d.rec;
  sa.wts = nullptr;
  sa.perm = d.idx;
  sa.dense = d.dense;
  sa.head = d.head;
  sa.slot_lin = d.slot_lin;
  sa.nunits = d.nun;
  sa.ustart = d.ust;
  for (int a = 0; a < 3; ++a) {
    sa.eblo[a] = b->eblo[a];
    sa.enb[a] = b->enb[a];
  }
  sa.ext2t = d.ext2t;
  sa.stats = d.stats;
  sa.tgt_elin = d.tgt;
  sa.tgt_active = d.active;
  sa.tgt_slot = d.tslot;
  sa.units = d.units;
  sa.uorder = d.uorder;
  sa.part = d.part;
  sa.part_elems = SMKI_PART_HEAD + (int64_t)b->cap_units * DR * DR * DR;
  sa.wide = (m->flags & SMKI_FLAG_WIDE_OFFSETS) ? 1 : 0;
  sa.umask = d.umask;
  sa.sinfo = d.sinfo;
  sa.n_slots = (int32_t)b->cap_slots;
  sa.contrib = d.contrib;
  sa.dn_slots = d.si;
  sa.dn_targets = d.si + 1;
  sa.dn_units = d.si + 2;
  sa.abort_word = d.err;
  sa.cap_units = (int32_t)b->cap_units;
  SMKI_HIP_TRY(launch_unit_table(d.nun, d.ust, d.head, d.slot_lin, g.n_blocks, m->chunk,
                                 (int32_t)b->cap_slots, ps.d_nslots, d.si + 2, d.units, d.uorder,
                                 q, (int32_t)b->cap_units));
  SMKI_HIP_TRY(launch_splat(sa, b->cap_units, q));
  SMKI_HIP_TRY(launch_list_targets(d.mark, d.mpos, ne, d.tgt, d.ext2t, q));
  SMKI_HIP_TRY(launch_slot_info(sa, q));
  SMKI_HIP_TRY(launch_contrib(sa, false, d.contrib, q));
  SMKI_HIP_TRY(launch_map_lookup(m->dev, sa, (int32_t)ne, d.tslot, d.isnew, q));
  SMKI_HIP_TRY(launch_need(m->dev, (int32_t)ne, d.contrib, d.isnew, d.tslot, d.need, d.cpos, q,
                           d.si + 1));
  SMKI_HIP_TRY(scan_excl_pair_i32(d.isnew, d.rank, ne, d.cnt, d.cpos, d.cpos, ne, d.cnt + 1,
                                  d.ctmp, q));
  SMKI_HIP_TRY(launch_batch_alloc_check(d.cnt, m->dev.counts, b->pool_cap, b->cpool_cap, b->hcap,
                                        d.err, q));
  SMKI_HIP_TRY(launch_assign(m->dev, sa, (int32_t)ne, d.isnew, d.rank, 0, d.tslot, d.need, d.cpos,
                             0, m->d_err, q));
  sa.map = m->dev;
  sa.alpha0 = m->alpha0;
  SMKI_HIP_TRY(launch_merge(sa, (int32_t)ne, q));
  SMKI_HIP_TRY(launch_batch_commit(d.cnt, m->dev.counts, d.err, m->d_err, d.pc, d.si, d.out, q));
  SMKI_HIP_TRY(hipMemcpyAsync(b->h_out, d.out, sizeof(int64_t) * (kBOut + 4 * SMKI_STAT_COPIES),
                              hipMemcpyDeviceToHost, q));
  return SMKI_OK;
}

void batch_release(smki_batch* b) {
  if (!b) return;
  if (b->launched && b->done) (void)hipEventSynchronize(b->done);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cs) (void)hipStreamDestroy(b->cs);
  if (b->done) (void)hipEventDestroy(b->done);
  dev_release(b->by, b->dbuf);
  if (b->d_offs) (void)hipFree(b->d_offs);
  if (b->h_in) (void)hipHostFree(b->h_in);
  if (b->h_out) (void)hipHostFree(b->h_out);
  if (b->m && b->m->stats_batch == b) b->m->stats_batch = nullptr;
  delete b;
}

bool batch_inputs_ok(const smki_map* m, int64_t n, const int64_t* offsets, const float* origins,
                     int32_t S) {
  if (offsets[0] != 0 || offsets[S] != n) return false;
  for (int32_t s = 0; s < S; ++s)
    if (offsets[s + 1] < offsets[s]) return false;
  for (int32_t s = 0; s < 3 * S; ++s) {
    if (!isfinite(origins[s])) return false;
    const float q = floorf((float)((double)origins[s] / (double)m->res));
    if (!(q >= -(float)SMKI_COORD_LIM && q < (float)SMKI_COORD_LIM)) return false;
  }
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* smki_status_string(smki_status s) {
  switch (s) {
    case SMKI_OK: return "ok";
    case SMKI_E_INVALID_ARG: return "invalid argument";
    case SMKI_E_OOM: return "device out of memory";
    case SMKI_E_CAPACITY: return "capacity exceeded";
    case SMKI_E_DEVICE: return "HIP runtime error";
    case SMKI_E_BAD_INPUT: return "bad input (label outside {-1..K-1} or non-finite coordinate)";
    case SMKI_E_RANGE: return "voxel index outside [-2^20, 2^20) or too many samples on a beam";
    default: return "unknown status";
  }
}

smki_status smki_create_map(float res, int32_t block_size, float l, float sigma0, int32_t K,
                            float alpha0, int32_t free_class, const smki_options* opt,
                            smki_map** out) {
  if (!out) return SMKI_E_INVALID_ARG;
  *out = nullptr;
  if (!finite_pos(res) || !finite_pos(l) || !finite_pos(sigma0) || !finite_pos(alpha0))
    return SMKI_E_INVALID_ARG;
  if (K < 2 || K > 255 || free_class < 0 || free_class >= K) return SMKI_E_INVALID_ARG;
  if (block_size < 1 || block_size > 32 || (block_size & (block_size - 1)) != 0)
    return SMKI_E_INVALID_ARG;
  if (opt && (opt->initial_blocks < 0 || opt->unit_budget < 0 || opt->unit_budget > (1 << 24) ||
              (opt->model != SMKI_MODEL_SBKI && opt->model != SMKI_MODEL_SCSM) ||
              (opt->selection != SMKI_SELECT_EXACT && opt->selection != SMKI_SELECT_FACE_BLOCKS) ||
              (opt->flags & ~SMKI_FLAG_WIDE_OFFSETS) != 0))
    return SMKI_E_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return SMKI_E_DEVICE;
  smki_map* m = new (std::nothrow) smki_map();
  if (!m) return SMKI_E_OOM;
  m->res = res;
  m->l = l;
  m->sigma0 = sigma0;
  m->alpha0 = alpha0;
  m->K = K;
  m->B = block_size;
  m->log2B = ilog2(block_size);
  m->free_class = free_class;
  m->chunk = (opt && opt->unit_budget > 0) ? opt->unit_budget : SMKI_CHUNK;
  m->model = opt ? opt->model : SMKI_MODEL_SBKI;
  m->selection = opt ? opt->selection : SMKI_SELECT_EXACT;
  m->flags = opt ? opt->flags : 0;
  (void)hipGetDevice(&m->device);
  m->dev.K = K;
  m->dev.B = block_size;
  m->dev.log2B = m->log2B;
  m->dev.alpha0 = alpha0;
  smki_status rc = SMKI_OK;
  if (hipMalloc((void**)&m->d_err, 64) != hipSuccess ||
      hipMalloc((void**)&m->d_stats, kStatAlloc) != hipSuccess ||
      hipMalloc((void**)&m->d_offs, sizeof(StencilOff) * SMKI_MAX_OFFS) != hipSuccess ||
      hipMalloc((void**)&m->d_cls, sizeof(float4) * K) != hipSuccess ||
      hipMalloc((void**)&m->dev.counts, sizeof(int64_t) * 2) != hipSuccess ||
      hipHostMalloc((void**)&m->h_pin, 8192, hipHostMallocDefault) != hipSuccess)
    rc = SMKI_E_OOM;
  for (int i = 0; rc == SMKI_OK && i < SMKI_TIMING_RING; ++i)
    for (int j = 0; j < 4; ++j)
      if (hipEventCreate(&m->evr[i][j]) != hipSuccess) rc = SMKI_E_OOM;
  if (rc == SMKI_OK && (hipMemset(m->d_err, 0, 64) != hipSuccess ||
                        hipMemset(m->dev.counts, 0, sizeof(int64_t) * 2) != hipSuccess))
    rc = SMKI_E_DEVICE;
  if (rc == SMKI_OK) {
    m->lk.assign(K, l);
    m->s0k.assign(K, sigma0);
    rc = upload_class_params(m);
  }
  const int64_t init_blocks = (opt && opt->initial_blocks > 0) ? opt->initial_blocks : 4096;
  if (rc == SMKI_OK) rc = ensure_pool(m, init_blocks);
  if (rc == SMKI_OK) rc = ensure_cpool(m, 2 * init_blocks);
  if (rc == SMKI_OK) rc = ensure_hash(m, 4096);
  if (rc == SMKI_OK && hipStreamSynchronize(m->stream) != hipSuccess) rc = SMKI_E_DEVICE;
  if (rc != SMKI_OK) {
    smki_destroy_map(m);
    return rc;
  }
  *out = m;
  return SMKI_OK;
}

smki_status smki_destroy_map(smki_map* m) {
  if (!m) return SMKI_E_INVALID_ARG;
  (void)hipStreamSynchronize(m->stream);
  dev_release(m->by_hash, m->dev.hkeys);
  dev_release(m->by_hash, m->dev.hvals);
  dev_release(m->by_pool, m->dev.bkeys);
  dev_release(m->by_pool, m->dev.cslot);
  dev_release(m->by_cpool, m->dev.calpha);
  if (m->d_err) (void)hipFree(m->d_err);
  if (m->d_stats) (void)hipFree(m->d_stats);
  if (m->d_offs) (void)hipFree(m->d_offs);
  if (m->d_cls) (void)hipFree(m->d_cls);
  if (m->dev.counts) (void)hipFree(m->dev.counts);
  if (m->h_pin) (void)hipHostFree(m->h_pin);
  if (m->h_hdr) (void)hipHostFree(m->h_hdr);
  for (auto& set : m->evr)
    for (hipEvent_t e : set)
      if (e) (void)hipEventDestroy(e);
  m->a_hits.release();
  m->a_sets.release();
  m->a_tgts.release();
  m->a_misc.release();
  delete m;
  return SMKI_OK;
}

smki_status smki_set_class_params(smki_map* m, const float* l, const float* sigma0) {
  if (!m || !l || !sigma0) return SMKI_E_INVALID_ARG;
  for (int32_t k = 0; k < m->K; ++k)
    if (!finite_pos(l[k]) || !finite_pos(sigma0[k])) return SMKI_E_INVALID_ARG;
  SMKI_HIP_TRY(hipSetDevice(m->device));
  m->lk.assign(l, l + m->K);
  m->s0k.assign(sigma0, sigma0 + m->K);
  ++m->epoch;   // a captured insert was sized for the old kernels
  return upload_class_params(m);
}

smki_status smki_set_allocator(smki_map* m, smki_alloc_fn alloc, smki_release_fn release,
                               void* ctx) {
  if (!m || (alloc == nullptr) != (release == nullptr)) return SMKI_E_INVALID_ARG;
  m->alloc_now.alloc = alloc;
  m->alloc_now.release = release;
  m->alloc_now.ctx = ctx;
  return SMKI_OK;
}

smki_status smki_set_stream(smki_map* m, void* hip_stream) {
  if (!m) return SMKI_E_INVALID_ARG;
  m->stream = (hipStream_t)hip_stream;
  return SMKI_OK;
}

smki_status smki_insert_scan(smki_map* m, const float* xyz, const int32_t* label, int64_t n,
                             const float* origin, float free_step) {
  if (!origin) return SMKI_E_INVALID_ARG;
  const int64_t off[2] = {0, n};
  return insert_impl(m, xyz, label, nullptr, n, off, origin, 1, free_step);
}

smki_status smki_insert_scan_soft(smki_map* m, const float* xyz, const float* probs, int64_t n,
                                  const float* origin, float free_step) {
  if (!origin) return SMKI_E_INVALID_ARG;
  const int64_t off[2] = {0, n};
  return insert_impl(m, xyz, nullptr, probs, n, off, origin, 1, free_step);
}

smki_status smki_insert_scans(smki_map* m, const float* xyz, const int32_t* label,
                              const int64_t* offsets, const float* origins, int32_t S,
                              float free_step) {
  if (!offsets || S < 1) return SMKI_E_INVALID_ARG;
  return insert_impl(m, xyz, label, nullptr, offsets[S], offsets, origins, S, free_step);
}

smki_status smki_query(smki_map* m, const int32_t* ijk, int64_t M, float* alpha, float* mean,
                       float* var, int32_t* label, float* p_occ) {
  if (!m || M < 0 || (M > 0 && !ijk)) return SMKI_E_INVALID_ARG;
  SMKI_HIP_TRY(launch_query(m->dev, ijk, M, alpha, mean, var, label, p_occ, m->free_class,
                            m->stream));
  return SMKI_OK;
}

smki_status smki_num_blocks(smki_map* m, int64_t* n_blocks) {
  if (!m || !n_blocks) return SMKI_E_INVALID_ARG;
  const smki_status rc = refresh_counts(m);
  if (rc != SMKI_OK) return rc;
  *n_blocks = m->n_blocks;
  return SMKI_OK;
}

smki_status smki_export(smki_map* m, int64_t capacity, int64_t* n_blocks, int32_t* block_ijk,
                        float* alpha) {
  if (!m || !n_blocks) return SMKI_E_INVALID_ARG;
  const smki_status rc = refresh_counts(m);
  if (rc != SMKI_OK) return rc;
  *n_blocks = m->n_blocks;
  if (!block_ijk && !alpha) return SMKI_OK;
  if (capacity < m->n_blocks) return SMKI_E_CAPACITY;
  const int64_t n = m->n_blocks;
  if (n == 0) return SMKI_OK;
  Sizer z;
  z.add<uint64_t>(n);
  z.add<uint64_t>(n);
  z.add<uint32_t>(n);
  z.add<uint32_t>(n);
  z.add<char>(radix_tmp_bytes(n));
  SMKI_HIP_TRY(m->a_misc.reserve(z.total, m->alloc_now));
  uint64_t* k = m->a_misc.take<uint64_t>(n);
  uint64_t* k2 = m->a_misc.take<uint64_t>(n);
  uint32_t* o = m->a_misc.take<uint32_t>(n);
  uint32_t* o2 = m->a_misc.take<uint32_t>(n);
  void* tmp = m->a_misc.take<char>(radix_tmp_bytes(n));
  SMKI_HIP_TRY(hipMemcpyAsync(k, m->dev.bkeys, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice,
                              m->stream));
  SMKI_HIP_TRY(launch_iota_u32(o, n, m->stream));
  SMKI_HIP_TRY(radix_sort_u64(k, o, k2, o2, n, 63, tmp, m->stream));
  if (block_ijk) SMKI_HIP_TRY(launch_block_keys_to_ijk(k, n, block_ijk, m->stream));
  if (alpha) SMKI_HIP_TRY(launch_gather_blocks(m->dev, o, n, alpha, m->stream));
  SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
  return SMKI_OK;
}

smki_status smki_import(smki_map* m, int64_t n, const int32_t* block_ijk, const float* alpha) {
  if (!m || n < 0 || (n > 0 && (!block_ijk || !alpha))) return SMKI_E_INVALID_ARG;
  SMKI_HIP_TRY(hipSetDevice(m->device));
  if (n == 0) {   // empty the map: no check, no synchronisation
    SMKI_HIP_TRY(launch_hash_clear(m->dev, m->stream));
    m->n_blocks = 0;
    m->n_cblocks = 0;
    m->host_counts_valid = true;   // (installed on the device by the next replay)
    return SMKI_OK;
  }
  {
    const smki_status rc0 = refresh_counts(m);
    if (rc0 != SMKI_OK) return rc0;
  }
  const int64_t nk = n * m->K;
  if (nk > (int64_t)INT32_MAX / 2) return SMKI_E_CAPACITY;
  // Validate and size everything in scratch first: the block keys (range
  // checked), a sorted copy of them (duplicates), and the class blocks to keep
  // (pairs holding a value other than alpha0).  The map is touched only after
  // all of that succeeded, so a failed import leaves it unchanged.
  Sizer z;
  z.add<int32_t>(4);
  z.add<uint64_t>(n);
  z.add<uint64_t>(n);
  z.add<uint64_t>(n);
  z.add<uint32_t>(n);
  z.add<uint32_t>(n);
  z.add<char>(radix_tmp_bytes(n));
  z.add<int32_t>(nk);
  z.add<int32_t>(nk);
  z.add<char>(scan_tmp_bytes(nk));
  SMKI_HIP_TRY(m->a_misc.reserve(z.total, m->alloc_now));
  Arena& Z = m->a_misc;
  int32_t* hdr = Z.take<int32_t>(4);   // [0] error word, [1] class blocks
  uint64_t* keys = Z.take<uint64_t>(n);
  uint64_t* skeys = Z.take<uint64_t>(n);
  uint64_t* k2 = Z.take<uint64_t>(n);
  uint32_t* o = Z.take<uint32_t>(n);
  uint32_t* o2 = Z.take<uint32_t>(n);
  void* stmp = Z.take<char>(radix_tmp_bytes(n));
  int32_t* flag = Z.take<int32_t>(nk);
  int32_t* pos = Z.take<int32_t>(nk);
  void* tmp = Z.take<char>(scan_tmp_bytes(nk));
  hipStream_t q = m->stream;
  SMKI_HIP_TRY(launch_fill_i32(hdr, 4, 0, q));
  SMKI_HIP_TRY(launch_ijk_to_block_keys(block_ijk, n, m->log2B, keys, (uint32_t*)hdr, q));
  SMKI_HIP_TRY(hipMemcpyAsync(skeys, keys, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, q));
  SMKI_HIP_TRY(launch_iota_u32(o, n, q));
  SMKI_HIP_TRY(radix_sort_u64(skeys, o, k2, o2, n, 63, stmp, q));
  SMKI_HIP_TRY(launch_adjacent_dups(skeys, n, (uint32_t*)hdr, q));
  SMKI_HIP_TRY(launch_import_flags(m->dev, alpha, n, flag, q));
  SMKI_HIP_TRY(scan_excl_i32(flag, pos, nk, hdr + 1, tmp, q));
  int32_t h[2];
  SMKI_HIP_TRY(sync_read(m, hdr, sizeof(h), h));
  if (h[0]) return status_of_err((uint32_t)h[0]);
  const int64_t nc = h[1];
  // capacity (growth keeps the current contents, so a failure here leaves the
  // map as it was)
  smki_status rc = ensure_pool(m, n);
  if (rc != SMKI_OK) return rc;
  rc = ensure_cpool(m, std::max<int64_t>(nc, 1));
  if (rc != SMKI_OK) return rc;
  rc = ensure_hash(m, n);
  if (rc != SMKI_OK) return rc;
  // commit: block i of the input is pool slot i
  SMKI_HIP_TRY(hipMemcpyAsync(m->dev.bkeys, keys, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice,
                              q));
  SMKI_HIP_TRY(launch_import_copy(m->dev, alpha, n, flag, pos, 0, q));
  SMKI_HIP_TRY(launch_hash_clear(m->dev, q));
  SMKI_HIP_TRY(launch_hash_insert_slots(m->dev, 0, n, m->d_err, q));
  m->n_blocks = n;
  m->n_cblocks = nc;
  SMKI_HIP_TRY(stream_wait(q));
  return SMKI_OK;
}

smki_status smki_last_scan_stats(smki_map* m, smki_scan_stats* out) {
  if (!m || !out) return SMKI_E_INVALID_ARG;
  if (m->stats_pending && m->stats_batch) {   // the last insert was a replay
    smki_batch* b = m->stats_batch;
    SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
    const int64_t* o = b->h_out;
    const unsigned long long* c = (const unsigned long long*)(o + kBOut);
    unsigned long long s[4] = {0, 0, 0, 0};
    for (int k = 0; k < SMKI_STAT_COPIES; ++k)
      for (int i = 0; i < 4; ++i) s[i] += c[k * 4 + i];
    smki_scan_stats st{};
    st.n_hits = o[4];
    st.n_free = o[5];
    st.n_point_blocks = o[6];
    st.n_target_blocks = o[7];
    st.n_units = o[8];
    st.n_new_blocks = o[1];
    st.n_new_class_blocks = o[2];
    st.n_updated_voxels = o[0] ? 0 : (int64_t)s[0];
    st.n_pairs = (int64_t)s[1];
    st.n_candidates = o[3] * (int64_t)b->sten.offs.size();
    st.n_lane_slots =
        o[3] * (int64_t)SMKI_WAVE * ((int64_t)(b->sten.offs.size() + SMKI_WAVE - 1) / SMKI_WAVE);
    m->last = st;
    m->stats_pending = false;
  }
  if (m->stats_pending) {
    // the last insert's counters (left on the device: no insert since), summed
    SMKI_HIP_TRY(sync_read(m, m->d_stats, kStatAlloc, m->h_pin + 256));
    const unsigned long long* c = (const unsigned long long*)(m->h_pin + 256);
    unsigned long long s[4] = {0, 0, 0, 0};
    for (int k = 0; k < SMKI_STAT_COPIES; ++k)
      for (int i = 0; i < 4; ++i) s[i] += c[k * 4 + i];
    m->last.n_updated_voxels = (int64_t)s[0];
    m->last.n_pairs = (int64_t)s[1];
    if (m->new_pending) {
      const int32_t* nc = (const int32_t*)(m->h_pin + kPinNew);
      m->last.n_new_blocks = nc[0];
      m->last.n_new_class_blocks = nc[1];
      m->new_pending = false;
    }
    float ms = 0.0f;
    if (m->last_timed) {
      if (hipEventElapsedTime(&ms, m->ev[0], m->ev[1]) == hipSuccess) m->last.splat_ms = ms;
      if (hipEventElapsedTime(&ms, m->ev[2], m->ev[3]) == hipSuccess) m->last.merge_ms = ms;
    }
    m->stats_pending = false;
  }
  *out = m->last;
  return SMKI_OK;
}

smki_status smki_kernel_times(smki_map* m, int32_t max, float* splat_ms, float* merge_ms,
                              int32_t* count) {
  if (!m || max < 0 || !count || (max > 0 && (!splat_ms || !merge_ms))) return SMKI_E_INVALID_ARG;
  SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
  const int64_t have = std::min<int64_t>(m->n_timed, SMKI_TIMING_RING);
  const int64_t k = std::min<int64_t>(have, max);
  for (int64_t i = 0; i < k; ++i) {   // oldest first
    hipEvent_t* e = m->evr[(m->n_timed - k + i) % SMKI_TIMING_RING];
    SMKI_HIP_TRY(hipEventElapsedTime(&splat_ms[i], e[0], e[1]));
    SMKI_HIP_TRY(hipEventElapsedTime(&merge_ms[i], e[2], e[3]));
  }
  *count = (int32_t)k;
  return SMKI_OK;
}

smki_status smki_set_kernel_timing(smki_map* m, int32_t enable) {
  if (!m) return SMKI_E_INVALID_ARG;
  m->timing = enable != 0;
  return SMKI_OK;
}

smki_status smki_sync(smki_map* m) {
  if (!m) return SMKI_E_INVALID_ARG;
  SMKI_HIP_TRY(hipStreamSynchronize(m->stream));
  const smki_status rc = refresh_counts(m);
  if (rc != SMKI_OK) return rc;
  return take_device_error(m);
}

smki_status smki_free_samples(const float* xyz, const int32_t* label, int64_t n, const float* origin,
                              float free_step, int32_t K, void* hip_stream, int64_t* n_out,
                              float* out_xyz, int64_t* out_parent) {
  if (!n_out || !origin || n < 0 || (n > 0 && (!xyz || !label)) || K < 1 || K > 255 ||
      !isfinite(free_step))
    return SMKI_E_INVALID_ARG;
  hipStream_t q = (hipStream_t)hip_stream;
  *n_out = 0;
  if (n == 0) return SMKI_OK;
  Sizer z;
  z.add<int64_t>(2);
  z.add<float>(4);
  z.add<int64_t>(n);
  z.add<int64_t>(n);
  z.add<int32_t>(n);
  z.add<int32_t>(kBboxInts);
  z.add<uint32_t>(1);
  z.add<int64_t>(2);
  z.add<char>(scan_tmp_bytes(n));
  char* base = nullptr;
  SMKI_HIP_TRY(hipMallocAsync((void**)&base, z.total, q));
  Arena A;
  A.base = base;
  A.cap = z.total;
  int64_t* soff = A.take<int64_t>(2);
  float* org = A.take<float>(4);
  int64_t* nfree = A.take<int64_t>(n);
  int64_t* off = A.take<int64_t>(n);
  int32_t* kept = A.take<int32_t>(n);
  int32_t* bbox = A.take<int32_t>(kBboxInts);
  uint32_t* err = A.take<uint32_t>(1);
  int64_t* tot = A.take<int64_t>(2);
  void* tmp = A.take<char>(scan_tmp_bytes(n));
  const int64_t so[2] = {0, n};
  std::vector<int32_t> bbox0(kBboxInts);
  bbox_init(bbox0.data());
  smki_status rc = SMKI_OK;
  hipError_t e = hipMemcpyAsync(soff, so, sizeof(so), hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = hipMemcpyAsync(org, origin, sizeof(float) * 3, hipMemcpyHostToDevice, q);
  if (e == hipSuccess)
    e = hipMemcpyAsync(bbox, bbox0.data(), sizeof(int32_t) * kBboxInts, hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = hipMemsetAsync(err, 0, sizeof(uint32_t), q);
  if (e == hipSuccess)
    e = launch_count(xyz, label, nullptr, n, soff, org, 1, 3.0e38f, free_step, K, nfree, kept,
                     bbox, err, q);
  if (e == hipSuccess) e = scan_excl_i64(nfree, off, n, tot, tmp, q);
  int64_t h[2] = {0, 0};
  uint32_t herr = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(h, tot, sizeof(int64_t), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  if (e != hipSuccess) rc = smki_hip_error(e);
  // the resolution used above (3e38) only feeds an unused bounding box
  if (rc == SMKI_OK && herr) rc = status_of_err(herr);
  if (rc == SMKI_OK) {
    *n_out = h[0];
    if (out_xyz) {
      e = launch_free_xyz(xyz, n, off, h[0], org, free_step, out_xyz, out_parent, q);
      if (e == hipSuccess) e = hipStreamSynchronize(q);
      if (e != hipSuccess) rc = smki_hip_error(e);
    }
  }
  (void)hipFreeAsync(base, q);
  (void)hipStreamSynchronize(q);
  return rc;
}

smki_status smki_bucket_cells(const float* xyz, int64_t n, float res, int32_t block_size,
                              void* hip_stream, int64_t* n_cells, uint64_t* cell_keys,
                              int32_t* cell_start, int32_t* cell_count, int32_t* order) {
  if (!n_cells || n < 0 || (n > 0 && !xyz) || !finite_pos(res) ||
      (block_size != 4 && block_size != 8 && block_size != 16 && block_size != 32))
    return SMKI_E_INVALID_ARG;
  if (n > (int64_t)INT32_MAX / 2) return SMKI_E_CAPACITY;
  hipStream_t q = (hipStream_t)hip_stream;
  *n_cells = 0;
  if (n == 0) return SMKI_OK;
  // bounding box pass (labels are not needed: validate with an all-valid label)
  smki_map tmp_map{};
  tmp_map.res = res;
  tmp_map.B = block_size;
  tmp_map.log2B = ilog2(block_size);
  Sizer z0;
  z0.add<int32_t>(kBboxInts);
  z0.add<uint32_t>(1);
  z0.add<int64_t>(n);
  z0.add<int32_t>(n);
  z0.add<int32_t>(n);
  z0.add<int64_t>(2);
  z0.add<float>(4);
  char* base0 = nullptr;
  SMKI_HIP_TRY(hipMallocAsync((void**)&base0, z0.total, q));
  Arena A0;
  A0.base = base0;
  A0.cap = z0.total;
  int32_t* bbox = A0.take<int32_t>(kBboxInts);
  uint32_t* err = A0.take<uint32_t>(1);
  int64_t* nfree = A0.take<int64_t>(n);
  int32_t* kept = A0.take<int32_t>(n);
  int32_t* lab = A0.take<int32_t>(n);
  int64_t* soff = A0.take<int64_t>(2);
  float* org = A0.take<float>(4);
  std::vector<int32_t> bbox0(kBboxInts), hbb(kBboxInts);
  bbox_init(bbox0.data());
  const int64_t so[2] = {0, n};
  const float o0[4] = {0, 0, 0, 0};
  hipError_t e =
      hipMemcpyAsync(bbox, bbox0.data(), sizeof(int32_t) * kBboxInts, hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = hipMemcpyAsync(soff, so, sizeof(so), hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = hipMemcpyAsync(org, o0, sizeof(o0), hipMemcpyHostToDevice, q);
  if (e == hipSuccess) e = hipMemsetAsync(err, 0, sizeof(uint32_t), q);
  if (e == hipSuccess) e = hipMemsetAsync(lab, 0, sizeof(int32_t) * n, q);
  if (e == hipSuccess)
    e = launch_count(xyz, lab, nullptr, n, soff, org, 1, res, 0.0f, 1, nfree, kept, bbox, err, q);
  int32_t hb[6];
  uint32_t herr = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(hbb.data(), bbox, sizeof(int32_t) * kBboxInts, hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  (void)hipFreeAsync(base0, q);
  if (e != hipSuccess) return smki_hip_error(e);
  if (herr) return status_of_err(herr);
  bbox_reduce(hbb.data(), hb);
  const BucketGeom g = make_geom(&tmp_map, hb, hb + 3, 1);
  if (g.n_blocks > (int64_t(1) << 28)) return SMKI_E_CAPACITY;
  Sizer z;
  z.add<uint64_t>(n);
  z.add<uint64_t>(n);
  z.add<uint32_t>(n);
  z.add<uint32_t>(n);
  z.add<float4>(n);
  z.add<int32_t>(n);
  z.add<int32_t>(n);
  z.add<char>(radix_tmp_bytes(n));
  z.add<char>(scan_tmp_bytes(n));
  z.add<int32_t>(2);
  z.add<uint32_t>(1);
  char* base = nullptr;
  SMKI_HIP_TRY(hipMallocAsync((void**)&base, z.total, q));
  Arena A;
  A.base = base;
  A.cap = z.total;
  BucketScratch scr{};
  scr.keys = A.take<uint64_t>(n);
  scr.akeys = A.take<uint64_t>(n);
  scr.idx = A.take<uint32_t>(n);
  scr.aidx = A.take<uint32_t>(n);
  scr.rec = A.take<float4>(n);
  scr.flag = A.take<int32_t>(n);
  scr.slot_excl = A.take<int32_t>(n);
  scr.sort_tmp = A.take<char>(radix_tmp_bytes(n));
  scr.scan_tmp = A.take<char>(scan_tmp_bytes(n));
  int32_t* d_nc = A.take<int32_t>(2);
  uint32_t* err2 = A.take<uint32_t>(1);
  smki_status rc = SMKI_OK;
  int32_t nc = 0;
  e = hipMemsetAsync(d_nc, 0, sizeof(int32_t) * 2, q);
  if (e == hipSuccess) e = hipMemsetAsync(err2, 0, sizeof(uint32_t), q);
  if (e == hipSuccess) e = bucket_cells_sort(xyz, n, g, scr, err2, d_nc, q);
  if (e == hipSuccess) e = hipMemcpyAsync(&nc, d_nc, sizeof(int32_t), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err2, sizeof(uint32_t), hipMemcpyDeviceToHost, q);
  if (e == hipSuccess) e = hipStreamSynchronize(q);
  if (e != hipSuccess) rc = smki_hip_error(e);
  if (rc == SMKI_OK && herr) rc = status_of_err(herr);
  if (rc == SMKI_OK) {
    *n_cells = nc;
    if (cell_keys && cell_start && cell_count) {
      e = bucket_cells_table(n, nc, g, scr, cell_keys, cell_start, cell_count, order, q);
      if (e == hipSuccess) e = hipStreamSynchronize(q);
      if (e != hipSuccess) rc = smki_hip_error(e);
    }
  }
  (void)hipFreeAsync(base, q);
  (void)hipStreamSynchronize(q);
  return rc;
}

size_t smki_loss_workspace_bytes(int64_t n_train, int64_t n_query, int32_t K);

smki_status smki_batch_capture(smki_map* m, const float* xyz, const int32_t* label,
                               const int64_t* offsets, const float* origins, int32_t S,
                               float free_step, float margin, smki_batch** out) {
  if (!out) return SMKI_E_INVALID_ARG;
  *out = nullptr;
  if (!m || !offsets || !origins || S < 1 || !(margin >= 0.0f && margin <= 16.0f) ||
      !isfinite(free_step) || offsets[S] < 1 || !xyz || !label)
    return SMKI_E_INVALID_ARG;
  if (m->model != SMKI_MODEL_SBKI) return SMKI_E_INVALID_ARG;
  const int64_t n = offsets[S];
  if (!batch_inputs_ok(m, n, offsets, origins, S)) return SMKI_E_INVALID_ARG;
  // 1. the ordinary insert of these scans (it sizes everything)
  smki_status rc = insert_impl(m, xyz, label, nullptr, n, offsets, origins, S, free_step);
  if (rc == SMKI_OK) rc = refresh_counts(m);   // (the insert leaves them on the device)
  smki_scan_stats st{};
  if (rc == SMKI_OK) rc = smki_last_scan_stats(m, &st);
  if (rc != SMKI_OK) return rc;
  if (st.n_hits == 0) return SMKI_E_INVALID_ARG;   // nothing to size the capture by
  smki_batch* b = new (std::nothrow) smki_batch();
  if (!b) return SMKI_E_OOM;
  b->m = m;
  b->xyz = xyz;
  b->label = label;
  b->n = n;
  b->S = S;
  b->step = free_step;
  const double grow = 1.0 + (double)margin;
  // 2. the window: the voxel box of that insert grown by margin of its extent per
  // side (at least two blocks), narrowed while that would widen the row keys
  // past 32 bits (or past the insert's own key width)
  const int kb0 = make_geom(m, m->last_vlo, m->last_vhi, m->K).key_bits;
  int64_t pad[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t ext = (int64_t)m->last_vhi[a] - m->last_vlo[a] + 1;
    pad[a] = std::max<int64_t>(2 * m->B, (int64_t)ceil(margin * ext));
  }
  int32_t wlo[3], whi[3];
  int64_t maxabs = 0;
  for (;;) {
    maxabs = 0;
    for (int a = 0; a < 3; ++a) {
      wlo[a] = (int32_t)std::max<int64_t>(m->last_vlo[a] - pad[a], -SMKI_COORD_LIM);
      whi[a] = (int32_t)std::min<int64_t>(m->last_vhi[a] + pad[a], SMKI_COORD_LIM - 1);
      maxabs = std::max<int64_t>(maxabs, std::max(std::abs((int64_t)wlo[a]), std::abs((int64_t)whi[a])));
    }
    b->g = make_geom(m, wlo, whi, m->K);
    bool shrink = false;
    for (int a = 0; a < 3; ++a) shrink = shrink || pad[a] > 2 * m->B;
    if (b->g.key_bits <= std::max(32, kb0) || !shrink) break;
    for (int a = 0; a < 3; ++a) pad[a] = std::max<int64_t>(2 * m->B, pad[a] / 2);
  }
  const BucketGeom& g = b->g;
  b->n_ext = 1;
  for (int a = 0; a < 3; ++a) {
    b->eblo[a] = g.blo[a] - 1;
    b->enb[a] = g.nb[a] + 2;
    b->n_ext *= b->enb[a];
  }
  const double lv = (double)max_class_l(m) / (double)m->res;
  const double smargin = std::max(1e-4, 4.0 * ldexp((double)maxabs + 1.0, -23));
  b->sten = make_stencil(lv, smargin);
  // 3. capacities
  b->cap_rows = std::max<int64_t>(n, (int64_t)ceil((double)(st.n_hits + st.n_free) * grow)) + 4096;
  b->cap_slots = std::min<int64_t>(std::min<int64_t>(b->cap_rows, g.n_blocks * m->K),
                                   (int64_t)ceil((double)st.n_point_blocks * grow) + 1024);
  b->cap_units = (int64_t)ceil((double)st.n_units * grow) + 1024;
  const int64_t DR = m->B + 2 * b->sten.R;
  // keep the partial sums under 4 GiB and 2^24 units (32-bit offsets in the
  // merge) when the sizing insert's fitted
  const int64_t narrow_units =
      std::min<int64_t>(((int64_t(1) << 32) - 4 * SMKI_PART_HEAD) / (int64_t)(sizeof(float) * DR * DR * DR),
                        (int64_t(1) << 24) - 1);
  if (st.n_units <= narrow_units && !(m->flags & SMKI_FLAG_WIDE_OFFSETS))
    b->cap_units = std::min(b->cap_units, narrow_units);
  if (g.n_blocks * m->K > (int64_t(1) << 30) || b->n_ext > (int64_t(1) << 30) ||
      b->n_ext * m->K > (int64_t)INT32_MAX / 2 || b->cap_rows > (int64_t)INT32_MAX - 1 ||
      !sbki_shape_ok(m->B, b->sten.R) ||
      (double)b->cap_units * DR * DR * DR * sizeof(float) > 64.0 * (1ull << 30)) {
    delete b;
    return SMKI_E_CAPACITY;
  }
  // room in the map for the replays: the blocks and class blocks of this
  // insert again, plus margin, on top of what the map holds now
  rc = ensure_pool(m, (int64_t)ceil((double)(m->n_blocks + st.n_new_blocks) * grow) + 64);
  if (rc == SMKI_OK)
    rc = ensure_cpool(m, (int64_t)ceil((double)(m->n_cblocks + st.n_new_class_blocks) * grow) + 64);
  if (rc == SMKI_OK) rc = ensure_hash(m, m->pool_cap);
  if (rc != SMKI_OK) {
    delete b;
    return rc;
  }
  b->pool_cap = m->pool_cap;
  b->cpool_cap = m->cpool_cap;
  b->hcap = m->dev.hcap;
  // 4. buffers, stencil, header
  b->in_bytes = kBTail + sizeof(int64_t) * (S + 1) + sizeof(float) * 3 * S;
  const size_t dbytes = carve_batch(b, nullptr) + kAlign;
  hipError_t e = dev_alloc(m->alloc_now, (void**)&b->dbuf, dbytes);
  b->by = m->alloc_now;
  if (e == hipSuccess)
    e = hipMalloc((void**)&b->d_offs, sizeof(StencilOff) * std::max<size_t>(b->sten.offs.size(), 1));
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_in, b->in_bytes, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&b->h_out, sizeof(int64_t) * (kBOut + 4 * SMKI_STAT_COPIES),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_offs, b->sten.offs.data(), sizeof(StencilOff) * b->sten.offs.size(),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    batch_release(b);
    return smki_hip_error(e);
  }
  carve_batch(b, (char*)(((uintptr_t)b->dbuf + kAlign - 1) / kAlign * kAlign));
  batch_header(b, offsets, origins);
  // 5. record the insert (nothing runs now)
  e = hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    batch_release(b);
    return smki_hip_error(e);
  }
  rc = batch_enqueue(b, b->cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(b->cs, &graph);
  b->graph = graph;
  if (rc == SMKI_OK && e != hipSuccess) rc = smki_hip_error(e);
  if (rc == SMKI_OK) {
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = smki_hip_error(e);
  }
  if (rc != SMKI_OK) {
    batch_release(b);
    return rc;
  }
  b->epoch = m->epoch;
  *out = b;
  return SMKI_OK;
}

smki_status smki_batch_replay(smki_batch* b, const int64_t* offsets, const float* origins) {
  if (!b || !offsets || !origins) return SMKI_E_INVALID_ARG;
  smki_map* m = b->m;
  if (!batch_inputs_ok(m, b->n, offsets, origins, b->S)) return SMKI_E_INVALID_ARG;
  if (m->epoch != b->epoch) return SMKI_E_CAPACITY;   // the map's storage moved: capture again
  SMKI_HIP_TRY(hipSetDevice(m->device));
  // the previous replay has read its header before this one is written
  if (b->launched) SMKI_HIP_TRY(hipEventSynchronize(b->done));
  batch_header(b, offsets, origins);
  SMKI_HIP_TRY(hipGraphLaunch(b->exec, m->stream));
  SMKI_HIP_TRY(hipEventRecord(b->done, m->stream));
  b->launched = true;
  m->host_counts_valid = false;
  m->stats_batch = b;
  m->stats_pending = true;
  return SMKI_OK;
}

smki_status smki_batch_destroy(smki_batch* b) {
  if (!b) return SMKI_E_INVALID_ARG;
  batch_release(b);
  return SMKI_OK;
}

}  // extern "C"
