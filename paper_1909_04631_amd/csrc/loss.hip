// Differentiable form: the S-BKI concentrations (Eq. (7)-(8) of Gan et al.,
// arXiv 1909.04631) at arbitrary labelled query points, the mean negative log
// predictive probability of their labels, and its adjoint with respect to the
// kernel length-scale l, the kernel scale sigma0 and every coordinate.
//
//   alpha_h^k = alpha0 + sum_t sigma0 f(r_ht) [y_t = k],  r = |x_t - x_h| / l < 1
//   loss      = -(1/H) sum_h log(alpha_h^{y_h} / S_h),     S_h = sum_k alpha_h^k
//   G_hk      = dloss/dalpha_hk = -(1/H)([k = y_h] / alpha_hk - 1/S_h)
//   dloss/dl      = sum over pairs  G_{h,y_t} sigma0 f'(r) (-r/l)
//   dloss/dsigma0 = sum_h sum_k G_hk (alpha_hk - alpha0) / sigma0      (closed form)
//   dloss/dx_t    = sum_h G_{h,y_t} sigma0 (f'(r)/r) (x_t - x_h) / l^2, dloss/dx_h = -(same)
//
// Rows and queries are bucketed in cells slightly larger than l, so a point's
// support lies in its own cell and the 26 around it.  Kernel weights are
// recomputed in the backward pass; nothing per pair is stored.  Each query (or
// training row) is owned by one lane; scalar gradients are reduced in double
// in a fixed order (deterministic, no floating-point atomics).
#include <algorithm>
#include <cmath>
#include <mutex>

#include "smki_gather.h"
#include "../../include/smki.h"

namespace {

constexpr int LB = 4;       // cells per block edge of the loss grid
constexpr int LLOG2B = 2;
constexpr int64_t kMaxLossBlocks = int64_t(1) << 22;

// f'(r)/r = s^4 P(s), s = 1 - r: P is a relative degree-10 fit on s in [0, 1]
// (error 1.5e-8) of [f'(1 - s)/s^4]/(1 - s), the series f'(1 - s) = sum_{n>=2}
// (-1)^(n+1) (2n-2) (2 pi)^(2n) s^(2n) / (3 (2n)!) divided by s^4 r;
// kernel_poly.py derives it.  Highest degree first.
__constant__ float kG[11] = {0.826695529413764f,  0.8883087167660566f, -18.68107694361095f,
                             33.6151725453642f,   12.821709617420272f, -46.914955742370914f,
                             -50.511732012322824f, 70.73862871627226f, 70.64347982896255f,
                             -43.2927725732048f,  -43.292930014879026f};

struct LossArgs {
  BucketGeom g;
  const float4* pts;     // sorted records of the set being walked (label bits in .w)
  const int32_t* dense;
  const int32_t* prefix;
  const int32_t* sidx;   // sorted position -> original row of the walked set
  float l, l2, inv_l, sigma0, alpha0;
  float coef[SMKI_POLY_N];  // sigma0 * Q (per-class form: Q, the class's sigma0 applied apart)
  int32_t K;
  int64_t H;
  const float4* cls;        // per-class form: [K] (l^2, 1/l, sigma0, l) of each class's kernel;
                            // l, l2 and inv_l above then hold the largest l (the search cut)
};

__device__ __forceinline__ float kernel_weight(const float* c, float s) {
  const float u = s * s;
  float q = c[0];
#pragma unroll
  for (int i = 1; i < SMKI_POLY_N; ++i) q = fmaf(q, u, c[i]);
  return (u * u) * (s * q);
}

__device__ __forceinline__ float dfdr_over_r(float s) {
  float p = kG[0];
#pragma unroll
  for (int i = 1; i < 11; ++i) p = fmaf(p, s, kG[i]);
  const float s2 = s * s;
  return (s2 * s2) * p;
}

__device__ __forceinline__ int cell_of(float x, float h) {
  return (int)floorf((float)((double)x / (double)h));
}

// Visit every row of the walked set in the 27 cells around point x (row ranges
// from the prefix tables); fn(record, dx, dy, dz, d2, sorted index).
template <typename Fn>
__device__ __forceinline__ void for_neighbours(const LossArgs& a, float x, float y, float z, Fn fn) {
  const BucketGeom& g = a.g;
  const int cx = cell_of(x, g.res), cy = cell_of(y, g.res), cz = cell_of(z, g.res);
  const int32_t B3 = LB * LB * LB;
  const double h = (double)g.res;
  for (int ox = -1; ox <= 1; ++ox)
    for (int oy = -1; oy <= 1; ++oy)
      for (int oz = -1; oz <= 1; ++oz) {
        const int vx = cx + ox, vy = cy + oy, vz = cz + oz;
        const int bx = vx >> LLOG2B, by = vy >> LLOG2B, bz = vz >> LLOG2B;
        const int px = bx - g.blo[0], py = by - g.blo[1], pz = bz - g.blo[2];
        if (px < 0 || py < 0 || pz < 0 || px >= g.nb[0] || py >= g.nb[1] || pz >= g.nb[2]) continue;
        const int32_t slot = a.dense[((int64_t)px * g.nb[1] + py) * g.nb[2] + pz];
        if (slot < 0) continue;
        const int32_t loc = ((vx - bx * LB) * LB + (vy - by * LB)) * LB + (vz - bz * LB);
        const int32_t* P = a.prefix + (int64_t)slot * (B3 + 1);
        const int32_t S = P[loc], E = P[loc + 1];
        if (S == E) continue;
        // the point relative to the exact centre of block (bx, by, bz)
        const float qx = (float)((double)x - ((double)(bx * LB) + 0.5 * LB) * h);
        const float qy = (float)((double)y - ((double)(by * LB) + 0.5 * LB) * h);
        const float qz = (float)((double)z - ((double)(bz * LB) + 0.5 * LB) * h);
        for (int32_t i = S; i < E; ++i) {
          const float4 p = a.pts[i];
          const float dx = p.x - qx, dy = p.y - qy, dz = p.z - qz;
          const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          if (d2 < a.l2) fn(p, dx, dy, dz, d2, i);
        }
      }
}

__global__ void k_validate(const float* __restrict__ xyz, const int32_t* __restrict__ lab,
                           int64_t n, int32_t K, float h, int32_t* __restrict__ bbox,
                           uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
  if (lab[i] < 0 || lab[i] >= K) atomicOr(err, DEVERR_LABEL);
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
    atomicOr(err, DEVERR_NONFINITE);
    return;
  }
  const float c[3] = {floorf((float)((double)x / (double)h)), floorf((float)((double)y / (double)h)),
                      floorf((float)((double)z / (double)h))};
  for (int a = 0; a < 3; ++a) {
    if (!(c[a] >= -(float)SMKI_COORD_LIM && c[a] < (float)SMKI_COORD_LIM)) {
      atomicOr(err, DEVERR_RANGE);
      return;
    }
  }
  for (int a = 0; a < 3; ++a) {
    atomicMin(&bbox[a], (int32_t)c[a]);
    atomicMax(&bbox[3 + a], (int32_t)c[a]);
  }
}

// alpha at each query, in query order.
__global__ void k_alpha_q(LossArgs a, const float* __restrict__ qxyz, float* __restrict__ alpha_q) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.H) return;
  float* A = alpha_q + h * a.K;
  for (int k = 0; k < a.K; ++k) A[k] = a.alpha0;
  for_neighbours(a, qxyz[3 * h], qxyz[3 * h + 1], qxyz[3 * h + 2],
                 [&](const float4& p, float, float, float, float d2, int32_t) {
                   const float d = __builtin_sqrtf(d2);
                   const float s = fmaxf(fmaf(-d, a.inv_l, 1.0f), 0.0f);
                   A[__float_as_int(p.w)] += kernel_weight(a.coef, s);
                 });
}

// loss = -(1/H) sum_h log(alpha[h][y_h] / S_h), double accumulation, fixed order
__global__ void __launch_bounds__(256) k_loss_value(const float* __restrict__ alpha_q,
                                                    const int32_t* __restrict__ qlab, int64_t H,
                                                    int32_t K, float* __restrict__ loss) {
  __shared__ double part[256];
  double s = 0.0;
  for (int64_t h = threadIdx.x; h < H; h += 256) {
    const float* A = alpha_q + h * K;
    double S = 0.0;
    for (int k = 0; k < K; ++k) S += (double)A[k];
    s += log((double)A[qlab[h]] / S);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(-part[0] / (double)H);
}

// Per query: 1/S, 1/alpha_y, and its closed-form dloss/dsigma0 share
//   sum_k G_hk (alpha_hk - alpha0) / sigma0 = -(g/(H sigma0)) (K alpha0/S - alpha0/alpha_y).
__global__ void k_prep(const float* __restrict__ alpha_q, const int32_t* __restrict__ qlab, int64_t H,
                       int32_t K, float alpha0, float sigma0, const float* __restrict__ gscale,
                       float* __restrict__ inv_s, float* __restrict__ inv_ay,
                       double* __restrict__ dsig) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H) return;
  const float* A = alpha_q + h * K;
  double S = 0.0;
  for (int k = 0; k < K; ++k) S += (double)A[k];
  const double ay = (double)A[qlab[h]];
  inv_s[h] = (float)(1.0 / S);
  inv_ay[h] = (float)(1.0 / ay);
  const double g = (double)gscale[0];
  dsig[h] = -(g / ((double)H * (double)sigma0)) * ((double)K * alpha0 / S - (double)alpha0 / ay);
}

// Query-side adjoint: dloss/dx_h and the per-query share of dloss/dl.
__global__ void k_query_grad(LossArgs a, const float* __restrict__ qxyz,
                             const int32_t* __restrict__ qlab, const float* __restrict__ inv_s,
                             const float* __restrict__ inv_ay, const float* __restrict__ gscale,
                             float* __restrict__ grad_q, double* __restrict__ dl_part) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.H) return;
  const float gH = gscale[0] / (float)a.H;
  const int32_t yh = qlab[h];
  const float is = inv_s[h], ia = inv_ay[h];
  float gx = 0.f, gy = 0.f, gz = 0.f;
  double dl = 0.0;
  const float il2 = a.inv_l * a.inv_l;
  for_neighbours(a, qxyz[3 * h], qxyz[3 * h + 1], qxyz[3 * h + 2],
                 [&](const float4& p, float dx, float dy, float dz, float d2, int32_t) {
                   const int32_t yt = __float_as_int(p.w);
                   const float G = -gH * ((yt == yh ? ia : 0.0f) - is);
                   const float d = __builtin_sqrtf(d2);
                   const float r = d * a.inv_l;
                   const float s = fmaxf(1.0f - r, 0.0f);
                   const float gr = a.sigma0 * dfdr_over_r(s);      // sigma0 f'(r)/r
                   const float c = G * gr * il2;                    // coefficient of (x_t - x_h)
                   gx -= c * dx;
                   gy -= c * dy;
                   gz -= c * dz;
                   dl += (double)(-G * gr * r * r * a.inv_l);       // G sigma0 f'(r) (-r/l)
                 });
  if (grad_q) {
    grad_q[3 * h] = gx;
    grad_q[3 * h + 1] = gy;
    grad_q[3 * h + 2] = gz;
  }
  dl_part[h] = dl;
}

// Training-side adjoint: dloss/dx_t, walking the bucketed queries around each row.
__global__ void k_train_grad(LossArgs a, const float* __restrict__ txyz,
                             const int32_t* __restrict__ tlab, int64_t n_train,
                             const int32_t* __restrict__ qlab, const float* __restrict__ inv_s,
                             const float* __restrict__ inv_ay, const float* __restrict__ gscale,
                             float* __restrict__ grad_t) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_train) return;
  const float gH = gscale[0] / (float)a.H;
  const int32_t yt = tlab[t];
  float gx = 0.f, gy = 0.f, gz = 0.f;
  const float il2 = a.inv_l * a.inv_l;
  for_neighbours(a, txyz[3 * t], txyz[3 * t + 1], txyz[3 * t + 2],
                 [&](const float4& p, float dx, float dy, float dz, float d2, int32_t j) {
                   // p is a query record; (dx, dy, dz) = x_h - x_t
                   const int32_t h = a.sidx[j];
                   const float G = -gH * ((yt == qlab[h] ? inv_ay[h] : 0.0f) - inv_s[h]);
                   const float d = __builtin_sqrtf(d2);
                   const float s = fmaxf(fmaf(-d, a.inv_l, 1.0f), 0.0f);
                   const float c = G * a.sigma0 * dfdr_over_r(s) * il2;
                   gx -= c * dx;
                   gy -= c * dy;
                   gz -= c * dz;
                 });
  grad_t[3 * t] = gx;
  grad_t[3 * t + 1] = gy;
  grad_t[3 * t + 2] = gz;
}

// ---------------------------------------------------------------------------
// per-class kernels: rows of class k use l_k and sigma0_k,
//   alpha_h^k = alpha0 + sum_{y_t = k} sigma0_k f(|x_t - x_h| / l_k),
//   dloss/dl_k      = sum over pairs with y_t = k  G_{h,k} sigma0_k f'(r) (-r/l_k)
//   dloss/dsigma0_k = sum over pairs with y_t = k  G_{h,k} f(r)
// per query into dl[h][k], ds[h][k] (double), then summed per class in a fixed order.
// ---------------------------------------------------------------------------
__global__ void k_alpha_q_pc(LossArgs a, const float* __restrict__ qxyz,
                             float* __restrict__ alpha_q) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.H) return;
  float* A = alpha_q + h * a.K;
  for (int k = 0; k < a.K; ++k) A[k] = a.alpha0;
  for_neighbours(a, qxyz[3 * h], qxyz[3 * h + 1], qxyz[3 * h + 2],
                 [&](const float4& p, float, float, float, float d2, int32_t) {
                   const int32_t y = __float_as_int(p.w);
                   const float4 c = a.cls[y];
                   if (!(d2 < c.x)) return;
                   const float d = __builtin_sqrtf(d2);
                   const float s = fmaxf(fmaf(-d, c.y, 1.0f), 0.0f);
                   A[y] += c.z * kernel_weight(a.coef, s);
                 });
}

__global__ void k_query_grad_pc(LossArgs a, const float* __restrict__ qxyz,
                                const int32_t* __restrict__ qlab, const float* __restrict__ inv_s,
                                const float* __restrict__ inv_ay, const float* __restrict__ gscale,
                                float* __restrict__ grad_q, double* __restrict__ dl,
                                double* __restrict__ ds) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.H) return;
  const float gH = gscale[0] / (float)a.H;
  const int32_t yh = qlab[h];
  const float is = inv_s[h], ia = inv_ay[h];
  double* DL = dl + h * a.K;
  double* DS = ds + h * a.K;
  for (int k = 0; k < a.K; ++k) {
    DL[k] = 0.0;
    DS[k] = 0.0;
  }
  float gx = 0.f, gy = 0.f, gz = 0.f;
  for_neighbours(a, qxyz[3 * h], qxyz[3 * h + 1], qxyz[3 * h + 2],
                 [&](const float4& p, float dx, float dy, float dz, float d2, int32_t) {
                   const int32_t yt = __float_as_int(p.w);
                   const float4 c = a.cls[yt];
                   if (!(d2 < c.x)) return;
                   const float G = -gH * ((yt == yh ? ia : 0.0f) - is);
                   const float d = __builtin_sqrtf(d2);
                   const float r = d * c.y;
                   const float s = fmaxf(1.0f - r, 0.0f);
                   const float gr = c.z * dfdr_over_r(s);          // sigma0_k f'(r)/r
                   const float cc = G * gr * (c.y * c.y);          // coefficient of (x_t - x_h)
                   gx -= cc * dx;
                   gy -= cc * dy;
                   gz -= cc * dz;
                   DL[yt] += (double)(-G * gr * r * r * c.y);     // G sigma0_k f'(r) (-r/l_k)
                   DS[yt] += (double)(G * kernel_weight(a.coef, s));
                 });
  if (grad_q) {
    grad_q[3 * h] = gx;
    grad_q[3 * h + 1] = gy;
    grad_q[3 * h + 2] = gz;
  }
}

__global__ void k_train_grad_pc(LossArgs a, const float* __restrict__ txyz,
                                const int32_t* __restrict__ tlab, int64_t n_train,
                                const int32_t* __restrict__ qlab, const float* __restrict__ inv_s,
                                const float* __restrict__ inv_ay, const float* __restrict__ gscale,
                                float* __restrict__ grad_t) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_train) return;
  const float gH = gscale[0] / (float)a.H;
  const int32_t yt = tlab[t];
  const float4 c = a.cls[yt];
  float gx = 0.f, gy = 0.f, gz = 0.f;
  const float il2 = c.y * c.y;
  for_neighbours(a, txyz[3 * t], txyz[3 * t + 1], txyz[3 * t + 2],
                 [&](const float4&, float dx, float dy, float dz, float d2, int32_t j) {
                   if (!(d2 < c.x)) return;
                   const int32_t h = a.sidx[j];
                   const float G = -gH * ((yt == qlab[h] ? inv_ay[h] : 0.0f) - inv_s[h]);
                   const float d = __builtin_sqrtf(d2);
                   const float s = fmaxf(fmaf(-d, c.y, 1.0f), 0.0f);
                   const float cc = G * c.z * dfdr_over_r(s) * il2;
                   gx -= cc * dx;
                   gy -= cc * dy;
                   gz -= cc * dz;
                 });
  grad_t[3 * t] = gx;
  grad_t[3 * t + 1] = gy;
  grad_t[3 * t + 2] = gz;
}

// out[k] = sum_h v[h][k] (one workgroup per class, fixed order)
__global__ void __launch_bounds__(256) k_colsum_f64(const double* __restrict__ v, int64_t H,
                                                    int32_t K, float* __restrict__ out) {
  __shared__ double part[256];
  const int32_t k = blockIdx.x;
  double s = 0.0;
  for (int64_t h = threadIdx.x; h < H; h += 256) s += v[h * K + k];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = (float)part[0];
}

__global__ void __launch_bounds__(256) k_sum_f64(const double* __restrict__ v, int64_t n,
                                                 float* __restrict__ out) {
  __shared__ double part[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)part[0];
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)ceil_div_i64(n > 0 ? n : 1, t); }

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
constexpr size_t kAl = 256;
struct Carve {
  char* base;
  size_t used;
  template <typename T>
  T* take(size_t n) {
    size_t off = (used + kAl - 1) / kAl * kAl;
    used = off + (n > 0 ? n : 1) * sizeof(T);
    return base ? (T*)(base + off) : nullptr;
  }
};

struct SetBufs {
  PointSet ps;
  BucketScratch scr;
};

void carve_set(Carve& c, SetBufs& s, int64_t n, int64_t nblocks_cap) {
  const int64_t slots = std::min<int64_t>(n, nblocks_cap);
  s.ps.n = n;
  s.ps.wts = nullptr;   // every training row of the loss weighs 1
  s.scr.wt = nullptr;
  s.ps.pts = c.take<float4>(n);
  s.ps.dense = c.take<int32_t>(nblocks_cap);
  s.ps.slot_lin = c.take<int32_t>(slots);
  s.ps.prefix = c.take<int32_t>(slots * (LB * LB * LB + 1));
  s.ps.d_nslots = c.take<int32_t>(1);
  s.scr.keys = c.take<uint64_t>(n);
  s.scr.akeys = c.take<uint64_t>(n);
  s.scr.idx = c.take<uint32_t>(n);
  s.scr.aidx = c.take<uint32_t>(n);
  s.scr.rec = c.take<float4>(n);
  s.scr.flag = c.take<int32_t>(n);
  s.scr.slot_excl = c.take<int32_t>(n);
  s.ps.head = c.take<int32_t>(n + 1);
  s.scr.sort_tmp = c.take<char>(radix_tmp_bytes(n));
  s.scr.scan_tmp = c.take<char>(scan_tmp_bytes(n));
}

struct LossBufs {
  SetBufs tr, qu;
  int32_t* bbox;
  uint32_t* err;
  float* alpha_q;
  float* inv_s;
  float* inv_ay;
  double* dsig;
  double* dl;
  double* dlk;   // [H][K] per-class form
  double* dsk;   // [H][K]
  float4* cls;   // [K] per-class form: class kernels (in the header)
};

// bounding box and error word (first 512 bytes) and the per-class kernel table
// (up to 255 float4), ahead of the carved buffers
constexpr size_t kHdr = 512 + 256 * sizeof(float4);

// Buffers after the header, for a grid of nblocks blocks (nullptr base: size only).
size_t carve_body(char* base, LossBufs& b, int64_t nt, int64_t nq, int32_t K, int64_t nblocks) {
  Carve c{base, 0};
  b.alpha_q = c.take<float>((size_t)nq * K);
  b.inv_s = c.take<float>(nq);
  b.inv_ay = c.take<float>(nq);
  b.dsig = c.take<double>(nq);
  b.dl = c.take<double>(nq);
  b.dlk = c.take<double>((size_t)nq * K);
  b.dsk = c.take<double>((size_t)nq * K);
  carve_set(c, b.tr, nt, nblocks);
  carve_set(c, b.qu, nq, nblocks);
  return c.used + kAl;
}

smki_status err_status(uint32_t e) {
  if (e & (DEVERR_LABEL | DEVERR_NONFINITE)) return SMKI_E_BAD_INPUT;
  if (e & DEVERR_RANGE) return SMKI_E_RANGE;
  return SMKI_E_DEVICE;
}

char* align_up(char* p) { return (char*)(((uintptr_t)p + kAl - 1) / kAl * kAl); }

// Validate both sets and size the grid (synchronous); then carve the body from
// the caller's workspace or a fresh allocation, and bucket the training rows
// (and the queries if both_sets).
// h_cls (nullable): per-class kernel table, copied into the header before the
// synchronisation (so the host array may go out of scope after the call).
smki_status prepare(const float* txyz, const int32_t* tlab, int64_t nt, const float* qxyz,
                    const int32_t* qlab, int64_t nq, float l, int32_t K, bool both_sets,
                    char* ws, size_t ws_bytes, char** own, LossBufs& b, BucketGeom& g,
                    hipStream_t st, const float4* h_cls = nullptr) {
  const float h = (float)((double)l * (1.0 + 1.0 / 1024.0));
  char* hdr = ws ? align_up(ws) : nullptr;
  if (ws && ws_bytes < kHdr + kAl) return SMKI_E_CAPACITY;
  if (!ws) {
    SMKI_HIP_TRY(hipMallocAsync((void**)own, kHdr, st));
    hdr = *own;
  }
  b.bbox = (int32_t*)hdr;
  b.err = (uint32_t*)(hdr + 64);
  b.cls = (float4*)(hdr + 512);
  if (h_cls)
    SMKI_HIP_TRY(hipMemcpyAsync(b.cls, h_cls, sizeof(float4) * K, hipMemcpyHostToDevice, st));
  const int32_t bbox0[8] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN, 0, 0};
  SMKI_HIP_TRY(hipMemcpyAsync(b.bbox, bbox0, sizeof(bbox0), hipMemcpyHostToDevice, st));
  SMKI_HIP_TRY(hipMemsetAsync(b.err, 0, sizeof(uint32_t) * 4, st));
  if (nt > 0)
    hipLaunchKernelGGL(k_validate, dim3(nblk(nt, 256)), dim3(256), 0, st, txyz, tlab, nt, K, h,
                       b.bbox, b.err);
  hipLaunchKernelGGL(k_validate, dim3(nblk(nq, 256)), dim3(256), 0, st, qxyz, qlab, nq, K, h,
                     b.bbox, b.err);
  SMKI_HIP_TRY(hipGetLastError());
  int32_t hb[8];
  uint32_t e = 0;
  SMKI_HIP_TRY(hipMemcpyAsync(hb, b.bbox, sizeof(hb), hipMemcpyDeviceToHost, st));
  SMKI_HIP_TRY(hipMemcpyAsync(&e, b.err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  SMKI_HIP_TRY(stream_wait(st));
  if (e) return err_status(e);
  g = BucketGeom{};
  g.planes = 1;
  g.res = h;
  g.B = LB;
  g.log2B = LLOG2B;
  g.n_blocks = 1;
  for (int a = 0; a < 3; ++a) {
    const int32_t lo = (hb[a] - 1) >> LLOG2B, hi = (hb[3 + a] + 1) >> LLOG2B;
    g.blo[a] = lo;
    g.nb[a] = hi - lo + 1;
    g.n_blocks *= g.nb[a];
  }
  if (g.n_blocks > kMaxLossBlocks) return SMKI_E_CAPACITY;
  int bits = 0;
  while (bits < 62 && (int64_t(1) << bits) < g.n_blocks) ++bits;
  g.key_bits = std::max(1, bits + 3 * LLOG2B);
  const size_t body = carve_body(nullptr, b, nt, nq, K, g.n_blocks);
  char* bbase = nullptr;
  if (ws) {
    bbase = align_up(hdr + kHdr);
    if ((size_t)(bbase - ws) + body > ws_bytes) return SMKI_E_CAPACITY;
  } else {
    char* p = nullptr;
    SMKI_HIP_TRY(hipMallocAsync((void**)&p, body, st));
    own[1] = p;
    bbase = align_up(p);
  }
  carve_body(bbase, b, nt, nq, K, g.n_blocks);
  SMKI_HIP_TRY(hipMemsetAsync(b.tr.ps.d_nslots, 0, sizeof(int32_t), st));
  SMKI_HIP_TRY(hipMemsetAsync(b.qu.ps.d_nslots, 0, sizeof(int32_t), st));
  SMKI_HIP_TRY(bucket_rows(txyz, tlab, nt, g, b.tr.ps, b.tr.scr, b.err, st));
  if (both_sets) SMKI_HIP_TRY(bucket_rows(qxyz, qlab, nq, g, b.qu.ps, b.qu.scr, b.err, st));
  return SMKI_OK;
}

void release(char** own, hipStream_t st) {
  for (int i = 0; i < 2; ++i)
    if (own[i]) (void)hipFreeAsync(own[i], st);
}

LossArgs make_args(const BucketGeom& g, const SetBufs& s, float l, float sigma0, float alpha0,
                   int32_t K, int64_t H) {
  LossArgs a{};
  a.g = g;
  a.pts = s.ps.pts;
  a.dense = s.ps.dense;
  a.prefix = s.ps.prefix;
  a.sidx = (const int32_t*)s.scr.idx;
  a.l = l;
  a.l2 = l * l;
  a.inv_l = 1.0f / l;
  a.sigma0 = sigma0;
  a.alpha0 = alpha0;
  for (int i = 0; i < SMKI_POLY_N; ++i) a.coef[i] = (float)(kSmkiQ[i] * (double)sigma0);
  a.K = K;
  a.H = H;
  return a;
}

bool bad_params(int64_t nt, int64_t nq, float l, float sigma0, float alpha0, int32_t K) {
  return nt < 0 || nq <= 0 || !(std::isfinite(l) && l > 0) || !(std::isfinite(sigma0) && sigma0 > 0) ||
         !(std::isfinite(alpha0) && alpha0 > 0) || K < 2 || K > 255 ||
         nt > (int64_t)INT32_MAX / 2 || nq > (int64_t)INT32_MAX / 2;
}

}  // namespace

extern "C" size_t smki_loss_workspace_bytes(int64_t n_train, int64_t n_query, int32_t K) {
  LossBufs b{};
  return kHdr + 2 * kAl + carve_body(nullptr, b, std::max<int64_t>(n_train, 0),
                                     std::max<int64_t>(n_query, 1), std::max(K, 1),
                                     kMaxLossBlocks);
}

extern "C" smki_status smki_loss_forward(const float* txyz, const int32_t* tlab, int64_t nt,
                                         const float* qxyz, const int32_t* qlab, int64_t nq,
                                         float l, float sigma0, float alpha0, int32_t K,
                                         void* hip_stream, void* workspace, size_t ws_bytes,
                                         float* loss, float* alpha_q) {
  if (bad_params(nt, nq, l, sigma0, alpha0, K) || !qxyz || !qlab || !loss ||
      (nt > 0 && (!txyz || !tlab)))
    return SMKI_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  char* own[2] = {nullptr, nullptr};
  LossBufs b{};
  BucketGeom g{};
  smki_status rc = prepare(txyz, tlab, nt, qxyz, qlab, nq, l, K, false, (char*)workspace,
                           ws_bytes, own, b, g, st);
  if (rc == SMKI_OK) {
    const LossArgs a = make_args(g, b.tr, l, sigma0, alpha0, K, nq);
    float* A = alpha_q ? alpha_q : b.alpha_q;
    hipLaunchKernelGGL(k_alpha_q, dim3(nblk(nq, 64)), dim3(64), 0, st, a, qxyz, A);
    hipLaunchKernelGGL(k_loss_value, dim3(1), dim3(256), 0, st, (const float*)A, qlab, nq, K, loss);
    if (hipGetLastError() != hipSuccess) rc = SMKI_E_DEVICE;
  }
  release(own, st);
  return rc;
}

extern "C" smki_status smki_loss_backward(const float* txyz, const int32_t* tlab, int64_t nt,
                                          const float* qxyz, const int32_t* qlab, int64_t nq,
                                          float l, float sigma0, float alpha0, int32_t K,
                                          void* hip_stream, void* workspace, size_t ws_bytes,
                                          const float* alpha_q, const float* grad_loss,
                                          float* grad_l, float* grad_sigma0, float* grad_train,
                                          float* grad_query) {
  if (bad_params(nt, nq, l, sigma0, alpha0, K) || !qxyz || !qlab || !alpha_q || !grad_loss ||
      (nt > 0 && (!txyz || !tlab)))
    return SMKI_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  char* own[2] = {nullptr, nullptr};
  LossBufs b{};
  BucketGeom g{};
  smki_status rc = prepare(txyz, tlab, nt, qxyz, qlab, nq, l, K, grad_train != nullptr,
                           (char*)workspace, ws_bytes, own, b, g, st);
  if (rc == SMKI_OK) {
    hipLaunchKernelGGL(k_prep, dim3(nblk(nq, 256)), dim3(256), 0, st, alpha_q, qlab, nq, K, alpha0,
                       sigma0, grad_loss, b.inv_s, b.inv_ay, b.dsig);
    if (grad_sigma0)
      hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, st, (const double*)b.dsig, nq,
                         grad_sigma0);
    const LossArgs aq = make_args(g, b.tr, l, sigma0, alpha0, K, nq);
    hipLaunchKernelGGL(k_query_grad, dim3(nblk(nq, 64)), dim3(64), 0, st, aq, qxyz, qlab,
                       (const float*)b.inv_s, (const float*)b.inv_ay, grad_loss, grad_query, b.dl);
    if (grad_l)
      hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, st, (const double*)b.dl, nq, grad_l);
    if (grad_train && nt > 0) {
      const LossArgs at = make_args(g, b.qu, l, sigma0, alpha0, K, nq);
      hipLaunchKernelGGL(k_train_grad, dim3(nblk(nt, 64)), dim3(64), 0, st, at, txyz, tlab, nt,
                         qlab, (const float*)b.inv_s, (const float*)b.inv_ay, grad_loss,
                         grad_train);
    }
    if (hipGetLastError() != hipSuccess) rc = SMKI_E_DEVICE;
  }
  release(own, st);
  return rc;
}

// ---------------------------------------------------------------------------
// per-class kernels (l_k, sigma0_k per class)
// ---------------------------------------------------------------------------
namespace {

// Host table of the class kernels and the largest l; false if a value is invalid.
bool class_table(const float* l, const float* sigma0, int32_t K, float4* t, float* lmax) {
  if (!l || !sigma0 || K < 2 || K > 255) return false;
  *lmax = 0.0f;
  for (int32_t k = 0; k < K; ++k) {
    if (!(std::isfinite(l[k]) && l[k] > 0) || !(std::isfinite(sigma0[k]) && sigma0[k] > 0))
      return false;
    t[k] = make_float4(l[k] * l[k], 1.0f / l[k], sigma0[k], l[k]);
    *lmax = std::max(*lmax, l[k]);
  }
  return true;
}

LossArgs make_args_pc(const BucketGeom& g, const SetBufs& s, float lmax, const float4* cls,
                      float alpha0, int32_t K, int64_t H) {
  LossArgs a = make_args(g, s, lmax, 1.0f, alpha0, K, H);   // coef = Q: sigma0_k applied per row
  a.cls = cls;
  return a;
}

}  // namespace

extern "C" smki_status smki_loss_forward_classes(const float* txyz, const int32_t* tlab,
                                                 int64_t nt, const float* qxyz,
                                                 const int32_t* qlab, int64_t nq, const float* l,
                                                 const float* sigma0, float alpha0, int32_t K,
                                                 void* hip_stream, void* workspace,
                                                 size_t ws_bytes, float* loss, float* alpha_q) {
  float4 tab[256];
  float lmax = 0.0f;
  if (!class_table(l, sigma0, K, tab, &lmax) || bad_params(nt, nq, lmax, 1.0f, alpha0, K) ||
      !qxyz || !qlab || !loss || (nt > 0 && (!txyz || !tlab)))
    return SMKI_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  char* own[2] = {nullptr, nullptr};
  LossBufs b{};
  BucketGeom g{};
  smki_status rc = prepare(txyz, tlab, nt, qxyz, qlab, nq, lmax, K, false, (char*)workspace,
                           ws_bytes, own, b, g, st, tab);
  if (rc == SMKI_OK) {
    const LossArgs a = make_args_pc(g, b.tr, lmax, b.cls, alpha0, K, nq);
    float* A = alpha_q ? alpha_q : b.alpha_q;
    hipLaunchKernelGGL(k_alpha_q_pc, dim3(nblk(nq, 64)), dim3(64), 0, st, a, qxyz, A);
    hipLaunchKernelGGL(k_loss_value, dim3(1), dim3(256), 0, st, (const float*)A, qlab, nq, K, loss);
    if (hipGetLastError() != hipSuccess) rc = SMKI_E_DEVICE;
  }
  release(own, st);
  return rc;
}

extern "C" smki_status smki_loss_backward_classes(
    const float* txyz, const int32_t* tlab, int64_t nt, const float* qxyz, const int32_t* qlab,
    int64_t nq, const float* l, const float* sigma0, float alpha0, int32_t K, void* hip_stream,
    void* workspace, size_t ws_bytes, const float* alpha_q, const float* grad_loss, float* grad_l,
    float* grad_sigma0, float* grad_train, float* grad_query) {
  float4 tab[256];
  float lmax = 0.0f;
  if (!class_table(l, sigma0, K, tab, &lmax) || bad_params(nt, nq, lmax, 1.0f, alpha0, K) ||
      !qxyz || !qlab || !alpha_q || !grad_loss || (nt > 0 && (!txyz || !tlab)))
    return SMKI_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)hip_stream;
  char* own[2] = {nullptr, nullptr};
  LossBufs b{};
  BucketGeom g{};
  smki_status rc = prepare(txyz, tlab, nt, qxyz, qlab, nq, lmax, K, grad_train != nullptr,
                           (char*)workspace, ws_bytes, own, b, g, st, tab);
  if (rc == SMKI_OK) {
    // 1/S and 1/alpha_y per query (the single-kernel sigma0 share is not used here)
    hipLaunchKernelGGL(k_prep, dim3(nblk(nq, 256)), dim3(256), 0, st, alpha_q, qlab, nq, K, alpha0,
                       1.0f, grad_loss, b.inv_s, b.inv_ay, b.dsig);
    const LossArgs aq = make_args_pc(g, b.tr, lmax, b.cls, alpha0, K, nq);
    hipLaunchKernelGGL(k_query_grad_pc, dim3(nblk(nq, 64)), dim3(64), 0, st, aq, qxyz, qlab,
                       (const float*)b.inv_s, (const float*)b.inv_ay, grad_loss, grad_query,
                       b.dlk, b.dsk);
    if (grad_l)
      hipLaunchKernelGGL(k_colsum_f64, dim3(K), dim3(256), 0, st, (const double*)b.dlk, nq, K,
                         grad_l);
    if (grad_sigma0)
      hipLaunchKernelGGL(k_colsum_f64, dim3(K), dim3(256), 0, st, (const double*)b.dsk, nq, K,
                         grad_sigma0);
    if (grad_train && nt > 0) {
      const LossArgs at = make_args_pc(g, b.qu, lmax, b.cls, alpha0, K, nq);
      hipLaunchKernelGGL(k_train_grad_pc, dim3(nblk(nt, 64)), dim3(64), 0, st, at, txyz, tlab, nt,
                         qlab, (const float*)b.inv_s, (const float*)b.inv_ay, grad_loss,
                         grad_train);
    }
    if (hipGetLastError() != hipSuccess) rc = SMKI_E_DEVICE;
  }
  release(own, st);
  return rc;
}

// ---------------------------------------------------------------------------
// the predictive loss without any allocation: a fixed device array as workspace
// ---------------------------------------------------------------------------
namespace {

// Workspace of smki_loss_forward_noalloc.  Each device the library runs on
// holds its own copy until the process ends.  Host code never passes this
// name to a kernel or a copy: it stands in for the array on the host side;
// the device address comes from hipGetSymbolAddress (static_scratch below).
constexpr size_t kStaticScratchBytes = SMKI_LOSS_NOALLOC_BYTES;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
smki_status static_scratch(char** out) {
  int dev = -1;
  SMKI_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SMKI_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SMKI_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return SMKI_E_DEVICE;
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return SMKI_OK;
}

}  // namespace

extern "C" smki_status smki_loss_forward_noalloc(const float* txyz, const int32_t* tlab,
                                                 int64_t nt, const float* qxyz,
                                                 const int32_t* qlab, int64_t nq, float l,
                                                 float sigma0, float alpha0, int32_t K,
                                                 void* hip_stream, float* loss, float* alpha_q) {
  if (bad_params(nt, nq, l, sigma0, alpha0, K) || !qxyz || !qlab || !loss ||
      (nt > 0 && (!txyz || !tlab)))
    return SMKI_E_INVALID_ARG;
  // the buffers that do not depend on the grid must fit before anything runs;
  // the grid-dependent tables are checked once the grid is known
  LossBufs b0{};
  if (kHdr + 2 * kAl + carve_body(nullptr, b0, nt, nq, K, 1) > kStaticScratchBytes)
    return SMKI_E_CAPACITY;
  char* ws = nullptr;
  const smki_status rc = static_scratch(&ws);
  if (rc != SMKI_OK) return rc;
  return smki_loss_forward(txyz, tlab, nt, qxyz, qlab, nq, l, sigma0, alpha0, K, hip_stream, ws,
                           kStaticScratchBytes, loss, alpha_q);
}
