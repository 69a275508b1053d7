// Geometry of the splat's partial-sum regions and the merge's candidates
// (internal; host and device).  A work unit of a (class, block) splats into
// the region of voxels its rows can reach, the block grown by the stencil reach
// R on every side; the merge of a target block adds, for each of its voxels,
// the region pieces of the neighbouring units that cover the voxel.
#pragma once
#include "smki_internal.h"


// The region of a (class, block) work unit, (B + 2R)^3 voxels, split into 27
// pieces: piece p = (dx+1)*9 + (dy+1)*3 + (dz+1) holds the voxels that lie in
// the block at offset (dx, dy, dz) from the unit's block.  Per axis a piece
// spans R voxels (d = -1, region coordinates [0, R)), B (d = 0, [R, R+B)) or
// R (d = +1, [R+B, 2R+B)).  Partial sums are stored piece after piece, each
// piece contiguous with z fastest.
template <int B, int R>
struct Pieces {
  static constexpr int ext(int d) { return d == 0 ? B : R; }
  static constexpr int rstart(int d) { return d < 0 ? 0 : (d == 0 ? R : R + B); }
  static constexpr int size(int p) { return ext(p / 9 - 1) * ext((p / 3) % 3 - 1) * ext(p % 3 - 1); }
  static constexpr int base(int p) {
    int b = 0;
    for (int q = 0; q < p; ++q) b += size(q);
    return b;
  }
};

// Start of piece p inside a unit's partial sums (p known at run time): the
// x-layers before it (each spans all (y, z)), then the y-rows of its layer
// before it, then the z-cells of its row before it.  Per axis the extents are
// (R, B, R), and the extent before index i is 0, R or R + B.
template <int B, int R>
__host__ __device__ inline int pbase(int p) {
  constexpr int DR = 2 * R + B;
  const int px = p / 9, py = (p / 3) % 3, pz = p % 3;
  auto ext = [](int i) { return i == 1 ? B : R; };
  auto before = [](int i) { return i == 0 ? 0 : (i == 1 ? R : R + B); };
  return before(px) * DR * DR + ext(px) * before(py) * DR + ext(px) * ext(py) * before(pz);
}

template <int B, int R>
struct MergeShape {
  static constexpr int B3 = B * B * B;
  static constexpr int NT = B3 < 1024 ? B3 : 1024;    // threads per workgroup
  static constexpr int VPT = B3 / NT;                 // voxels per thread
  static constexpr int CPG = NT < 32 ? NT : 32;       // classes per lookup group (<= threads)
  static constexpr int RW = NT < SMKI_WAVE ? NT : SMKI_WAVE;   // lanes of one wavefront in use
  // neighbours whose region can cover one voxel: per axis 1, 2 (R > 0), or 3 (2R > B)
  static constexpr int AX = R == 0 ? 1 : (2 * R > B ? 3 : 2);
  static constexpr int MAXC = AX * AX * AX;
};

// Candidate k of voxel vv (coordinates in the target block): the neighbour c
// (per axis 0, -1 if v < R, +1 if v >= B - R; both only when 2R > B) whose
// region covers the voxel, which lies in piece 26 - c of that region.  Packed
// as (neighbour index << 16) | offset of the voxel in the region's pieces, or
// -1 when the candidate does not apply to this voxel.
template <int B, int R>
__host__ __device__ inline int merge_candidate(const int vv[3], int k) {
  constexpr int AX = MergeShape<B, R>::AX;
  const int kk[3] = {k / (AX * AX), (k / AX) % AX, k % AX};
  int c3[3], l3[3];
  bool valid = true;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    int c = 0;
    if (kk[q] == 1) {
      if (AX == 2) {
        c = vv[q] < R ? -1 : (vv[q] >= B - R ? 1 : 0);
        valid = valid && c != 0;
      } else {
        c = -1;
        valid = valid && vv[q] < R;
      }
    } else if (kk[q] == 2) {
      c = 1;
      valid = valid && vv[q] >= B - R;
    }
    c3[q] = c;
    l3[q] = c > 0 ? vv[q] - (B - R) : vv[q];
  }
  const int ci = (c3[0] + 1) * 9 + (c3[1] + 1) * 3 + (c3[2] + 1);
  const int ey = c3[1] == 0 ? B : R, ez = c3[2] == 0 ? B : R;
  const int off = pbase<B, R>(26 - ci) + (l3[0] * ey + l3[1]) * ez + l3[2];
  return valid ? (ci << 16) | off : -1;
}
