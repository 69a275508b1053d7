// Host check of the splat regions' piece layout and the merge's candidate
// list (paper_1909_04631_amd/csrc/smki_pieces.h) against a direct enumeration:
// for every voxel of a target block, the neighbouring blocks (offset c in
// {-1, 0, 1}^3) whose region -- the block grown by R voxels on every side --
// holds the voxel, and where in that region's piece-ordered partial sums the
// voxel sits (pieces counted out one by one, not by formula).  Prints one line
// per (B, R) shape and "ok" when every shape agrees.
#include <cstdio>
#include <set>
#include <utility>

#include "smki_pieces.h"

template <int B, int R>
int check_shape() {
  constexpr int DR = B + 2 * R;
  // the element offset of region coordinate r, by enumerating pieces in order
  auto direct_offset = [](const int r[3], int* piece) {
    int d[3], l[3], e[3];
    for (int a = 0; a < 3; ++a) {
      d[a] = r[a] < R ? -1 : (r[a] < R + B ? 0 : 1);
      const int start = d[a] < 0 ? 0 : (d[a] == 0 ? R : R + B);
      l[a] = r[a] - start;
      e[a] = d[a] == 0 ? B : R;
    }
    *piece = (d[0] + 1) * 9 + (d[1] + 1) * 3 + (d[2] + 1);
    int base = 0;
    for (int q = 0; q < *piece; ++q) {
      const int qx = q / 9 - 1, qy = (q / 3) % 3 - 1, qz = q % 3 - 1;
      base += (qx == 0 ? B : R) * (qy == 0 ? B : R) * (qz == 0 ? B : R);
    }
    return base + (l[0] * e[1] + l[1]) * e[2] + l[2];
  };
  int bad = 0, covered = 0;
  for (int x = 0; x < B; ++x)
    for (int y = 0; y < B; ++y)
      for (int z = 0; z < B; ++z) {
        const int vv[3] = {x, y, z};
        std::set<std::pair<int, int>> want, got;
        for (int cx = -1; cx <= 1; ++cx)
          for (int cy = -1; cy <= 1; ++cy)
            for (int cz = -1; cz <= 1; ++cz) {
              const int c[3] = {cx, cy, cz};
              int r[3];
              bool in = true;
              for (int a = 0; a < 3; ++a) {
                r[a] = vv[a] - c[a] * B + R;   // region coordinate in the neighbour's region
                in = in && r[a] >= 0 && r[a] < DR;
              }
              if (!in) continue;
              int piece = -1;
              const int off = direct_offset(r, &piece);
              const int ci = (cx + 1) * 9 + (cy + 1) * 3 + (cz + 1);
              if (piece != 26 - ci) ++bad;   // the voxel lies in the part of the region inside T
              want.insert({ci, off});
            }
        for (int k = 0; k < MergeShape<B, R>::MAXC; ++k) {
          const int pk = merge_candidate<B, R>(vv, k);
          if (pk >= 0) {
            if (!got.insert({pk >> 16, pk & 0xffff}).second) ++bad;   // listed twice
          }
        }
        if (want != got) ++bad;
        covered += (int)want.size();
        // pbase agrees with the compile-time piece bases
        for (int p = 0; p < 27; ++p)
          if (pbase<B, R>(p) != Pieces<B, R>::base(p)) ++bad;
      }
  std::printf("B=%d R=%d voxels=%d candidates=%d mismatches=%d\n", B, R, B * B * B, covered, bad);
  return bad;
}

int main() {
  int bad = 0;
  bad += check_shape<2, 1>() + check_shape<2, 2>();
  bad += check_shape<4, 1>() + check_shape<4, 2>() + check_shape<4, 3>() + check_shape<4, 4>();
  bad += check_shape<8, 1>() + check_shape<8, 2>() + check_shape<8, 3>() + check_shape<8, 4>();
  bad += check_shape<16, 2>() + check_shape<16, 4>();
  std::printf(bad ? "FAILED\n" : "ok\n");
  return bad ? 1 : 0;
}
