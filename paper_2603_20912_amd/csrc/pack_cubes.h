// Index arithmetic of the cube-blocked packing of V+- from the natural output of the
// upper-triangle build (T[(a, c)][(x, y)] = (ac|xy) over packed pairs c >= a, x <= y).
// Shared by the packing kernel and the host-side replay that checks its coverage.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define PPL_HD __host__ __device__
#else
#define PPL_HD
#endif

namespace ppl {

// For virtual a the indices b, c, d >= a are cut into blocks of kCube; a cube is a
// triple (bi, ci, di) of blocks with ci <= di (the pair (c, d) of a V+- column has c <= d).
constexpr int kCube = 16;

PPL_HD inline int cube_blocks(int v, int a) { return (v - a + kCube - 1) / kCube; }

PPL_HD inline int64_t cubes_of(int v, int a) {
  const int64_t nt = cube_blocks(v, a);
  return nt * nt * (nt + 1) / 2;
}

// The r-th cube of a virtual with nt blocks. Cubes (x, ci, y) and (y, ci, x) stage the same
// integrals (ac|bd) (rows c of block ci, pairs {b, d} with one index in block x and one in
// block y), so they are taken one after the other: ci slowest; for each ci first the cubes
// with bi < ci (no such partner), then the square bi, di >= ci by unordered pairs {x <= y},
// (x, x) alone and (x, y), (y, x) together. nt (nt - ci) cubes per ci.
PPL_HD inline void cube_decode(int64_t r, int nt, int& bi, int& ci, int& di) {
  int64_t q = r;
  ci = 0;
  while (q >= (int64_t)nt * (nt - ci)) {
    q -= (int64_t)nt * (nt - ci);
    ++ci;
  }
  const int w = nt - ci;
  if (q < (int64_t)ci * w) {
    bi = (int)(q / w);
    di = ci + (int)(q % w);
    return;
  }
  int p = (int)(q - (int64_t)ci * w), x = 0;
  while (p >= 1 + 2 * (w - 1 - x)) {
    p -= 1 + 2 * (w - 1 - x);
    ++x;
  }
  if (p == 0) {
    bi = di = ci + x;
    return;
  }
  const int y = x + 1 + (p - 1) / 2;
  const bool swap = (p - 1) % 2 != 0;
  bi = ci + (swap ? y : x);
  di = ci + (swap ? x : y);
}

// Virtual a of cube g given the prefix table off (off[a] = cubes of all virtuals below a),
// searched in [lo, hi) with off[lo] <= g < off[hi].
PPL_HD inline int cube_virtual(const int64_t* off, int lo, int hi, int64_t g) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (off[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Cube of launch slot `bid` among `total`: consecutive slots go to different XCDs, so slot
// bid is given the cube x * q + min(x, r) + j (x = bid % 8, j = bid / 8) and each XCD walks a
// contiguous run of cubes.
PPL_HD inline int64_t cube_of_slot(int64_t bid, int64_t total) {
  const int64_t x = bid % 8, j = bid / 8, q = total / 8, r = total % 8;
  return x * q + (x < r ? x : r) + j;
}

}  // namespace ppl
