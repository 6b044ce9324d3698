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

// The r-th cube of a virtual with nt blocks: bi slowest, then (ci, di >= ci) row-major.
PPL_HD inline void cube_decode(int64_t r, int nt, int& bi, int& ci, int& di) {
  const int64_t per = (int64_t)nt * (nt + 1) / 2;
  bi = (int)(r / per);
  int q = (int)(r - (int64_t)bi * per);
  ci = 0;
  while (q >= nt - ci) {
    q -= nt - ci;
    ++ci;
  }
  di = ci + q;
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
