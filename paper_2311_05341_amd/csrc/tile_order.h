// Workgroup -> (output block, time tile) maps of the 1-D grids, shared by the
// forward kernels.  Workgroups are handed to the 8 XCDs (each with its own L2)
// round-robin by linear id, so workgroup w runs on XCD w % 8.
#pragma once

namespace dd {

constexpr int kXcds = 8;
constexpr int kDmGroup = 4;  // output blocks per group in the grouped order

// order 0: time tiles fastest.  Neighbouring tiles (whose staged rows overlap
//   by the delay spread) run at once on different XCDs; each output block
//   streams the whole input once.
// order 1: each XCD takes whole time tiles (x, x + 8, ...), every output block
//   of a tile in turn, so the workgroups on one XCD stage nearby input rows.
// order 2: each XCD takes its tiles x, x + 8, ... for kDmGroup consecutive
//   output blocks at a time (the blocks of one tile next to each other), one
//   group of output blocks after another: kDmGroup blocks share each staged
//   tile in L2 while the grid still sweeps time.
// order 3: XCD x takes the contiguous run of time tiles [x * T, (x + 1) * T)
//   (T = n_tiles / 8 rounded down), time tiles fastest, one output block after
//   another.  The workgroups resident on one XCD then cover neighbouring tiles
//   of one output block, whose windows overlap wherever a block's delay spread
//   is wider than a tile (the direct-read plans), so they share input lines in
//   that XCD's L2.
// Tiles or blocks left over from whole rounds go last, in tile order.
__device__ __forceinline__ void tile_of(int w, int n_oblk, int n_tiles, int order, int &oblk, int &tblk) {
  if (order == 0) {
    tblk = w % n_tiles;
    oblk = w / n_tiles;
    return;
  }
  if (order == 1) {
    const int full = n_tiles / kXcds * kXcds;
    if (w < n_oblk * full) {
      const int x = w % kXcds, k = w / kXcds;
      tblk = x + kXcds * (k / n_oblk);
      oblk = k % n_oblk;
    } else {
      const int r = w - n_oblk * full;
      tblk = full + r / n_oblk;
      oblk = r % n_oblk;
    }
    return;
  }
  if (order == 3) {
    const int per = n_tiles / kXcds, main = kXcds * per * n_oblk;
    if (w < main) {
      const int x = w % kXcds, k = w / kXcds;
      oblk = k / per;
      tblk = x * per + (k - oblk * per);
    } else {
      const int r = w - main, tail_t = n_tiles - kXcds * per;
      tblk = kXcds * per + r % tail_t;
      oblk = r / tail_t;
    }
    return;
  }
  const int full_t = n_tiles / kXcds * kXcds, full_o = n_oblk / kDmGroup * kDmGroup;
  const int main = full_t * full_o;
  if (w < main) {
    const int x = w % kXcds, k = w / kXcds;
    const int per_group = (full_t / kXcds) * kDmGroup;  // workgroups of one XCD per output group
    const int g = k / per_group, r = k - g * per_group;
    tblk = x + kXcds * (r / kDmGroup);
    oblk = g * kDmGroup + r % kDmGroup;
    return;
  }
  const int r = w - main, tail_t = n_tiles - full_t;
  if (r < tail_t * n_oblk) {
    tblk = full_t + r % tail_t;
    oblk = r / tail_t;
  } else {
    const int r2 = r - tail_t * n_oblk;
    tblk = r2 % full_t;
    oblk = full_o + r2 / full_t;
  }
}

}  // namespace dd
