// Host-side geometry shared by the rho kernels: Miller extents, plane-wave
// sphere tables grouped by z-slot, argument validation.
#pragma once

#include <algorithm>
#include <vector>

#include "xo_common.h"

namespace xo {

constexpr int kMaxAxis = 128;

struct SphereEntry {
  int src;  // index of the plane wave in the caller's coefficient row
  int bx;   // m_x - min m_x over the sphere
  int by;   // m_y - min m_y over the sphere
};

struct Extent {
  int lo[3], hi[3];
};

inline Extent extent_of(const int32_t* m, int n, const int* shift) {
  Extent e;
  for (int a = 0; a < 3; ++a) {
    e.lo[a] = 1 << 30;
    e.hi[a] = -(1 << 30);
  }
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      int v = m[3 * i + a] - (shift ? shift[a] : 0);
      e.lo[a] = std::min(e.lo[a], v);
      e.hi[a] = std::max(e.hi[a], v);
    }
  return e;
}

struct SphereTable {
  std::vector<SphereEntry> ent;
  std::vector<int> zoff;
  int nslot = 0;
};

inline SphereTable sphere_table(const int32_t* m, int npw, const Extent& ex) {
  SphereTable t;
  t.nslot = ex.hi[2] - ex.lo[2] + 1;
  std::vector<std::vector<SphereEntry>> by(t.nslot);
  for (int i = 0; i < npw; ++i)
    by[m[3 * i + 2] - ex.lo[2]].push_back({i, m[3 * i] - ex.lo[0], m[3 * i + 1] - ex.lo[1]});
  t.zoff.push_back(0);
  for (auto& v : by) {
    t.ent.insert(t.ent.end(), v.begin(), v.end());
    t.zoff.push_back((int)t.ent.size());
  }
  return t;
}


// Host validation of one pair (sizes, alias-free grid, q0 requirements).
// Fills the Miller extents of the conduction sphere, the valence sphere and
// the shifted G-set e = m_G - G0.
int validate_rho(const xo_rho_args* a, Extent* xc, Extent* xv, Extent* xe);

}  // namespace xo
