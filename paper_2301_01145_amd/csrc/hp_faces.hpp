// Boundary terms of the inhomogeneous FD2 solves (Section 2.4.2): the
// weighted face values added to the source at the unknowns next to a face.
#pragma once

#include "hp_device.hpp"
#include "hp_internal.hpp"

namespace hp {

// Boundary terms of inhomogeneous FD2 problems (added to the source value of
// an unknown next to a face).
template <typename T>
__device__ __forceinline__ double face_terms(const PassArgs& a, int j, int p, int o) {
  int c[3] = {0, 0, 0};
  if (a.ax_j >= 0) c[a.ax_j] = j;
  if (a.ax_p >= 0) c[a.ax_p] = p;
  if (a.ax_o >= 0) c[a.ax_o] = o;
  double add = 0.0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const T* g = (const T*)a.face[ax][side];
      if (!g) continue;
      const int edge = side == 0 ? 0 : a.nunk[ax] - 1;
      if (c[ax] != edge) continue;
      long long off = 0;
      int r = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (b == ax || a.nunk[b] <= 0) continue;
        if (r < 2) off += (long long)(c[b] + ((a.face_off >> b) & 1)) * a.face_s[ax][r];
        ++r;
      }
      add += a.face_w[ax][side] * (double)g[off];
    }
  }
  return add;
}

}  // namespace hp
