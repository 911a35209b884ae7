// Column walker shared by the residual, restriction and PCG kernels.
#pragma once

#include "gmg_device.h"

namespace gmg {

// Walk column (i, j) of the field v (v(idx) gives its value at a cell) over
// the z-planes [k0, k1) and call f(idx, ax, D, vc) for each cell with
// ax = (A v)(cell), D its diagonal and vc = v(cell), computed with the same
// arithmetic, term by term, as stencil_Ax.  The x and y neighbour offsets are
// fixed for the column, and the z-neighbours and z-faces roll through
// registers as the walk goes up.
template <typename T, typename TL, typename V, typename F>
__device__ __forceinline__ void walk_column_v(const Geom& g, V&& v, const TL* __restrict__ L, int i,
                                              int j, int k0, int k1, F&& f) {
  if (i >= g.nx || j >= g.ny || k0 >= k1) return;
  const Nb nx = neighbours(i, g.nx, g.px, 1);
  const Nb ny = neighbours(j, g.ny, g.py, g.sy);
  const TL* __restrict__ Ly = L + g.n;
  const TL* __restrict__ Lz = L + 2 * g.n;
  const long long base = (long long)j * g.sy + i;
  const long long top = (long long)(g.nz - 1) * g.sz;
  long long idx = (long long)k0 * g.sz + base;
  T xc = v(idx);
  T xb = (k0 > 0) ? v(idx - g.sz) : (g.pz ? v(top + base) : xc);  // z low neighbour
  T lzm = ldL<T>(Lz, idx);
#pragma unroll 2
  for (int k = k0; k < k1; ++k, idx += g.sz) {
    // z high neighbour and face: next plane, wrap, or (wall) self with face 0
    const bool zin = k + 1 < g.nz;
    const long long hi = zin ? idx + g.sz : base;
    const T xt = (zin || g.pz) ? v(hi) : xc;
    const T lzp = (zin || g.pz) ? ldL<T>(Lz, hi) : T(0);
    T ax = T(0), s = T(0);
    {
      const T lm = ldL<T>(L, idx);
      const T lp = nx.hi_ok ? ldL<T>(L, idx + nx.hi) : T(0);
      ax += lp * (v(idx + nx.hi) - xc);
      ax += lm * (v(idx + nx.lo) - xc);
      s += lm + lp;
    }
    {
      const T lm = ldL<T>(Ly, idx);
      const T lp = ny.hi_ok ? ldL<T>(Ly, idx + ny.hi) : T(0);
      ax += lp * (v(idx + ny.hi) - xc);
      ax += lm * (v(idx + ny.lo) - xc);
      s += lm + lp;
    }
    ax += lzp * (xt - xc);
    ax += lzm * (xb - xc);
    s += lzm + lzp;
    f(idx, ax, -s, xc);
    xb = xc;
    xc = xt;
    lzm = lzp;
  }
}

}  // namespace gmg
