// Column walker shared by the residual, restriction and PCG kernels.
#pragma once

#include "gmg_device.h"

namespace gmg {

// Walk column (i, j) of the field v (v(idx) gives its value at a cell) over
// the z-planes [k0, k1) and call f(idx, ax, D, vc, sd) for each cell with
// ax = (A v)(cell), D its diagonal, vc = v(cell) and sd = side(idx) (a second
// per-cell value the caller needs, e.g. sigma), computed with the same
// arithmetic, term by term, as stencil_Ax.  The x and y neighbour offsets are
// fixed for the column, and the z-neighbours and z-faces roll through
// registers as the walk goes up.
//
// The loads of planes k+1 .. k+PF-1 are issued before plane k is computed,
// so each wave keeps PF planes of loads in flight (the walk is otherwise one
// memory latency per plane).  PF = 2: the next plane's loads, the last plane
// peeled off the loop.  PF > 2: a ring of PF plane registers with PF plane
// steps per loop iteration, so that the ring is indexed by constants; the
// planes past the last one are loaded again (clamped: at most PF - 1 extra
// plane loads, which hit the cache) instead of branched around, and the last
// planes, which load nothing, are computed after the loop.  ALL: a walk of
// at most PF planes that issues every load at once.  Every load is issued on every
// path (a missing neighbour's offset points at the cell itself) and the
// value selected afterwards, so no branch forces the compiler to wait for
// all of them.
//
// walk_column_vsf takes the faces through face(d, q, hi), the face of
// direction d stored at cell q, where hi tells a cell's high face (q is the
// neighbour's index) from its low one: the stored faces, or a block's constant
// faces (uniform bricks, whose low walls keep their zero faces), with the same
// arithmetic either way.
template <typename T, int PF = 2, bool ALL = false, typename V, typename S, typename FL,
          typename F>
__device__ __forceinline__ void walk_column_vsf(const Geom& g, V&& v, S&& side, FL&& face, int i,
                                                int j, int k0, int k1, F&& f) {
  static_assert(PF >= 2, "at least the next plane in flight");
  if (i >= g.nx || j >= g.ny || k0 >= k1) return;
  const Nb nx = neighbours(i, g.nx, g.px, 1);
  const Nb ny = neighbours(j, g.ny, g.py, g.sy);
  const long long base = (long long)j * g.sy + i;
  const long long top = (long long)(g.nz - 1) * g.sz;
  // the loads of one plane
  struct Plane {
    T vt, lzt, lmx, lhx, ve, vw, lmy, lhy, vn, vs, sd;
  };
  auto load = [&](int k, Plane& p) {
    const long long id = (long long)k * g.sz + base;
    const long long hi = (k + 1 < g.nz) ? id + g.sz : base;
    p.vt = v(hi);
    p.lzt = face(2, hi, true);
    p.lmx = face(0, id, false);
    p.lhx = face(0, id + nx.hi, true);
    p.ve = v(id + nx.hi);
    p.vw = v(id + nx.lo);
    p.lmy = face(1, id, false);
    p.lhy = face(1, id + ny.hi, true);
    p.vn = v(id + ny.hi);
    p.vs = v(id + ny.lo);
    p.sd = side(id);
  };
  long long idx = (long long)k0 * g.sz + base;
  T xc = v(idx);
  T xb = (k0 > 0) ? v(idx - g.sz) : (g.pz ? v(top + base) : xc);  // z low neighbour
  T lzm = face(2, idx, false);
  // plane k from its loads, then roll the z-neighbours up
  auto plane = [&](int k, const Plane& cur) {
    // z high neighbour and face: next plane, wrap, or (wall) self with face 0
    const bool zok = k + 1 < g.nz || g.pz;
    const T xt = zok ? cur.vt : xc;
    const T lzp = zok ? cur.lzt : T(0);
    T ax = T(0), s = T(0);
    {
      const T lm = cur.lmx;
      const T lp = nx.hi_ok ? cur.lhx : T(0);
      ax += lp * (cur.ve - xc);
      ax += lm * (cur.vw - xc);
      s += lm + lp;
    }
    {
      const T lm = cur.lmy;
      const T lp = ny.hi_ok ? cur.lhy : T(0);
      ax += lp * (cur.vn - xc);
      ax += lm * (cur.vs - xc);
      s += lm + lp;
    }
    ax += lzp * (xt - xc);
    ax += lzm * (xb - xc);
    s += lzm + lzp;
    f(idx, ax, -s, xc, cur.sd);
    xb = xc;
    xc = xt;
    lzm = lzp;
    idx += g.sz;
  };
  if constexpr (ALL) {  // a walk of at most PF planes: every load in flight at once
    Plane ring[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) load(min(k0 + q, k1 - 1), ring[q]);
#pragma unroll
    for (int q = 0; q < PF; ++q)
      if (k0 + q < k1) plane(k0 + q, ring[q]);
  } else if constexpr (PF == 2) {  // the last plane peeled off; no plane loaded twice
    Plane cur, nxt;
    load(k0, cur);
    int k = k0;
    for (; k + 1 < k1; ++k) {
      load(k + 1, nxt);
      plane(k, cur);
      cur = nxt;
    }
    plane(k, cur);
  } else {
    Plane ring[PF];  // ring[q] holds plane k + q at the top of an iteration
#pragma unroll
    for (int q = 0; q + 1 < PF; ++q) load(min(k0 + q, k1 - 1), ring[q]);
    int k = k0;
    for (; k + PF <= k1; k += PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        load(min(k + q + PF - 1, k1 - 1), ring[(q + PF - 1) % PF]);
        plane(k + q, ring[q]);
      }
    }
#pragma unroll
    for (int q = 0; q + 1 < PF; ++q)
      if (k + q < k1) plane(k + q, ring[q]);
  }
}

template <typename T, typename TL, typename V, typename S, typename F>
__device__ __forceinline__ void walk_column_vs(const Geom& g, V&& v, S&& side,
                                               const TL* __restrict__ L, int i, int j, int k0,
                                               int k1, F&& f) {
  walk_column_vsf<T>(
      g, v, side, [&](int d, long long q, bool) { return ldL<T>(L + d * g.n, q); }, i, j, k0,
      k1, f);
}

// walk_column_vs without a side value: f(idx, ax, D, vc).
template <typename T, typename TL, typename V, typename F>
__device__ __forceinline__ void walk_column_v(const Geom& g, V&& v, const TL* __restrict__ L, int i,
                                              int j, int k0, int k1, F&& f) {
  walk_column_vs<T, TL>(g, v, [](long long) { return T(0); }, L, i, j, k0, k1,
                        [&](long long idx, T ax, T D, T vc, T) { f(idx, ax, D, vc); });
}

}  // namespace gmg
