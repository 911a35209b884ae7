// Fused red-black Gauss-Seidel sweep for gfx950.
//
// One launch performs a whole sweep (red half-sweep, then black) out of place:
// W = sweep(S).  Each workgroup owns a 64 x TY tile of (x, y) columns and a
// chunk of z-planes and marches up the chunk with rings of three LDS planes:
//
//   step k:  issue the global loads of plane k+3 (S, sigma, the three face
//            arrays; tile plus halo) into registers -> red update on plane
//            k+1 over the tile and a one-cell ring -> black update on plane k
//            over the tile from the red values of planes k-1, k, k+1, store
//            plane k of W -> write the prefetched plane into the LDS slot that
//            plane k used.
//
// Each thread owns an x-pair of cells (one red, one black on every plane), so
// no lane idles on the wrong colour, and loads/stores are 2-wide.  The red
// values on the ring are recomputed redundantly by neighbouring tiles: no
// workgroup reads another one's output, and no grid-wide synchronisation is
// needed.  HBM traffic per cell is one read of S, sigma and L and one write of
// W (24 B in FP32), half that of two separate half-sweeps; halo re-reads are
// served by L2 / Infinity Cache.
//
// Optionally the prolongation + correction of the coarse-grid correction is
// folded into the load: S(a) += x_c[a / c] on active cells before smoothing
// (the coarse value and the mask are prefetched with the plane and added when
// it is written to LDS).
#pragma once

#include "gmg_device.h"

namespace gmg {

constexpr int SW_TX = 64;  // tile width in x
constexpr int SW_EX = 68;  // LDS row: tile plus a 2-cell halo on each side

// Wrap / clip a coordinate: the in-domain index, or -1 outside a wall.
__device__ __forceinline__ int wrap_coord(int c, int n, int periodic) {
  if (c >= 0 && c < n) return c;
  if (!periodic) return -1;
  c %= n;
  return c < 0 ? c + n : c;
}

__device__ __forceinline__ int ring3(int p) {
  const int m = p % 3;
  return m < 0 ? m + 3 : m;
}

template <int TY, int VEC>
struct SweepCfg {
  static constexpr int NT = 32 * TY;    // threads: one per x-pair of the tile
  static constexpr int IPR = SW_EX / VEC;  // load items per LDS row
  static constexpr int RS = TY + 4;     // S rows: j0-2 .. j0+TY+1
  static constexpr int RF = TY + 2;     // sigma, Lx, Lz, red rows: j0-1 .. j0+TY
  static constexpr int RY = TY + 3;     // Ly rows: j0-1 .. j0+TY+1 (high face)
  static constexpr int NS = (RS * IPR + NT - 1) / NT;
  static constexpr int NF = (RF * IPR + NT - 1) / NT;
  static constexpr int NY = (RY * IPR + NT - 1) / NT;
  static constexpr int NRING = 64 + 2 * TY;  // ring work items of the red phase
};

template <typename T, int TY>
struct SweepSmem {
  T s[3][TY + 4][SW_EX];
  T sg[3][TY + 2][SW_EX];
  T lx[3][TY + 2][SW_EX];
  T ly[3][TY + 3][SW_EX];
  T lz[3][TY + 2][SW_EX];
  T r[3][TY + 2][SW_EX];  // red values after the red half-sweep (red cells only)
};

// VEC consecutive face coefficients as T.
template <typename T, int VEC>
__device__ __forceinline__ void ldLv(const float* p, long long i, T* v) {
  if constexpr (VEC == 2) {
    const float2 a = *reinterpret_cast<const float2*>(p + i);
    v[0] = (T)a.x;
    v[1] = (T)a.y;
  } else {
    v[0] = (T)p[i];
  }
}
template <typename T, int VEC>
__device__ __forceinline__ void ldLv(const double* p, long long i, T* v) {
  if constexpr (VEC == 2) {
    const double2 a = *reinterpret_cast<const double2*>(p + i);
    v[0] = (T)a.x;
    v[1] = (T)a.y;
  } else {
    v[0] = (T)p[i];
  }
}
template <typename T, int VEC>
__device__ __forceinline__ void ldLv(const uint16_t* p, long long i, T* v) {
  if constexpr (VEC == 2) {
    const uint32_t a = *reinterpret_cast<const uint32_t*>(p + i);
    v[0] = (T)__uint_as_float(a << 16);
    v[1] = (T)__uint_as_float(a & 0xFFFF0000u);
  } else {
    v[0] = (T)__uint_as_float(((uint32_t)p[i]) << 16);
  }
}
template <typename T, int VEC>
__device__ __forceinline__ void ldv(const T* p, long long i, T* v) {
  if constexpr (VEC == 2) {
    if constexpr (sizeof(T) == 4) {
      const float2 a = *reinterpret_cast<const float2*>(p + i);
      v[0] = a.x;
      v[1] = a.y;
    } else {
      const double2 a = *reinterpret_cast<const double2*>(p + i);
      v[0] = a.x;
      v[1] = a.y;
    }
  } else {
    v[0] = p[i];
  }
}

// Per-thread load plan of one array: for each item the in-plane element
// offset (or -1 outside a wall) and the LDS position.
template <int N>
struct LoadPlan {
  int ii[N], jj[N];  // in-domain column / row of the item's first element, -1 outside
  int row[N], col[N];
  bool use[N];
};

template <int TY, int VEC, int N>
__device__ __forceinline__ void make_plan(LoadPlan<N>& pl, const Geom& g, int i0, int jbase,
                                          int rows) {
  using C = SweepCfg<TY, VEC>;
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < N; ++u) {
    const int q = tid + u * C::NT;
    pl.use[u] = q < rows * C::IPR;
    const int row = q / C::IPR, it = q - row * C::IPR;
    pl.row[u] = row;
    pl.col[u] = it * VEC;
    // VEC == 2 is only used with an even nx: a pair is wholly in or out
    pl.ii[u] = wrap_coord(i0 - 2 + it * VEC, g.nx, g.px);
    pl.jj[u] = wrap_coord(jbase + row, g.ny, g.py);
  }
}

// Registers holding one prefetched plane.
template <typename T, int TY, int VEC>
struct PlaneRegs {
  using C = SweepCfg<TY, VEC>;
  T s[C::NS][VEC], sg[C::NF][VEC], lx[C::NF][VEC], ly[C::NY][VEC], lz[C::NF][VEC];
  T pc[C::NS][VEC];        // coarse correction of each S element (prolongation only)
  uint32_t pa[C::NS];      // bit e set: element e is active and takes the correction
  uint32_t in;             // bit u (S), 8 + u (sigma, Lx, Lz), 16 + u (Ly): item in the domain
};

template <typename T, typename TL, int TY, int VEC>
struct SweepArgs {
  Geom g;
  const T* S;
  const T* sigma;
  const TL* L;
  const T* xc;
  const uint8_t* active;
  Geom gc;
  int cx, cy, cz;
  double* res_part;  // non-null: FP64 partial of ||sigma - A S||^2 per workgroup
};

template <typename T, typename TL, int TY, int VEC>
__device__ __forceinline__ void fetch_plane(PlaneRegs<T, TY, VEC>& rg,
                                            const SweepArgs<T, TL, TY, VEC>& a, int k,
                                            const LoadPlan<SweepCfg<TY, VEC>::NS>& ps,
                                            const LoadPlan<SweepCfg<TY, VEC>::NF>& pf,
                                            const LoadPlan<SweepCfg<TY, VEC>::NY>& py) {
  using C = SweepCfg<TY, VEC>;
  static_assert(C::NS <= 8 && C::NF <= 8 && C::NY <= 8, "item bits");
  const Geom& g = a.g;
  const int kw = wrap_coord(k, g.nz, g.pz);
  const long long po = (long long)(kw >= 0 ? kw : 0) * g.sz;
  // Every item's main loads are issued, at a clamped in-domain address when
  // the item lies outside a wall (store_plane zeroes those), so the number of
  // loads in flight is the same on every path and the compiler waits only
  // for the plane being stored.
  rg.in = 0;
#pragma unroll
  for (int u = 0; u < C::NS; ++u) {
    rg.pa[u] = 0;
    const bool in = ps.use[u] && ps.ii[u] >= 0 && ps.jj[u] >= 0 && kw >= 0;
    rg.in |= (uint32_t)in << u;
    {
      const int ii = in ? ps.ii[u] : 0, jj = in ? ps.jj[u] : 0;
      const long long idx = po + (long long)jj * g.sy + ii;
      ldv<T, VEC>(a.S, idx, rg.s[u]);
      if (a.xc != nullptr) {
        // Issued unconditionally (every in-domain cell has a coarse parent)
        // and applied when the plane is written to LDS, so no load waits on
        // another inside the prefetch.  Factors are 1 or 2: shift by c >> 1.
        const long long cb = (long long)((kw >= 0 ? kw : 0) >> (a.cz >> 1)) * a.gc.sz +
                             (long long)(jj >> (a.cy >> 1)) * a.gc.sy;
        if constexpr (VEC == 2)
          rg.pa[u] = *reinterpret_cast<const uint16_t*>(a.active + idx);
        else
          rg.pa[u] = a.active[idx];
#pragma unroll
        for (int e = 0; e < VEC; ++e) rg.pc[u][e] = a.xc[cb + ((ii + e) >> (a.cx >> 1))];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < C::NF; ++u) {
    const bool in = pf.use[u] && pf.ii[u] >= 0 && pf.jj[u] >= 0 && kw >= 0;
    rg.in |= (uint32_t)in << (8 + u);
    const long long idx = po + (long long)(in ? pf.jj[u] : 0) * g.sy + (in ? pf.ii[u] : 0);
    ldv<T, VEC>(a.sigma, idx, rg.sg[u]);
    ldLv<T, VEC>(a.L, idx, rg.lx[u]);
    ldLv<T, VEC>(a.L + 2 * g.n, idx, rg.lz[u]);
  }
#pragma unroll
  for (int u = 0; u < C::NY; ++u) {
    const bool in = py.use[u] && py.ii[u] >= 0 && py.jj[u] >= 0 && kw >= 0;
    rg.in |= (uint32_t)in << (16 + u);
    ldLv<T, VEC>(a.L + g.n, po + (long long)(in ? py.jj[u] : 0) * g.sy + (in ? py.ii[u] : 0),
                 rg.ly[u]);
  }
}

template <typename T, int TY, int VEC>
__device__ __forceinline__ void store_plane(SweepSmem<T, TY>& sm, int slot, bool prol,
                                            const PlaneRegs<T, TY, VEC>& rg,
                                            const LoadPlan<SweepCfg<TY, VEC>::NS>& ps,
                                            const LoadPlan<SweepCfg<TY, VEC>::NF>& pf,
                                            const LoadPlan<SweepCfg<TY, VEC>::NY>& py) {
  using C = SweepCfg<TY, VEC>;
  // items outside a wall were loaded at a clamped address: store zeros
#pragma unroll
  for (int u = 0; u < C::NS; ++u)
    if (ps.use[u]) {
      const bool in = (rg.in >> u) & 1u;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        // active-mask bytes: element e is byte e of pa (nonzero = active)
        const bool corr = prol && ((rg.pa[u] >> (8 * e)) & 0xFFu) != 0;
        const T v = corr ? rg.s[u][e] + rg.pc[u][e] : rg.s[u][e];
        sm.s[slot][ps.row[u]][ps.col[u] + e] = in ? v : T(0);
      }
    }
#pragma unroll
  for (int u = 0; u < C::NF; ++u)
    if (pf.use[u]) {
      const bool in = (rg.in >> (8 + u)) & 1u;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        sm.sg[slot][pf.row[u]][pf.col[u] + e] = in ? rg.sg[u][e] : T(0);
        sm.lx[slot][pf.row[u]][pf.col[u] + e] = in ? rg.lx[u][e] : T(0);
        sm.lz[slot][pf.row[u]][pf.col[u] + e] = in ? rg.lz[u][e] : T(0);
      }
    }
#pragma unroll
  for (int u = 0; u < C::NY; ++u)
    if (py.use[u]) {
      const bool in = (rg.in >> (16 + u)) & 1u;
#pragma unroll
      for (int e = 0; e < VEC; ++e) sm.ly[slot][py.row[u]][py.col[u] + e] = in ? rg.ly[u][e] : T(0);
    }
}

// Relaxed Gauss-Seidel update of a red cell from S (rows of the S ring are
// offset by one from the face rows: fr = sr - 1).
template <typename T, int TY>
__device__ __forceinline__ T red_update(const SweepSmem<T, TY>& sm, int dm, int d, int dp, int sr,
                                        int ex, T omega) {
  const int fr = sr - 1;
  return relax_cell<T>(sm.s[d][sr][ex], sm.s[d][sr][ex + 1], sm.s[d][sr][ex - 1],
                       sm.s[d][sr + 1][ex], sm.s[d][sr - 1][ex], sm.s[dp][sr][ex],
                       sm.s[dm][sr][ex], sm.lx[d][fr][ex], sm.lx[d][fr][ex + 1],
                       sm.ly[d][fr][ex], sm.ly[d][fr + 1][ex], sm.lz[d][fr][ex],
                       sm.lz[dp][fr][ex], sm.sg[d][fr][ex], omega);
}

// Black update from the red values (rows of the red ring = face rows).
template <typename T, int TY>
__device__ __forceinline__ T black_update(const SweepSmem<T, TY>& sm, int dm, int d, int dp,
                                          int fr, int ex, T omega) {
  return relax_cell<T>(sm.s[d][fr + 1][ex], sm.r[d][fr][ex + 1], sm.r[d][fr][ex - 1],
                       sm.r[d][fr + 1][ex], sm.r[d][fr - 1][ex], sm.r[dp][fr][ex],
                       sm.r[dm][fr][ex], sm.lx[d][fr][ex], sm.lx[d][fr][ex + 1],
                       sm.ly[d][fr][ex], sm.ly[d][fr + 1][ex], sm.lz[d][fr][ex],
                       sm.lz[dp][fr][ex], sm.sg[d][fr][ex], omega);
}

// Squared residual sigma - A S of the input (active cells) at the thread's
// x-pair of plane p, from the LDS rings (same term order as the updates).
template <typename T, int TY>
__device__ __forceinline__ double input_residual_sq(const SweepSmem<T, TY>& sm, const Geom& g,
                                                   int i0, int j0, int p) {
  const int tid = threadIdx.x;
  const int px = tid & 31, ty = tid >> 5;
  const int j = j0 + ty;
  if (j >= g.ny) return 0.0;
  const int d = ring3(p), dm = ring3(p - 1), dp = ring3(p + 1);
  const int sr = ty + 2, fr = ty + 1;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int ex = 2 + 2 * px + e;
    if (i0 + 2 * px + e >= g.nx) continue;
    const T xc = sm.s[d][sr][ex];
    const T lxm = sm.lx[d][fr][ex], lxp = sm.lx[d][fr][ex + 1];
    const T lym = sm.ly[d][fr][ex], lyp = sm.ly[d][fr + 1][ex];
    const T lzm = sm.lz[d][fr][ex], lzp = sm.lz[dp][fr][ex];
    T ax = T(0);
    ax += lxp * (sm.s[d][sr][ex + 1] - xc);
    ax += lxm * (sm.s[d][sr][ex - 1] - xc);
    ax += lyp * (sm.s[d][sr + 1][ex] - xc);
    ax += lym * (sm.s[d][sr - 1][ex] - xc);
    ax += lzp * (sm.s[dp][sr][ex] - xc);
    ax += lzm * (sm.s[dm][sr][ex] - xc);
    const T s = ((lxm + lxp) + (lym + lyp)) + (lzm + lzp);
    const T r = (s != T(0)) ? sm.sg[d][fr][ex] - ax : T(0);
    acc += (double)r * (double)r;
  }
  return acc;
}

// Red phase for plane p: interior pairs (one red cell each) and the ring.
template <typename T, int TY>
__device__ __forceinline__ void red_phase(SweepSmem<T, TY>& sm, int i0, int j0, int p, T omega) {
  const int tid = threadIdx.x;
  const int d = ring3(p), dm = ring3(p - 1), dp = ring3(p + 1);
  {
    const int px = tid & 31, ty = tid >> 5;
    const int j = j0 + ty;
    const int ex = 2 + 2 * px + ((i0 + j + p) & 1);
    sm.r[d][ty + 1][ex] = red_update<T, TY>(sm, dm, d, dp, ty + 2, ex, omega);
  }
  if (tid < SweepCfg<TY, 1>::NRING) {
    int fr, ex;
    bool red = true;
    if (tid < 64) {  // ring rows below (j0-1) and above (j0+TY)
      const int px = tid & 31;
      fr = (tid < 32) ? 0 : TY + 1;
      const int j = j0 - 1 + fr;
      ex = 2 + 2 * px + ((i0 + j + p) & 1);
    } else {  // ring columns left (i0-1) and right (i0+64)
      const int q = tid - 64;
      const int right = q >= TY;
      const int ty = right ? q - TY : q;
      fr = ty + 1;
      ex = right ? SW_TX + 2 : 1;
      const int i = i0 - 2 + ex, j = j0 + ty;
      red = ((i + j + p) & 1) == 0;
    }
    if (red) sm.r[d][fr][ex] = red_update<T, TY>(sm, dm, d, dp, fr + 1, ex, omega);
  }
}

// One plane step k of the sweep: red update of plane k+1, black update and
// store of plane k (k >= k0), then the plane held in `cur` (plane k+3, loaded
// two steps earlier) goes to the LDS slot plane k used, while `nxt` receives
// plane k+4.  Two register sets alternate, so each load has two steps of
// compute to arrive.
template <typename T, typename TL, int TY, int VEC>
__device__ __forceinline__ void sweep_step(SweepSmem<T, TY>& sm, const SweepArgs<T, TL, TY, VEC>& a,
                                           T* __restrict__ W, int i0, int j0, int k0, int k1, int k,
                                           T omega, PlaneRegs<T, TY, VEC>& cur,
                                           PlaneRegs<T, TY, VEC>& nxt, double& racc,
                                           const LoadPlan<SweepCfg<TY, VEC>::NS>& ps,
                                           const LoadPlan<SweepCfg<TY, VEC>::NF>& pf,
                                           const LoadPlan<SweepCfg<TY, VEC>::NY>& py) {
  const Geom& g = a.g;
  const int tid = threadIdx.x;
  const int px = tid & 31, ty = tid >> 5;
  const int j = j0 + ty;
  const int ib = i0 + 2 * px;
  if (k + 4 <= k1 + 1) fetch_plane<T, TL, TY, VEC>(nxt, a, k + 4, ps, pf, py);
  red_phase<T, TY>(sm, i0, j0, k + 1, omega);
  // input residual of plane k+1 (its S neighbours k .. k+2 are all present)
  if (a.res_part != nullptr && k + 1 < k1) racc += input_residual_sq<T, TY>(sm, g, i0, j0, k + 1);
  __syncthreads();
  if (k >= k0) {
    const int d = ring3(k), dm = ring3(k - 1), dp = ring3(k + 1);
    const int ob = (i0 + j + k + 1) & 1;  // black offset within the pair
    const int exb = 2 + 2 * px + ob, exr = 2 + 2 * px + (ob ^ 1);
    const T vb = black_update<T, TY>(sm, dm, d, dp, ty + 1, exb, omega);
    const T vr = sm.r[d][ty + 1][exr];
    T w[2];
    w[ob] = vb;
    w[ob ^ 1] = vr;
    if (j < g.ny) {
      const long long idx = (long long)k * g.sz + (long long)j * g.sy + ib;
      if constexpr (VEC == 2) {
        if (ib + 1 < g.nx) {
          if constexpr (sizeof(T) == 4)
            *reinterpret_cast<float2*>(W + idx) = make_float2(w[0], w[1]);
          else
            *reinterpret_cast<double2*>(W + idx) = make_double2(w[0], w[1]);
        }
      } else {
        if (ib < g.nx) W[idx] = w[0];
        if (ib + 1 < g.nx) W[idx + 1] = w[1];
      }
    }
  }
  __syncthreads();
  if (k + 3 <= k1 + 1) store_plane<T, TY, VEC>(sm, ring3(k + 3), a.xc != nullptr, cur, ps, pf, py);
  __syncthreads();
}

// Sweep of the tile with origin (i0, j0) over the z-planes [k0, k1).
template <typename T, typename TL, int TY, int VEC>
__device__ __forceinline__ void rb_sweep_tile(SweepSmem<T, TY>& sm,
                                              const SweepArgs<T, TL, TY, VEC>& a,
                                              T* __restrict__ W, int i0, int j0, int k0, int k1,
                                              T omega) {
  using C = SweepCfg<TY, VEC>;
  const Geom& g = a.g;

  LoadPlan<C::NS> ps;
  LoadPlan<C::NF> pf;
  LoadPlan<C::NY> py;
  make_plan<TY, VEC, C::NS>(ps, g, i0, j0 - 2, C::RS);
  make_plan<TY, VEC, C::NF>(pf, g, i0, j0 - 1, C::RF);
  make_plan<TY, VEC, C::NY>(py, g, i0, j0 - 1, C::RY);

  // Prologue: establish, for k = k0, that LDS holds planes k .. k+2, the red
  // values of planes k-1 and k are computed, and plane k+3 is in flight.
  PlaneRegs<T, TY, VEC> ra, rb;
  fetch_plane<T, TL, TY, VEC>(ra, a, k0 - 2, ps, pf, py);
  fetch_plane<T, TL, TY, VEC>(rb, a, k0 - 1, ps, pf, py);
  store_plane<T, TY, VEC>(sm, ring3(k0 - 2), a.xc != nullptr, ra, ps, pf, py);
  store_plane<T, TY, VEC>(sm, ring3(k0 - 1), a.xc != nullptr, rb, ps, pf, py);
  fetch_plane<T, TL, TY, VEC>(ra, a, k0, ps, pf, py);
  fetch_plane<T, TL, TY, VEC>(rb, a, k0 + 1, ps, pf, py);
  store_plane<T, TY, VEC>(sm, ring3(k0), a.xc != nullptr, ra, ps, pf, py);
  __syncthreads();
  red_phase<T, TY>(sm, i0, j0, k0 - 1, omega);  // reads planes k0-2 .. k0
  __syncthreads();
  store_plane<T, TY, VEC>(sm, ring3(k0 + 1), a.xc != nullptr, rb, ps, pf, py);  // slot of plane k0-2
  fetch_plane<T, TL, TY, VEC>(ra, a, k0 + 2, ps, pf, py);
  __syncthreads();
  red_phase<T, TY>(sm, i0, j0, k0, omega);  // reads planes k0-1 .. k0+1
  double racc = 0.0;
  if (a.res_part != nullptr && k0 < k1) racc = input_residual_sq<T, TY>(sm, g, i0, j0, k0);
  __syncthreads();
  store_plane<T, TY, VEC>(sm, ring3(k0 + 2), a.xc != nullptr, ra, ps, pf, py);  // slot of plane k0-1
  fetch_plane<T, TL, TY, VEC>(ra, a, k0 + 3, ps, pf, py);
  __syncthreads();
  int k;
  for (k = k0; k < k1; k += 2) {
    sweep_step<T, TL, TY, VEC>(sm, a, W, i0, j0, k0, k1, k, omega, ra, rb, racc, ps, pf, py);
    if (k + 1 < k1)
      sweep_step<T, TL, TY, VEC>(sm, a, W, i0, j0, k0, k1, k + 1, omega, rb, ra, racc, ps, pf,
                                 py);
  }
  if (a.res_part != nullptr) {  // one FP64 partial per workgroup, fixed order
    const double sum = block_sum(racc, threadIdx.x, C::NT);
    if (threadIdx.x == 0) a.res_part[blockIdx.x] = sum;
  }
}

}  // namespace gmg

// The fused sweep kernel: X[rd] = sweep(X[rs] (+ P x_c)), at global scope
// so that its symbol carries no namespace.  With res_part it also leaves one
// partial of ||sigma - A X[rs]||^2 per workgroup; with gate it runs only
// when *gate is nonzero.
template <typename T, typename TL, int TY, int VEC>
__global__ __launch_bounds__(32 * TY) void k_rb_sweep(gmg::Geom g, gmg::Roles<T> X, int rs, int rd,
                                                      const T* __restrict__ sigma,
                                                      const TL* __restrict__ L,
                                                      const T* __restrict__ xc,
                                                      const uint8_t* __restrict__ active, gmg::Geom gc,
                                                      int cx, int cy, int cz, int kchunk,
                                                      const double* omega_p, const int* done,
                                                      double* res_part, const int* gate) {
  if (gmg::stopped(done)) return;
  if (gate != nullptr && *gate == 0) return;  // a conditional sweep that is not needed
  __shared__ gmg::SweepSmem<T, TY> sm;
  gmg::SweepArgs<T, TL, TY, VEC> a{g, X.get(rs), sigma, L, xc, active, gc, cx, cy, cz, res_part};
  // 1-D grid of tiles, x fastest, then y, then z-chunks, in XCD-aware order
  const int ntx = (g.nx + gmg::SW_TX - 1) / gmg::SW_TX, nty = (g.ny + TY - 1) / TY;
  const int t = gmg::xcd_tile(blockIdx.x, gridDim.x);
  const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
  const int k0 = tz * kchunk;
  gmg::rb_sweep_tile<T, TL, TY, VEC>(sm, a, X.get(rd), tx * gmg::SW_TX, ty * TY, k0,
                                     min(g.nz, k0 + kchunk), (T)(*omega_p));
}
