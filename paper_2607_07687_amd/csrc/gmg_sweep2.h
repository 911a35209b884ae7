// Two red-black Gauss-Seidel sweeps in one pass (temporal blocking):
// W = sweep(sweep(S)), for the nu = 2 pre- and post-smoothing of a level.
//
// A fused single sweep must read S, sigma and the three face arrays and
// write W once per sweep.  Two consecutive sweeps of a V-cycle use the same
// sigma, faces and omega, so one pass can do both and move those bytes once.
//
// Each workgroup owns a 64 x TY tile of (x, y) columns and a chunk of
// z-planes.  One thread holds one x-pair column (two cells, one of each
// colour on every plane) of the tile grown by four cells on each side, and
// marches up the chunk.  A plane step k performs four half-sweeps, each one
// plane behind the previous and one cell ring narrower:
//
//   stage 1  red cells of sweep 1 on plane k+3, tile + 3 cells
//   stage 2  black cells of sweep 1 on plane k+2, tile + 2 cells
//   stage 3  red cells of sweep 2 on plane k+1, tile + 1 cell
//   stage 4  black cells of sweep 2 on plane k, the tile; plane k of W stored
//
// A cell's z-neighbours are in its own column, so the thread keeps the
// inputs of five planes (S, sigma, faces) and the stage results of three
// planes in registers.  x- and y-neighbours come from the neighbouring
// threads through LDS: each step writes the values the next step's stages
// read (S of the newest plane, and every stage's new results) into one half
// of double-buffered LDS arrays and reads the half written by the previous
// step, so a step needs one workgroup barrier.  High faces (Lx at x+1, Ly at
// y+1) of the newest plane come through LDS the same way.
//
// Every update is relax_cell on the same operands as in two fused sweeps,
// so the result is bitwise theirs.  Cells outside a wall hold zeros (their
// faces are zero and relax_cell leaves them at their input).  Neighbouring
// tiles recompute the grown rings redundantly; no workgroup reads another
// one's output.
//
// Requires an even nx (x-pairs never straddle the domain edge).  Optionally
// folds the prolongation + correction into the load of S, as the fused
// sweep does.
#pragma once

#include <type_traits>

#include "gmg_kernels.h"  // UBrick
#include "gmg_sweep.h"    // wrap_coord (and gmg_device.h: relax_cell, xcd_tile)

namespace gmg {

constexpr int S2_TX = 64;  // tile width in x
constexpr int S2_PX = 36;  // x-pairs per row of the grown region (64 + 2 x 4 cells)

// Tile heights: TY = 8 (9 waves) keeps two planes of loads in flight per
// thread; TY = 16 (14 waves, 25 % less grown-ring work per tile cell) has
// the registers for one only.
//
// With TY = 16 the even and the odd rows of the grown region go to separate
// whole waves (7 each).  In a pair column the red cell is the first or the
// second by the parity of x + y + k, and x + y has the parity of the row, so
// every lane of a wave then updates the same element of its pair: the stages
// branch once on it, uniformly, instead of selecting per lane.  (With TY = 8
// the split would cost a tenth wave, more than the selects save.)
template <int TY>
struct S2Cfg {
  static_assert(TY == 8 || TY == 16, "two-sweep tile height");
  static constexpr int RY = TY + 8;                // rows of the grown region
  static constexpr int NT = S2_PX * RY;            // threads holding a column
  static constexpr bool SPLIT = TY == 16;          // waves of one row parity
  static constexpr int NH = S2_PX * (RY / 2);      // columns of one row parity
  static constexpr int H = (NH + 63) / 64 * 64;    // threads of one row parity
  static constexpr int NTB = SPLIT ? 2 * H : (NT + 63) / 64 * 64;  // workgroup size
  static constexpr int NSET = TY == 8 ? 2 : 1;     // load sets in flight
};

// Rows and columns carry one entry of padding on each side, so that every
// thread's neighbours are in bounds without clamping and each neighbour is
// the thread's own entry plus a constant offset.  Padding is never written;
// only threads outside every stage's region would read it.
template <typename T, int TY>
struct S2Smem {
  T s[2][TY + 10][2 * S2_PX + 2];   // S of the newest plane
  T ly[2][TY + 10][2 * S2_PX + 2];  // Ly of the newest plane (high y-faces of the row below)
  T lx0[2][TY + 10][S2_PX + 2];     // Lx of each pair's first cell (high x-face of the pair before)
  T r1[2][TY + 10][S2_PX + 2];      // sweep-1 red value of each pair
  T b1[2][TY + 10][S2_PX + 2];      // sweep-1 black value of each pair
  T r2[2][TY + 10][S2_PX + 2];      // sweep-2 red value of each pair
};

// Inputs of one plane of a thread's pair column.
template <typename T>
struct S2Plane {
  T s[2], sg[2], lx[2], ly[2], lz[2];
  T lxh;     // Lx at x+2: high x-face of the pair's second cell
  T lyh[2];  // Ly at y+1: high y-faces
};

// Loads of one plane in flight (the prolongation operands separate, so
// that no load waits on another).
template <typename T>
struct S2Load {
  T s[2], sg[2], lx[2], ly[2], lz[2];
  T pc[2];      // coarse value of each cell (prolongation)
  uint32_t pa;  // active-mask bytes of the pair
};

// The per-plane inputs are read with raw buffer loads.  Such a load whose
// offset lies at or past its descriptor's size returns zero and touches no
// memory, which gives the zeros of columns and planes outside a wall with no
// per-lane selects: an outside column uses lane offset S2_OUT, an outside
// plane the descriptor `zero` of size 0.  Every in-domain offset (plane offset
// plus lane offset) stays below the field's size, so the result does not
// depend on whether the hardware counts the plane (scalar) offset in its
// range check, and S2_OUT plus any plane offset stays below 2^32.  This needs
// every field to be at most 2^30 bytes (n <= 2^28 cells; the host enables
// the pass only then).
constexpr int S2_OUT = 1 << 30;
constexpr long long S2_MAX_CELLS = 1LL << 28;
// descriptor word 3 of the gfx9 family: 32-bit data format, raw addressing
constexpr int S2_RSRC_W3 = 0x00020000;

struct S2Bufs {
  __amdgpu_buffer_rsrc_t S, sg, lx, ly, lz, act, zero;
};

template <typename T>
__device__ __forceinline__ void s2_ld2(__amdgpu_buffer_rsrc_t b, int vo, int so, T* v) {
  static_assert(sizeof(T) == 4, "the two-sweep pass runs FP32 cycles");
  const float2 f = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(b, vo, so, 0));
  v[0] = f.x;
  v[1] = f.y;
}
// faces: FP32, or BF16 bits (two in one dword)
template <typename T, typename TL>
__device__ __forceinline__ void s2_ldL2(__amdgpu_buffer_rsrc_t b, int vo4, int vo2, int so4,
                                        int so2, T* v) {
  if constexpr (sizeof(TL) == 4) {
    s2_ld2<T>(b, vo4, so4, v);
  } else {
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(b, vo2, so2, 0);
    v[0] = __uint_as_float(w << 16);
    v[1] = __uint_as_float(w & 0xFFFF0000u);
  }
}

template <typename T, typename TL>
struct S2Args {
  Geom g;
  const T* S;
  const T* sigma;
  const TL* L;
  const T* xc;
  const uint8_t* active;
  Geom gc;
  int cx, cy, cz;
  // PROL: 0 adds no correction (the mask then reads zero everywhere; xc and
  // gc must still describe readable memory, e.g. the level's own iterate and
  // geometry with factors 1)
  int corr = 1;
};

// The faces of a thread's pair column in a tile of uniform bricks (see
// UBrick), as the loads would return them: u_d, +0 on a low wall, and zeros
// outside a wall (columns and, per plane, planes); lxh and lyh, the high x-
// and y-faces the LDS exchange would deliver (the low faces of the pair to
// the east and of the row above).
template <typename T>
struct S2Uni {
  T lx0, lx1, ly, lz;
  T lxh, lyh;
  uint32_t pa;  // S2_CONST with the correction: the active-mask bytes of the pair
};

// Face modes of the pass: loaded (S2_LOADED), uniform with per-plane wall
// handling (S2_UNIFORM), or uniform on a tile whose fetched planes are all
// inside the domain (S2_CONST): then every face a thread uses is the same
// value on every plane, the exchange of faces is skipped, and the compiler
// hoists each cell's diagonal and its reciprocal out of the plane loop.  With
// the folded correction S2_CONST also needs every cell of the region's
// bricks active, and then takes the active mask as 1 on the domain's cells
// instead of loading it.
constexpr int S2_LOADED = 0, S2_UNIFORM = 1, S2_CONST = 2;

// Issue the loads of plane m for the column with lane offsets vo4, vo2, vo1
// (its in-plane offset in 4-, 2- and 1-byte elements, S2_OUT outside a wall)
// and coarse in-plane offset `coff` (PROL: also the prolongation operands).
// Every lane issues every load, so the number of loads in flight is the same
// on every path and the compiler waits for exactly the plane being taken.
// UM (face mode) other than S2_LOADED: the faces are the constants of f
// instead of loads.
template <typename T, typename TL, bool PROL, int UM>
__device__ __forceinline__ void s2_fetch(S2Load<T>& ld, const S2Args<T, TL>& a, const S2Bufs& b,
                                         int m, int vo4, int vo2, int vo1, int coff,
                                         const S2Uni<T>& f) {
  const Geom& g = a.g;
  const int mw = wrap_coord(m, g.nz, g.pz);  // uniform
  const bool pin = mw >= 0;
  const int mm = pin ? mw : 0;
  const int so1 = mm * (int)g.sz, so2 = 2 * so1, so4 = 4 * so1;
  s2_ld2<T>(pin ? b.S : b.zero, vo4, so4, ld.s);
  s2_ld2<T>(pin ? b.sg : b.zero, vo4, so4, ld.sg);
  if constexpr (UM == S2_CONST) {
    ld.lx[0] = f.lx0;
    ld.lx[1] = f.lx1;
    ld.ly[0] = ld.ly[1] = f.ly;
    ld.lz[0] = ld.lz[1] = f.lz;
  } else if constexpr (UM == S2_UNIFORM) {
    ld.lx[0] = pin ? f.lx0 : T(0);
    ld.lx[1] = pin ? f.lx1 : T(0);
    ld.ly[0] = ld.ly[1] = pin ? f.ly : T(0);
    ld.lz[0] = ld.lz[1] = (pin && (mw > 0 || g.pz)) ? f.lz : T(0);
  } else {
    s2_ldL2<T, TL>(pin ? b.lx : b.zero, vo4, vo2, so4, so2, ld.lx);
    s2_ldL2<T, TL>(pin ? b.ly : b.zero, vo4, vo2, so4, so2, ld.ly);
    s2_ldL2<T, TL>(pin ? b.lz : b.zero, vo4, vo2, so4, so2, ld.lz);
  }
  if constexpr (PROL) {
    // factors are 1 or 2; the pair's second cell has the next parent only
    // when c_x = 1.  Outside a wall the mask reads zero, and the coarse
    // value (at a clamped address) is not used.
    const long long cb = (long long)(mm >> (a.cz >> 1)) * a.gc.sz + coff;
    if constexpr (UM == S2_CONST)
      ld.pa = f.pa;
    else
      ld.pa = __builtin_amdgcn_raw_buffer_load_b16(pin ? b.act : b.zero, vo1, so1, 0);
#pragma unroll
    for (int e = 0; e < 2; ++e) ld.pc[e] = a.xc[cb + (a.cx == 1 ? e : 0)];
  }
}

// Loaded plane -> column registers (PROL: S corrected on active cells).  The
// high faces are completed later from the exchange (S2_CONST: from f).
template <typename T, bool PROL, int UM>
__device__ __forceinline__ void s2_take(S2Plane<T>& p, const S2Load<T>& ld, const S2Uni<T>& f) {
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if constexpr (PROL)
      p.s[e] = ((ld.pa >> (8 * e)) & 0xFFu) != 0 ? ld.s[e] + ld.pc[e] : ld.s[e];
    else
      p.s[e] = ld.s[e];
    p.sg[e] = ld.sg[e];
    p.lx[e] = ld.lx[e];
    p.ly[e] = ld.ly[e];
    p.lz[e] = ld.lz[e];
    p.lyh[e] = UM == S2_CONST ? f.lyh : T(0);
  }
  p.lxh = UM == S2_CONST ? f.lxh : T(0);
}

// Element e of a pair held in registers: a select when e is known only at
// run time (an indexed access would move the pair to scratch memory), a
// plain register when it is a constant.
template <typename T>
__device__ __forceinline__ T pick(const T (&v)[2], int e) {
  return e ? v[1] : v[0];
}

// Residual sigma - A S of element e of a pair on a completed plane (x: the
// pair's S values xc and its neighbours; faces low and high per direction),
// summed in the order of stencil_Ax (per direction the high-face term, then
// the low-face one); `act` is D != 0.
template <typename T>
__device__ __forceinline__ T s2_residual(T xc, T xe, T xw, T xn, T xs, T xt, T xb, T lxm, T lxp,
                                         T lym, T lyp, T lzm, T lzp, T sg, bool& act) {
  T ax = T(0), d = T(0);
  ax += lxp * (xe - xc);
  ax += lxm * (xw - xc);
  d += lxm + lxp;
  ax += lyp * (xn - xc);
  ax += lym * (xs - xc);
  d += lym + lyp;
  ax += lzp * (xt - xc);
  ax += lzm * (xb - xc);
  d += lzm + lzp;
  act = -d != T(0);
  return sg - ax;
}

// Sweeps 1 and 2 of the tile with origin (i0, j0) over the z-planes [k0, k1)
// (PROL: with the coarse correction folded into S).  RES: also the sum of the
// squared residuals of S over the tile's own active cells and planes (the
// norm of the pass's input), returned to thread 0 (0 elsewhere).  UM other
// than S2_LOADED: the tile's grown region lies in uniform bricks of constants
// uc (s2_uniform_tile), whose faces are then not loaded; S2_CONST also needs
// every fetched plane inside the domain (s2_const_planes).
template <typename T, typename TL, int TY, bool PROL, bool RES = false, int UM = S2_LOADED>
__device__ __forceinline__ double rb_sweep2_tile(S2Smem<T, TY>& sm, const S2Args<T, TL>& a,
                                                 T* __restrict__ W, int i0, int j0, int k0,
                                                 int k1, T omega, const double* uc = nullptr) {
  using C = S2Cfg<TY>;
  const Geom& g = a.g;
  const int t = threadIdx.x;
  // row parity of the wave (SPLIT; C::H is a multiple of the wave size, so
  // it is uniform) and the thread's index among the threads of that parity
  const int hw = C::SPLIT ? __builtin_amdgcn_readfirstlane(t / C::H) : 0;
  const int u = t - hw * C::H;
  // padding threads only join the barriers
  const bool col = C::SPLIT ? u < C::NH : t < C::NT;
  const int p = !col ? 0 : C::SPLIT ? u % S2_PX : t % S2_PX;
  const int r = !col ? hw : C::SPLIT ? 2 * (u / S2_PX) + hw : t / S2_PX;
  const int xa = i0 - 4 + 2 * p;  // x of the pair's first cell
  const int y = j0 - 4 + r;
  const int ii = wrap_coord(xa, g.nx, g.px), jj = wrap_coord(y, g.ny, g.py);
  const int off = (col && ii >= 0 && jj >= 0) ? (int)(jj * g.sy) + ii : -1;
  const int coff = (off >= 0) ? (int)((jj >> (a.cy >> 1)) * a.gc.sy) + (ii >> (a.cx >> 1)) : 0;
  const int vo1 = off >= 0 ? off : S2_OUT, vo2 = off >= 0 ? 2 * off : S2_OUT,
            vo4 = off >= 0 ? 4 * off : S2_OUT;
  S2Uni<T> fu{};
  if constexpr (UM != S2_LOADED) {
    const bool in = off >= 0;
    fu.lx0 = (in && (ii > 0 || g.px)) ? T(uc[0]) : T(0);
    fu.lx1 = in ? T(uc[0]) : T(0);
    fu.ly = (in && (jj > 0 || g.py)) ? T(uc[1]) : T(0);
    fu.lz = in ? T(uc[2]) : T(0);
    const int xe = wrap_coord(xa + 2, g.nx, g.px), yn = wrap_coord(y + 1, g.ny, g.py);
    fu.lxh = (jj >= 0 && xe >= 0 && (xe > 0 || g.px)) ? T(uc[0]) : T(0);
    fu.lyh = (ii >= 0 && yn >= 0 && (yn > 0 || g.py)) ? T(uc[1]) : T(0);
    fu.pa = in ? 0x0101u : 0u;
  }
  const int nb = (int)g.n;  // at most S2_MAX_CELLS
  const S2Bufs b{__builtin_amdgcn_make_buffer_rsrc((void*)a.S, 0, 4 * nb, S2_RSRC_W3),
                 __builtin_amdgcn_make_buffer_rsrc((void*)a.sigma, 0, 4 * nb, S2_RSRC_W3),
                 __builtin_amdgcn_make_buffer_rsrc((void*)a.L, 0, (int)sizeof(TL) * nb, S2_RSRC_W3),
                 __builtin_amdgcn_make_buffer_rsrc((void*)(a.L + g.n), 0, (int)sizeof(TL) * nb,
                                                   S2_RSRC_W3),
                 __builtin_amdgcn_make_buffer_rsrc((void*)(a.L + 2 * g.n), 0,
                                                   (int)sizeof(TL) * nb, S2_RSRC_W3),
                 __builtin_amdgcn_make_buffer_rsrc((void*)a.active, 0, a.corr ? nb : 0,
                                                   S2_RSRC_W3),
                 __builtin_amdgcn_make_buffer_rsrc((void*)a.S, 0, 0, S2_RSRC_W3)};
  // LDS indices (padded by one): the thread's row R and its neighbours RN
  // (y+1) and RS (y-1); its pair column c and the pairs to the west cw and
  // east ce; cs, the cell column of its pair's first cell
  const int R = r + 1, RN = r + 2, RS = r;
  const int c = p + 1, cw = p, ce = p + 2, cs = 2 * p + 1;
  // cell e of the pair lies in the tile grown by d cells
  auto in_ring = [&](int e, int d) {
    const int x = xa + e;
    return x >= i0 - d && x < i0 + S2_TX + d && y >= j0 - d && y < j0 + TY + d;
  };
  const bool in3[2] = {in_ring(0, 3), in_ring(1, 3)}, in2[2] = {in_ring(0, 2), in_ring(1, 2)};
  const bool in1[2] = {in_ring(0, 1), in_ring(1, 1)};
  const bool out_ok = col && in_ring(0, 0) && y < g.ny && xa < g.nx;
  // parity of x + y of the pair's first cell (colour by unwrapped
  // coordinates; every periodic extent is even, and tile origins are even, so
  // it is the parity of r: hw with SPLIT)
  const int par = C::SPLIT ? hw : (xa + y) & 1;

  double racc = 0.0;               // RES: squared input residuals of own cells
  S2Plane<T> P0, P1, P2, P3, P4;  // planes k .. k+4 at step k
  T r1a = T(0), r1b = T(0);       // sweep-1 red of planes k+1, k+2
  T b1a = T(0), b1b = T(0);       // sweep-1 black of planes k, k+1
  T r2a = T(0), r2b = T(0);       // sweep-2 red of planes k-1, k
  S2Load<T> la, lb;
  {
    // planes before the first fetched one (never computed on); S2_CONST gives
    // them the tile's faces, so that every plane register holds the same
    // faces and the per-cell diagonals stay loop-invariant
    S2Plane<T> z{};
    if constexpr (UM == S2_CONST) {
      z.lx[0] = fu.lx0;
      z.lx[1] = fu.lx1;
      z.ly[0] = z.ly[1] = fu.ly;
      z.lz[0] = z.lz[1] = fu.lz;
      z.lxh = fu.lxh;
      z.lyh[0] = z.lyh[1] = fu.lyh;
    }
    P0 = P1 = P2 = z;
  }
  // prologue: planes k0-4 and k0-3 in registers (with two load sets, k0-2 in
  // flight); the loop starts at step k0-7, whose P3, P4 are those planes
  s2_fetch<T, TL, PROL, UM>(la, a, b, k0 - 4, vo4, vo2, vo1, coff, fu);
  s2_fetch<T, TL, PROL, UM>(lb, a, b, k0 - 3, vo4, vo2, vo1, coff, fu);
  s2_take<T, PROL, UM>(P3, la, fu);
  s2_take<T, PROL, UM>(P4, lb, fu);
  if constexpr (C::NSET == 2)
    s2_fetch<T, TL, PROL, UM>(la, a, b, k0 - 2, vo4, vo2, vo1, coff, fu);
  // step k0-8's exchange (S, Ly, Lx of plane k0-4 = P3) so that step k0-7
  // can complete P3's high faces
  {
    const int q = (k0 - 8) & 1;
    if (col) {
      sm.s[q][R][cs] = P3.s[0];
      sm.s[q][R][cs + 1] = P3.s[1];
      if constexpr (UM != S2_CONST) {
        sm.ly[q][R][cs] = P3.ly[0];
        sm.ly[q][R][cs + 1] = P3.ly[1];
        sm.lx0[q][R][c] = P3.lx[0];
      }
      sm.r1[q][R][c] = sm.b1[q][R][c] = sm.r2[q][R][c] = T(0);
    }
  }
  __syncthreads();

  auto step = [&](int k, S2Load<T>& cur, S2Load<T>& nxt) {
    const int q = (k - 1) & 1, w = k & 1;
    // issue the loads of plane k+6 into `nxt` (k+5 is in flight in `cur`),
    // or with one load set those of plane k+5 into `cur`; beyond the chunk's
    // last needed plane (k1+3) they are loaded but never used
    if constexpr (C::NSET == 2)
      s2_fetch<T, TL, PROL, UM>(nxt, a, b, k + 6, vo4, vo2, vo1, coff, fu);
    else
      s2_fetch<T, TL, PROL, UM>(cur, a, b, k + 5, vo4, vo2, vo1, coff, fu);
    // complete plane k+3: high faces from the previous step's exchange
    // (S2_CONST: they are already the tile's)
    if constexpr (UM != S2_CONST) {
      P3.lxh = sm.lx0[q][R][ce];
      P3.lyh[0] = sm.ly[q][RN][cs];
      P3.lyh[1] = sm.ly[q][RN][cs + 1];
    }
    if constexpr (RES) {
      // plane k+3 is complete: the residual of S on both cells of the pair
      // (own cells of the tile on the chunk's own planes), from the values
      // stage 1 reads
      if (out_ok && k + 3 >= k0 && k + 3 < k1) {
        bool a0, a1;
        const T q0 = s2_residual<T>(P3.s[0], P3.s[1], sm.s[q][R][cs - 1], sm.s[q][RN][cs],
                                    sm.s[q][RS][cs], P4.s[0], P2.s[0], P3.lx[0], P3.lx[1],
                                    P3.ly[0], P3.lyh[0], P3.lz[0], P4.lz[0], P3.sg[0], a0);
        const T q1 = s2_residual<T>(P3.s[1], sm.s[q][R][cs + 2], P3.s[0], sm.s[q][RN][cs + 1],
                                    sm.s[q][RS][cs + 1], P4.s[1], P2.s[1], P3.lx[1], P3.lxh,
                                    P3.ly[1], P3.lyh[1], P3.lz[1], P4.lz[1], P3.sg[1], a1);
        if (a0) racc += (double)q0 * (double)q0;
        if (a1) racc += (double)q1 * (double)q1;
      }
    }
    T r1n = T(0), b1n = T(0), r2n = T(0);
    // The four stages of step k all update element e = 1 - (par + k) mod 2
    // of their pairs: the red one on planes k+3 and k+1, the black one on
    // k+2 and k.  Each stage takes it as `ec`: with SPLIT a compile-time
    // constant, entered through a wave-uniform branch per stage.
    auto run = [&](auto&& stage) {
      if constexpr (C::SPLIT) {
        if ((par + k) & 1)
          stage(std::integral_constant<int, 0>{});
        else
          stage(std::integral_constant<int, 1>{});
      } else {
        stage(((par + k) & 1) ^ 1);
      }
    };
    // stage 1: sweep-1 red on plane k+3 from S
    if (k + 3 >= k0 - 3 && k + 3 < k1 + 3) {
      run([&](auto ec) {
        const int e = ec;
        if (e ? in3[1] : in3[0]) {  // whole waves outside the ring skip the update
          const T xe = e == 0 ? P3.s[1] : sm.s[q][R][cs + 2];
          const T xw = e == 0 ? sm.s[q][R][cs - 1] : P3.s[0];
          r1n = relax_cell<T>(pick(P3.s, e), xe, xw, sm.s[q][RN][cs + e],
                              sm.s[q][RS][cs + e], pick(P4.s, e), pick(P2.s, e),
                              pick(P3.lx, e), e == 0 ? P3.lx[1] : P3.lxh, pick(P3.ly, e),
                              pick(P3.lyh, e), pick(P3.lz, e), pick(P4.lz, e), pick(P3.sg, e),
                              omega);
        }
      });
    }
    // stage 2: sweep-1 black on plane k+2 from the sweep-1 red values
    if (k + 2 >= k0 - 2 && k + 2 < k1 + 2) {
      run([&](auto ec) {
        const int e = ec;
        if (e ? in2[1] : in2[0]) {
          const T xe = e == 0 ? r1b : sm.r1[q][R][ce];
          const T xw = e == 0 ? sm.r1[q][R][cw] : r1b;
          b1n = relax_cell<T>(pick(P2.s, e), xe, xw, sm.r1[q][RN][c], sm.r1[q][RS][c], r1n, r1a,
                              pick(P2.lx, e), e == 0 ? P2.lx[1] : P2.lxh, pick(P2.ly, e),
                              pick(P2.lyh, e), pick(P2.lz, e), pick(P3.lz, e), pick(P2.sg, e),
                              omega);
        }
      });
    }
    // stage 3: sweep-2 red on plane k+1 from the sweep-1 values
    if (k + 1 >= k0 - 1 && k + 1 < k1 + 1) {
      run([&](auto ec) {
        const int e = ec;
        if (e ? in1[1] : in1[0]) {
          const T xe = e == 0 ? b1b : sm.b1[q][R][ce];
          const T xw = e == 0 ? sm.b1[q][R][cw] : b1b;
          r2n = relax_cell<T>(r1a, xe, xw, sm.b1[q][RN][c], sm.b1[q][RS][c], b1n, b1a,
                              pick(P1.lx, e), e == 0 ? P1.lx[1] : P1.lxh, pick(P1.ly, e),
                              pick(P1.lyh, e), pick(P1.lz, e), pick(P2.lz, e), pick(P1.sg, e),
                              omega);
        }
      });
    }
    // stage 4: sweep-2 black on plane k; store plane k of W
    if (k >= k0 && k < k1) {
      run([&](auto ec) {
        const int e = ec;
        if (!out_ok) return;
        const T xe = e == 0 ? r2b : sm.r2[q][R][ce];
        const T xw = e == 0 ? sm.r2[q][R][cw] : r2b;
        const T b2 = relax_cell<T>(b1a, xe, xw, sm.r2[q][RN][c], sm.r2[q][RS][c], r2n, r2a,
                                   pick(P0.lx, e), e == 0 ? P0.lx[1] : P0.lxh, pick(P0.ly, e),
                                   pick(P0.lyh, e), pick(P0.lz, e), pick(P1.lz, e),
                                   pick(P0.sg, e), omega);
        const long long idx = (long long)k * g.sz + (long long)y * g.sy + xa;
        const T o0 = e == 0 ? b2 : r2b, o1 = e == 0 ? r2b : b2;
        if constexpr (sizeof(T) == 4)
          *reinterpret_cast<float2*>(W + idx) = make_float2(o0, o1);
        else
          *reinterpret_cast<double2*>(W + idx) = make_double2(o0, o1);
      });
    }
    // the next plane into the column registers, then exchange for step k+1
    P0 = P1;
    P1 = P2;
    P2 = P3;
    P3 = P4;
    s2_take<T, PROL, UM>(P4, cur, fu);  // plane k+5
    r1a = r1b;
    r1b = r1n;
    b1a = b1b;
    b1b = b1n;
    r2a = r2b;
    r2b = r2n;
    if (col) {
      sm.s[w][R][cs] = P3.s[0];  // plane k+4
      sm.s[w][R][cs + 1] = P3.s[1];
      if constexpr (UM != S2_CONST) {
        sm.ly[w][R][cs] = P3.ly[0];
        sm.ly[w][R][cs + 1] = P3.ly[1];
        sm.lx0[w][R][c] = P3.lx[0];
      }
      sm.r1[w][R][c] = r1b;  // plane k+3
      sm.b1[w][R][c] = b1b;  // plane k+2
      sm.r2[w][R][c] = r2b;  // plane k+1
    }
    __syncthreads();
  };
  int k = k0 - 7;
  if constexpr (C::NSET == 2) {
    for (; k + 1 < k1; k += 2) {
      step(k, la, lb);
      step(k + 1, lb, la);
    }
    if (k < k1) step(k, la, lb);
  } else {
    // five steps per iteration: the five plane registers then rotate by
    // renaming instead of by moves (with FP32 faces; with BF16 faces the
    // unrolled loop needs more than 128 VGPRs and spills, the plain loop
    // fewer than 100)
    for (; sizeof(TL) == 4 && k + 4 < k1; k += 5) {
      step(k, la, la);
      step(k + 1, la, la);
      step(k + 2, la, la);
      step(k + 3, la, la);
      step(k + 4, la, la);
    }
    for (; k < k1; ++k) step(k, la, la);
  }
  if constexpr (RES) return block_sum(racc, threadIdx.x, C::NTB);
  return 0.0;
}

// Whether every face the tile with origin (i0, j0) and z-planes [k0, k1)
// reads (the low faces of the in-domain cells of its grown region: columns
// i0 - 4 .. i0 + 67, rows j0 - 4 .. j0 + TY + 3, planes k0 - 4 .. k1 + 3,
// wrapped where periodic) lies in uniform bricks with the constants of the
// brick of the tile's origin; then u holds them.  The region spans at most
// two bricks in x, those of its first and last columns (or of i0 where the
// first is outside a wall); the workgroup checks the bricks of those columns
// on every row and plane of the region, a few independent loads per thread.
// Called by the whole workgroup.
// act: whether every cell of those bricks is also active.
template <int TY>
__device__ bool s2_uniform_tile(const Geom& g, const UBrick* __restrict__ ub, int ubx, int uby,
                                int i0, int j0, int k0, int k1, double (&u)[3], bool& act) {
  act = false;
  if (ub == nullptr) return false;  // uniform over the workgroup
  const UBrick* ref = ub + ((long long)(k0 / kUBZ) * uby + j0 / BY) * ubx + i0 / BX;
  u[0] = ref->u[0];
  u[1] = ref->u[1];
  u[2] = ref->u[2];
  bool ok = ref->ok != 0;
  bool all = ref->act != 0;
  const int nys = TY + 8, nzs = k1 - k0 + 8, nslot = 3 * nys * nzs;
#pragma unroll 4
  for (int q = threadIdx.x; q < nslot; q += blockDim.x) {
    const int xs = q % 3, ys = (q / 3) % nys, zs = q / (3 * nys);
    const int ii = wrap_coord(xs == 0 ? i0 - 4 : (xs == 1 ? i0 : i0 + S2_TX + 3), g.nx, g.px);
    const int jj = wrap_coord(j0 - 4 + ys, g.ny, g.py);
    const int mw = wrap_coord(k0 - 4 + zs, g.nz, g.pz);
    const bool in = ii >= 0 && jj >= 0 && mw >= 0;  // outside a wall: no faces
    const UBrick& b = in ? ub[((long long)(mw / kUBZ) * uby + jj / BY) * ubx + ii / BX] : *ref;
    ok &= b.ok != 0 && __double_as_longlong(b.u[0]) == __double_as_longlong(u[0]) &&
          __double_as_longlong(b.u[1]) == __double_as_longlong(u[1]) &&
          __double_as_longlong(b.u[2]) == __double_as_longlong(u[2]);
    all &= b.act != 0;
  }
  act = __syncthreads_and(all ? 1 : 0) != 0;
  return __syncthreads_and(ok ? 1 : 0) != 0;
}

// Whether every plane the tile over [k0, k1) fetches and uses (k0 - 4 ..
// k1 + 3) lies inside the domain and off the low z-wall's plane 0, so that
// a uniform tile's faces are the same on all of them (S2_CONST).
__device__ __forceinline__ bool s2_const_planes(const Geom& g, int k0, int k1) {
  return g.pz || (k0 - 4 >= 1 && k1 + 3 < g.nz);
}

// A tile's face mode for one tiling, found once per set of faces and tiling
// (k_pass_modes) so that the pass reads it instead of checking the bricks.
struct S2TileMode {
  double u[3];  // the bricks' constants (uniform tiles)
  int flags;    // S2M_UNIFORM, S2M_PLANES (s2_const_planes), S2M_ACTIVE
  int pad;
};
constexpr int S2M_UNIFORM = 1, S2M_PLANES = 2, S2M_ACTIVE = 4;

// The face mode of a pass tile: from the table tm when given, else by
// checking the bricks of the map ub (or none: S2_LOADED).  Called by the
// whole workgroup.
template <int TY, bool PROL>
__device__ __forceinline__ int s2_tile_mode(const Geom& g, const S2TileMode* __restrict__ tm,
                                            const UBrick* __restrict__ ub, int ubx, int uby,
                                            int t, int i0, int j0, int k0, int k1,
                                            double (&u)[3]) {
  int f;
  if (tm != nullptr) {
    const S2TileMode m = tm[t];
    u[0] = m.u[0];
    u[1] = m.u[1];
    u[2] = m.u[2];
    f = m.flags;
  } else {
    bool act;
    const bool uni = s2_uniform_tile<TY>(g, ub, ubx, uby, i0, j0, k0, k1, u, act);
    f = (uni ? S2M_UNIFORM : 0) | (s2_const_planes(g, k0, k1) ? S2M_PLANES : 0) |
        (act ? S2M_ACTIVE : 0);
  }
  if (!(f & S2M_UNIFORM)) return S2_LOADED;
  return ((f & S2M_PLANES) && ((f & S2M_ACTIVE) || !PROL)) ? S2_CONST : S2_UNIFORM;
}

}  // namespace gmg

// Two sweeps in one pass: X[rd] = sweep(sweep(X[rs] (+ P x_c))), at global
// scope so that its symbol carries no namespace.
template <typename T, typename TL, int TY, bool PROL>
__global__ __launch_bounds__(gmg::S2Cfg<TY>::NTB) void k_rb_sweep2(
    gmg::Geom g, gmg::Roles<T> X, int rs, int rd, const T* __restrict__ sigma,
    const TL* __restrict__ L, const T* __restrict__ xc, const uint8_t* __restrict__ active,
    gmg::Geom gc, int cx, int cy, int cz, int kchunk, const double* omega_p, const int* done,
    const gmg::UBrick* ub, int ubx, int uby, const gmg::S2TileMode* tm) {
  if (gmg::stopped(done)) return;
  __shared__ gmg::S2Smem<T, TY> sm;
  gmg::S2Args<T, TL> a{g, X.get(rs), sigma, L, xc, active, gc, cx, cy, cz};
  const int ntx = (g.nx + gmg::S2_TX - 1) / gmg::S2_TX, nty = (g.ny + TY - 1) / TY;
  const int t = gmg::xcd_tile(blockIdx.x, gridDim.x);
  const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
  const int i0 = tx * gmg::S2_TX, j0 = ty * TY, k0 = tz * kchunk, k1 = min(g.nz, k0 + kchunk);
  const T omega = (T)(*omega_p);
  double u[3];
  const int mode = gmg::s2_tile_mode<TY, PROL>(g, tm, ub, ubx, uby, t, i0, j0, k0, k1, u);
  if (mode == gmg::S2_LOADED)
    gmg::rb_sweep2_tile<T, TL, TY, PROL>(sm, a, X.get(rd), i0, j0, k0, k1, omega);
  else if (mode == gmg::S2_CONST)
    gmg::rb_sweep2_tile<T, TL, TY, PROL, false, gmg::S2_CONST>(sm, a, X.get(rd), i0, j0, k0, k1,
                                                               omega, u);
  else
    gmg::rb_sweep2_tile<T, TL, TY, PROL, false, gmg::S2_UNIFORM>(sm, a, X.get(rd), i0, j0, k0,
                                                                 k1, omega, u);
}

// The first pass of a cycle under the deferred decision: the same pass
// without correction, which also leaves one FP64 partial of ||sigma - A S||^2
// (its input's residual over the active cells) per workgroup, in dispatch
// order, in res_part; with a gate it runs only when *gate != 0.
template <typename T, typename TL, int TY>
__global__ __launch_bounds__(gmg::S2Cfg<TY>::NTB) void k_rb_sweep2_res(
    gmg::Geom g, gmg::Roles<T> X, int rs, int rd, const T* __restrict__ sigma,
    const TL* __restrict__ L, const uint8_t* __restrict__ active, int kchunk,
    const double* omega_p, const int* done, double* res_part, const int* gate,
    const gmg::UBrick* ub, int ubx, int uby, const gmg::S2TileMode* tm) {
  if (gmg::stopped(done)) return;
  if (gate != nullptr && *gate == 0) return;
  __shared__ gmg::S2Smem<T, TY> sm;
  gmg::S2Args<T, TL> a{g, X.get(rs), sigma, L, X.get(rs), active, g, 1, 1, 1, 0};
  const int ntx = (g.nx + gmg::S2_TX - 1) / gmg::S2_TX, nty = (g.ny + TY - 1) / TY;
  const int t = gmg::xcd_tile(blockIdx.x, gridDim.x);
  const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
  const int i0 = tx * gmg::S2_TX, j0 = ty * TY, k0 = tz * kchunk, k1 = min(g.nz, k0 + kchunk);
  const T omega = (T)(*omega_p);
  double u[3];
  double s;
  const int mode = gmg::s2_tile_mode<TY, false>(g, tm, ub, ubx, uby, t, i0, j0, k0, k1, u);
  if (mode == gmg::S2_LOADED)
    s = gmg::rb_sweep2_tile<T, TL, TY, false, true>(sm, a, X.get(rd), i0, j0, k0, k1, omega);
  else if (mode == gmg::S2_CONST)
    s = gmg::rb_sweep2_tile<T, TL, TY, false, true, gmg::S2_CONST>(sm, a, X.get(rd), i0, j0, k0,
                                                                   k1, omega, u);
  else
    s = gmg::rb_sweep2_tile<T, TL, TY, false, true, gmg::S2_UNIFORM>(sm, a, X.get(rd), i0, j0,
                                                                     k0, k1, omega, u);
  if (res_part != nullptr && threadIdx.x == 0) res_part[blockIdx.x] = s;
}

// The face modes of the tiles of a pass over level g with tiles of 64 x TY
// columns and z-chunks of kchunk planes, one workgroup per tile (indexed as
// the pass indexes them after xcd_tile).
template <int TY>
__global__ __launch_bounds__(gmg::S2Cfg<TY>::NTB) void k_pass_modes(
    gmg::Geom g, const gmg::UBrick* __restrict__ ub, int ubx, int uby, int kchunk,
    gmg::S2TileMode* __restrict__ tm) {
  const int ntx = (g.nx + gmg::S2_TX - 1) / gmg::S2_TX, nty = (g.ny + TY - 1) / TY;
  const int t = blockIdx.x;
  const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
  const int i0 = tx * gmg::S2_TX, j0 = ty * TY, k0 = tz * kchunk, k1 = min(g.nz, k0 + kchunk);
  double u[3];
  bool act;
  const bool uni = gmg::s2_uniform_tile<TY>(g, ub, ubx, uby, i0, j0, k0, k1, u, act);
  if (threadIdx.x == 0) {
    gmg::S2TileMode& m = tm[t];
    m.u[0] = u[0];
    m.u[1] = u[1];
    m.u[2] = u[2];
    m.flags = (uni ? gmg::S2M_UNIFORM : 0) | (gmg::s2_const_planes(g, k0, k1) ? gmg::S2M_PLANES : 0) |
              (act ? gmg::S2M_ACTIVE : 0);
    m.pad = 0;
  }
}
