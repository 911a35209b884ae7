// libgmg.so: geometric-multigrid Poisson solver for MI355X (gfx950).
//
// The C ABI is declared (with the contract of every entry point) in
// include/gmg.h.  This file holds the kernels of the V-cycle, the level
// hierarchy, and the host orchestration of residual, smoothing, transfers,
// V-cycle and the adaptive solve.
//
// Method (the paper, Sec. 3): GMG with red-black Gauss-Seidel smoothing whose
// relaxation factor adapts after every V-cycle (Sec. 3.1), and anisotropic
// coarsening that halves each direction independently (Sec. 3.2).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "gmg_kernels.h"
#include "gmg_sweep.h"
#include "gmg_sweep2.h"
#include "gmg_tail.h"
#include "gmg_walk.h"

using namespace gmg;

// ---------------------------------------------------------------------------
// Error plumbing
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

static gmg_status fail(gmg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? GMG_ENOMEM : GMG_EHIP,                   \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

#define GMG_TRY(expr)             \
  do {                            \
    gmg_status s_ = (expr);       \
    if (s_ != GMG_OK) return s_;  \
  } while (0)

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Walk column (i, j) of x over the z-planes [k0, k1), calling f(idx, ax, D)
// per cell (gmg_walk.h).
template <typename T, typename TL, typename F>
__device__ __forceinline__ void walk_column(const Geom& g, const T* __restrict__ x,
                                            const TL* __restrict__ L, int i, int j, int k0, int k1,
                                            F&& f) {
  walk_column_v<T, TL>(g, [&](long long q) { return x[q]; }, L, i, j, k0, k1,
                       [&](long long idx, T ax, T D, T) { f(idx, ax, D); });
}

// The same with sigma loaded alongside each plane: f(idx, ax, D, sigma(idx)).
template <typename T, typename TL, typename F>
__device__ __forceinline__ void walk_column_s(const Geom& g, const T* __restrict__ x,
                                              const T* __restrict__ sigma,
                                              const TL* __restrict__ L, int i, int j, int k0,
                                              int k1, F&& f) {
  walk_column_vs<T, TL>(g, [&](long long q) { return x[q]; },
                        [&](long long q) { return sigma[q]; }, L, i, j, k0, k1,
                        [&](long long idx, T ax, T D, T, T sv) { f(idx, ax, D, sv); });
}

// r = sigma - A x on active cells (0 elsewhere) for column (i, j) over the
// z-planes [k0, k1); optional store of r; returns the column's sum of r^2.
// Faces through face(d, q, hi) (walk_column_vsf, PF planes of loads in
// flight).
template <typename T, int PF = 2, typename FL>
__device__ __forceinline__ double residual_column_f(const Geom& g, const T* __restrict__ x,
                                                    const T* __restrict__ sigma, FL&& face,
                                                    T* __restrict__ r, int i, int j, int k0,
                                                    int k1) {
  double acc = 0.0;
  walk_column_vsf<T, PF>(
      g, [&](long long q) { return x[q]; }, [&](long long q) { return sigma[q]; }, face, i, j,
      k0, k1, [&](long long idx, T ax, T D, T, T sv) {
        const T rv = (D != T(0)) ? sv - ax : T(0);
        if (r) r[idx] = rv;
        acc += (double)rv * (double)rv;
      });
  return acc;
}

template <typename T, typename TL>
__device__ __forceinline__ double residual_column(const Geom& g, const T* __restrict__ x,
                                                  const T* __restrict__ sigma,
                                                  const TL* __restrict__ L, T* __restrict__ r,
                                                  int i, int j, int k0, int k1) {
  return residual_column_f<T>(
      g, x, sigma, [&](int d, long long q, bool) { return ldL<T>(L + d * g.n, q); }, r, i, j, k0,
      k1);
}

__device__ __forceinline__ bool same_bits(double a, double b) {
  return __double_as_longlong(a) == __double_as_longlong(b);
}

// Whether the block of BX x BY columns (bx, by) over planes [k0, k1) lies in
// uniform bricks of one set of constants (then u holds them).  Every thread
// of the block reads the same entries.
__device__ __forceinline__ bool uniform_block(const UBrick* ub, int ubx, int uby, int bx, int by,
                                              int k0, int k1, double (&u)[3]) {
  if (ub == nullptr || k0 >= k1) return false;
  const UBrick* b = ub + ((long long)(k0 / kUBZ) * uby + by) * ubx + bx;
  if (!b->ok) return false;
  u[0] = b->u[0];
  u[1] = b->u[1];
  u[2] = b->u[2];
  for (int z = k0 / kUBZ + 1; z <= (k1 - 1) / kUBZ; ++z) {
    const UBrick* c = ub + ((long long)z * uby + by) * ubx + bx;
    if (!c->ok || !same_bits(c->u[0], u[0]) || !same_bits(c->u[1], u[1]) ||
        !same_bits(c->u[2], u[2]))
      return false;
  }
  return true;
}

// The faces of a uniform block for the column (i, j) walked from plane k0:
// u_d, or +0 for the low face of a cell on a low wall (the walk asks for a
// z low face only at its first plane).
template <typename T>
struct UniformFaces {
  T u[3];
  bool wx, wy, wz;
  __device__ UniformFaces(const Geom& g, const double* c, int i, int j, int k0)
      : u{T(c[0]), T(c[1]), T(c[2])},
        wx(i == 0 && !g.px),
        wy(j == 0 && !g.py),
        wz(k0 == 0 && !g.pz) {}
  __device__ __forceinline__ T operator()(int d, long long, bool hi) const {
    const bool wall = !hi && (d == 0 ? wx : (d == 1 ? wy : wz));
    return wall ? T(0) : u[d];
  }
};

// The brick map of a level (see UBrick): the constants are the faces of the
// brick's cell (1, 1, 1), which is on no wall.
template <typename TL>
__global__ __launch_bounds__(BT) void k_uniform_bricks(Geom g, const TL* __restrict__ L,
                                                       const uint8_t* __restrict__ active,
                                                       UBrick* __restrict__ out) {
  const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
  const int i0 = bx * BX, j0 = by * BY, k0 = bz * kUBZ;
  const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
  const bool whole = i0 + BX <= g.nx && j0 + BY <= g.ny && k0 + kUBZ <= g.nz;
  double u[3] = {0.0, 0.0, 0.0};
  bool ok = whole;
  if (whole) {
    const long long c1 = (long long)(k0 + 1) * g.sz + (long long)(j0 + 1) * g.sy + i0 + 1;
    for (int d = 0; d < 3; ++d) u[d] = ldL<double>(L + d * g.n, c1);
    const TL* Lx = L;
    const TL* Ly = L + g.n;
    const TL* Lz = L + 2 * g.n;
    for (int k = k0; k < k0 + kUBZ; ++k) {
      const long long row = (long long)k * g.sz + (long long)j * g.sy;
      const long long c = row + i;
      // low faces
      ok = ok && same_bits(ldL<double>(Lx, c), (i == 0 && !g.px) ? 0.0 : u[0]);
      ok = ok && same_bits(ldL<double>(Ly, c), (j == 0 && !g.py) ? 0.0 : u[1]);
      ok = ok && same_bits(ldL<double>(Lz, c), (k == 0 && !g.pz) ? 0.0 : u[2]);
      // high faces beyond the brick: the next brick's low face or the
      // periodic wrap's (never a wall face)
      if (threadIdx.x == BX - 1 && (i + 1 < g.nx || g.px))
        ok = ok && same_bits(ldL<double>(Lx, row + (i + 1 < g.nx ? i + 1 : 0)), u[0]);
      if (threadIdx.y == BY - 1 && (j + 1 < g.ny || g.py))
        ok = ok && same_bits(ldL<double>(Ly, (long long)k * g.sz +
                                                 (long long)(j + 1 < g.ny ? j + 1 : 0) * g.sy + i),
                             u[1]);
      if (k == k0 + kUBZ - 1 && (k + 1 < g.nz || g.pz))
        ok = ok && same_bits(ldL<double>(Lz, (long long)(k + 1 < g.nz ? k + 1 : 0) * g.sz +
                                                 (long long)j * g.sy + i),
                             u[2]);
    }
  }
  bool act = whole;  // the active mask of the level, already built
  if (whole)
    for (int k = k0; k < k0 + kUBZ; ++k)
      act = act && active[(long long)k * g.sz + (long long)j * g.sy + i] != 0;
  ok = __syncthreads_and(ok ? 1 : 0) != 0;
  act = __syncthreads_and(act ? 1 : 0) != 0;
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    UBrick& b = out[((long long)bz * gridDim.y + by) * gridDim.x + bx];
    b.u[0] = u[0];
    b.u[1] = u[1];
    b.u[2] = u[2];
    b.ok = ok ? 1 : 0;
    b.act = act ? 1 : 0;
  }
}

// Order of the z-blocks of a level-0 pass over x, sigma and L that follows a
// two-sweep pass.  That pass marches each of its z-chunks upwards, so when it
// ends the upper part of every chunk is what it touched last and is the most
// likely to be still in the 256 MB Infinity Cache.  With `per` z-blocks of
// this kernel per chunk of the pass (per > 1, dividing the z-block count),
// dispatch index b is mapped so that the top z-block of every chunk goes
// first, then the one below, and so on; per = 1 keeps the natural order.  A
// bijection on [0, nzb): results do not depend on it.
__device__ __forceinline__ int chunk_top_first(int b, int nzb, int per) {
  if (per <= 1 || nzb % per != 0) return b;
  const int ng = nzb / per;  // chunks of the pass
  return (b % ng) * per + (per - 1 - b / ng);
}

// Logical (x, y, z) block of a 3-D grid from the hardware block, with the
// linear block index mapped by xcd_tile: each XCD then runs a contiguous
// range of blocks (whole rows of blocks, whole z-chunks), so the neighbour
// rows and planes a column walk reads beyond its own block are mostly in the
// same L2.  The residual norm at 256^3 takes 32.5 us so against 40.3 us in
// the hardware order, the fused residual + restriction with four coarse
// planes per block 39.9 against 41.8 us; with two coarse planes per block it
// took longer (49.4 against 46.1 us) and keeps the hardware order.
__device__ __forceinline__ int3 xcd_block() {
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const int t = xcd_tile(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
  return make_int3(t % gridDim.x, (t / gridDim.x) % gridDim.y, t / (gridDim.x * gridDim.y));
}

// Planes of loads in flight in the residual norm's walk over a block of
// uniform faces: with the face loads gone a wave's plane is 24 B per lane
// (FP32), so two planes in flight leave the walk bound by memory latency.
template <typename T>
constexpr int kResPF = sizeof(T) == 4 ? 3 : 2;

// r = sigma - A x over a chunk of z-planes; one FP64 partial of r^2 per block
// (stored by the block's z-chunk, whatever the dispatch order).
template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_residual(Geom g, Roles<T> X, int role,
                                                 const T* __restrict__ sigma,
                                                 const TL* __restrict__ L, T* r,
                                                 double* partials, int kchunk, const int* done,
                                                 int zper, const UBrick* ub, int ubx, int uby) {
  if (stopped(done)) return;
  const int3 b = xcd_block();
  const int zb = chunk_top_first(b.z, gridDim.z, zper);
  const int k0 = zb * kchunk, k1 = min(g.nz, k0 + kchunk);
  const int i = b.x * BX + threadIdx.x, j = b.y * BY + threadIdx.y;
  double u[3];
  const double acc =
      uniform_block(ub, ubx, uby, b.x, b.y, k0, k1, u)
          ? residual_column_f<T, kResPF<T>>(g, X.get(role), sigma, UniformFaces<T>(g, u, i, j, k0),
                                            r, i, j, k0, k1)
          : residual_column<T, TL>(g, X.get(role), sigma, L, r, i, j, k0, k1);
  if (partials) {
    const int tid = threadIdx.x + BX * threadIdx.y;
    const double s = block_sum(acc, tid, BT);
    if (tid == 0) partials[((long long)zb * gridDim.y + b.y) * gridDim.x + b.x] = s;
  }
}

// Start of a solve, one pass over x0, sigma and L: per-block partials of
// ||sigma||^2 over the active cells (pa) and of ||sigma - A x0||^2 (pb), in
// the order of k_masked_sumsq and k_residual (active <=> D != 0, as in the
// mask), so both norms are bitwise those of the two separate kernels.
template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_start_norms(Geom g, const T* __restrict__ x,
                                                    const T* __restrict__ sigma,
                                                    const TL* __restrict__ L, double* pa,
                                                    double* pb, int kchunk) {
  const int k0 = blockIdx.z * kchunk;
  double as = 0.0, ar = 0.0;
  walk_column_s<T, TL>(g, x, sigma, L, blockIdx.x * BX + threadIdx.x,
                       blockIdx.y * BY + threadIdx.y, k0, min(g.nz, k0 + kchunk),
                       [&](long long, T ax, T D, T sv) {
                         const T rv = (D != T(0)) ? sv - ax : T(0);
                         if (D != T(0)) as += (double)sv * (double)sv;
                         ar += (double)rv * (double)rv;
                       });
  const int tid = threadIdx.x + BX * threadIdx.y;
  const long long blk = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const double ss = block_sum(as, tid, BT);
  __syncthreads();
  const double sr = block_sum(ar, tid, BT);
  if (tid == 0) {
    pa[blk] = ss;
    pb[blk] = sr;
  }
}

// Sum of v^2 over active cells (mask != 0), per-block partials, z-chunked.
template <typename T>
__global__ __launch_bounds__(BT) void k_masked_sumsq(Geom g, const T* __restrict__ v,
                                                     const uint8_t* __restrict__ mask,
                                                     double* partials, int kchunk) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
  double acc = 0.0;
  if (i < g.nx && j < g.ny) {
    for (int k = k0; k < k1; ++k) {
      const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
      if (mask[idx]) acc += (double)v[idx] * (double)v[idx];
    }
  }
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double s = block_sum(acc, tid, BT);
  if (tid == 0)
    partials[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// Fused residual + restriction, one thread per FINE cell of the BX x BY tile
// at (i0, j0): each thread sums the residuals of its column over the cz fine
// planes of each coarse plane of [K0, K1) (at most RC = 1, 2 or 4 of them,
// one walk up the column); x-pairs are combined by a lane shuffle and y-pairs through LDS
// (rows[r] for coarse plane K0 + r); the thread at each block's origin writes
// sigma_c and zeroes x_c.
template <typename T, typename TL, int RC = 1>
__device__ __forceinline__ void restrict_tile(T (*rows)[BY][BX], const Geom& gf,
                                              const T* __restrict__ x,
                                              const T* __restrict__ sigma,
                                              const TL* __restrict__ L, const Geom& gc, int cx,
                                              int cy, int cz, T* __restrict__ sigma_c,
                                              T* __restrict__ x_c, int i0, int j0, int K0, int K1,
                                              const double* uni = nullptr) {
  static_assert(RC == 1 || RC == 2 || RC == 4, "1, 2 or 4 coarse planes per tile");
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = i0 + tx, j = j0 + ty;
  const int k0 = K0 * cz, k1 = K1 * cz;
  T acc[RC];
#pragma unroll
  for (int r = 0; r < RC; ++r) acc[r] = T(0);
  int pl = 0;  // fine planes walked so far
  auto add = [&](long long, T ax, T D, T, T sv) {
    if constexpr (RC == 1) {
      if (D != T(0)) acc[0] += sv - ax;
    } else {
      if (D != T(0)) {
        const int c = cz == 2 ? pl >> 1 : pl;  // the plane's coarse plane in the tile
#pragma unroll
        for (int r = 0; r < RC; ++r)
          if (c == r) acc[r] += sv - ax;
      }
      ++pl;
    }
  };
  auto xv = [&](long long q) { return x[q]; };
  auto sv = [&](long long q) { return sigma[q]; };
  if (uni) {  // a uniform block: the constant faces, every plane's loads in flight at once
    const UniformFaces<T> uf(gf, uni, i, j, k0);
    if (RC == 4 && cz == 2)  // eight planes: a ring of three (no plane loaded twice)
      walk_column_vsf<T, 3>(gf, xv, sv, uf, i, j, k0, k1, add);
    else if (RC * cz >= 4)
      walk_column_vsf<T, 4, true>(gf, xv, sv, uf, i, j, k0, k1, add);
    else
      walk_column_vsf<T, 2, true>(gf, xv, sv, uf, i, j, k0, k1, add);
  } else {  // stored faces: the next plane's loads in flight (the registers of four
            // planes of faces would cost occupancy)
    walk_column_vsf<T>(
        gf, xv, sv, [&](int d, long long q, bool) { return ldL<T>(L + d * gf.n, q); }, i, j, k0,
        k1, add);
  }
#pragma unroll
  for (int r = 0; r < RC; ++r)
    if (cx == 2) acc[r] += __shfl_xor(acc[r], 1, 64);
  if (cy == 2) {
#pragma unroll
    for (int r = 0; r < RC; ++r) rows[r][ty][tx] = acc[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] += rows[r][ty ^ 1][tx];
  }
  if (i < gf.nx && j < gf.ny && (i % cx) == 0 && (j % cy) == 0) {
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      if (K0 + r >= K1) break;
      const long long cidx = (long long)(K0 + r) * gc.sz + (long long)(j / cy) * gc.sy + i / cx;
      sigma_c[cidx] = acc[r];
      if (x_c) x_c[cidx] = T(0);
    }
  }
}

// Coarse planes per workgroup of the fused residual + restriction: 4 (eight
// fine planes, three planes of loads in flight) or 2 (four fine planes, all
// loads in flight at once) where one plane per workgroup would need at least
// this many workgroups, else 1.  At 256^3: level 0 62 -> 45 (2) -> 42 us
// (4); level 1 11.5 -> 9.1 us (2); level 2 took 5.4 against 4.7 us with 2.
constexpr long long kRestrictPairBlocks = 4096;
constexpr long long kRestrictQuadBlocks = 16384;

template <typename T, typename TL, int RC>
__global__ __launch_bounds__(BT) void k_restrict_residual(
    Geom gf, Roles<T> X, int role, const T* __restrict__ sigma, const TL* __restrict__ L,
    Geom gc, int cx, int cy, int cz, T* __restrict__ sigma_c, T* __restrict__ x_c,
    const int* done, int zper, const UBrick* ub, int ubx, int uby) {
  if (stopped(done)) return;
  __shared__ T rows[RC][BY][BX];
  const int3 b = RC == 4 ? xcd_block() : make_int3(blockIdx.x, blockIdx.y, blockIdx.z);
  const int K0 = RC * chunk_top_first(b.z, gridDim.z, zper);
  const int K1 = min(gc.nz, K0 + RC);
  double u[3];
  const bool uni = uniform_block(ub, ubx, uby, b.x, b.y, K0 * cz, min(gf.nz, K1 * cz), u);
  restrict_tile<T, TL, RC>(rows, gf, X.get(role), sigma, L, gc, cx, cy, cz, sigma_c, x_c,
                           b.x * BX, b.y * BY, K0, K1, uni ? u : nullptr);
}

// Piecewise-constant prolongation + correction on active fine cells:
// X[rd] = X[rs] + P x_c (in place when rs == rd).
template <typename T>
__global__ __launch_bounds__(BT) void k_prolong(Geom gf, Roles<T> X, int rs, int rd,
                                                const uint8_t* __restrict__ active,
                                                const T* __restrict__ x_c, Geom gc, int cx,
                                                int cy, int cz, const int* done) {
  if (stopped(done)) return;
  const T* src = X.get(rs);
  T* dst = X.get(rd);
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= gf.nx || j >= gf.ny) return;
  const long long idx = (long long)k * gf.sz + (long long)j * gf.sy + i;
  T v = src[idx];
  if (active[idx]) v += x_c[(long long)(k / cz) * gc.sz + (long long)(j / cy) * gc.sy + i / cx];
  dst[idx] = v;
}

// Copy X[rs] -> X[rd].
template <typename T>
__global__ __launch_bounds__(BT) void k_copy_role(Geom g, Roles<T> X, int rs, int rd,
                                                  const int* done) {
  if (stopped(done)) return;
  const T* src = X.get(rs);
  T* dst = X.get(rd);
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const long long idx = (long long)blockIdx.z * g.sz + (long long)j * g.sy + i;
  dst[idx] = src[idx];
}

// Level-0 face copy from the caller's dtype into storage, zeroing the low
// face at index 0 of every wall direction.
template <typename TI, typename TL>
__global__ __launch_bounds__(BT) void k_copy_faces(Geom g, const TI* __restrict__ Lin,
                                                   TL* __restrict__ Lout, int* bad) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
  const int c[3] = {i, j, k};
  const int per[3] = {g.px, g.py, g.pz};
  for (int d = 0; d < 3; ++d) {
    double v = (double)Lin[d * g.n + idx];
    if (!per[d] && c[d] == 0) v = 0.0;
    if (!isfinite(v)) *bad = 1;  // the set-up then fails with GMG_EINVAL
    Lout[d * g.n + idx] = to_storage<TL>(v);
  }
}

// Coarse faces: L_d^c[J] = (1/c_d) * sum of the fine d-faces with offset 0
// along d and every offset along the other directions (the fine faces that
// tile the coarse cell's low d-face).  Accumulated in FP64, then stored.
template <typename TL>
__global__ __launch_bounds__(BT) void k_restrict_faces(Geom gf, const TL* __restrict__ Lf,
                                                       Geom gc, int cx, int cy, int cz,
                                                       TL* __restrict__ Lc) {
  const int I = blockIdx.x * BX + threadIdx.x;
  const int J = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= gc.nx || J >= gc.ny) return;
  const int c[3] = {cx, cy, cz};
  const long long cidx = (long long)K * gc.sz + (long long)J * gc.sy + I;
  for (int d = 0; d < 3; ++d) {
    const int ex = (d == 0) ? 1 : cx, ey = (d == 1) ? 1 : cy, ez = (d == 2) ? 1 : cz;
    double s = 0.0;
    for (int sz = 0; sz < ez; ++sz)
      for (int sy = 0; sy < ey; ++sy)
        for (int sx = 0; sx < ex; ++sx) {
          const long long f = (long long)(K * cz + sz) * gf.sz + (long long)(J * cy + sy) * gf.sy +
                              (I * cx + sx);
          s += ldL<double>(Lf + d * gf.n, f);
        }
    Lc[d * gc.n + cidx] = to_storage<TL>(s / (double)c[d]);
  }
}

// active[I] = (D(I) != 0), i.e. at least one of the six faces is nonzero.
template <typename TL>
__global__ __launch_bounds__(BT) void k_active(Geom g, const TL* __restrict__ L,
                                               uint8_t* __restrict__ active) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
  double D;
  // reuse the stencil on a zero field: only D is needed
  double s = 0.0;
  const int c[3] = {i, j, k};
  const int n[3] = {g.nx, g.ny, g.nz};
  const int per[3] = {g.px, g.py, g.pz};
  const long long st[3] = {1, g.sy, g.sz};
  for (int d = 0; d < 3; ++d) {
    const Nb nb = neighbours(c[d], n[d], per[d], st[d]);
    s += ldL<double>(L + d * g.n, idx);
    if (nb.hi_ok) s += ldL<double>(L + d * g.n, idx + nb.hi);
  }
  D = -s;
  active[idx] = (D != 0.0) ? 1 : 0;
}

// Deterministic sum of n partials (single block, fixed order).
__device__ double reduce_partials(const double* p, long long n) {
  const int tid = threadIdx.x;
  const long long st = blockDim.x;
  double s = 0.0;
  long long q = tid;
  // eight loads in flight per thread, added in index order as one at a time
  for (; q + 7 * st < n; q += 8 * st) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[q + u * st];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; q < n; q += st) s += p[q];
  return block_sum(s, tid, blockDim.x);
}

// Start of a solve: ||sigma|| (partials a) and ||r(x0)|| (partials b).  The
// tolerance is rtol, or *rtol_p when given (a refinement step's inner
// tolerance, set on the device).
__global__ __launch_bounds__(256) void k_solve_init(const double* pa, long long na,
                                                    const double* pb, long long nb,
                                                    SolveState* st, double rtol,
                                                    int max_cycles, double omega0,
                                                    const int* skip, const double* rtol_p) {
  if (skip != nullptr && *skip) return;
  if (rtol_p != nullptr) rtol = *rtol_p;
  const double ss = reduce_partials(pa, na);
  __syncthreads();
  const double rr = reduce_partials(pb, nb);
  if (threadIdx.x == 0) {
    st->snorm = sqrt(ss);
    st->rho = st->rho0 = st->last = sqrt(rr);
    const bool bad = !isfinite(st->snorm) || !isfinite(st->rho);
    st->omega = omega0;
    st->rtol = rtol;
    st->cur = 0;
    st->cycles = 0;
    st->accepted = 0;
    st->max_cycles = max_cycles;
    st->map[0] = st->map[1] = 0;  // the first pass reads x0 itself as its input
    st->map[2] = 1;
    st->map[3] = 2;
    st->pending = 0;
    st->redo = 0;
    st->omega_spec = omega0;
    const bool conv = !bad && ((st->snorm == 0.0) || (st->rho <= rtol * st->snorm));
    st->status = bad ? kStNonFinite : (conv ? 0 : 5);
    st->done = (bad || conv || max_cycles <= 0) ? 1 : 0;
  }
}

// A cycle's residual norm that is not finite stops the solve; the accepted
// iterate (role 0) is kept.  Returns true if it did.
__device__ __forceinline__ bool stop_non_finite(SolveState* st, double rn, int c) {
  if (isfinite(rn)) return false;
  if (c < GMG_MAX_HISTORY) st->acc[c] = 0;
  st->cycles = c + 1;
  st->status = kStNonFinite;
  st->done = 1;
  return true;
}

// End of a V-cycle: new residual norm, the adaptive-relaxation decision
// (Sec. 3.1) and the convergence flag.
__global__ __launch_bounds__(256) void k_cycle_finish(const double* p, long long n,
                                                      SolveState* st, OmegaRule rule,
                                                      int final_role) {
  if (st->done) return;
  const double rr = reduce_partials(p, n);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(rr);
  const int c = st->cycles;
  if (c < GMG_MAX_HISTORY) {
    st->hist[c] = (st->snorm > 0.0) ? rn / st->snorm : 0.0;
    st->omegas[c] = st->omega;
  }
  st->last = rn;
  if (stop_non_finite(st, rn, c)) return;
  // the cycle's result sits in role `final_role`; accepting it makes that
  // buffer the new role 0
  const int next = (st->cur + final_role) % 3;
  if (rn > st->rho) {  // growth: lower omega, and discard the cycle with rollback
    st->omega = fmax(rule.omega_min, rule.theta_dec * st->omega);
    if (c < GMG_MAX_HISTORY) st->acc[c] = rule.rollback ? 0 : 1;
    if (!rule.rollback) {
      st->cur = next;
      st->rho = rn;
    }
  } else {  // decay (or a tie): keep the cycle and raise omega
    st->cur = next;
    st->rho = rn;
    st->omega = fmin(rule.omega_max, rule.theta_inc * st->omega);
    st->accepted += 1;
    if (c < GMG_MAX_HISTORY) st->acc[c] = 1;
  }
  st->cycles = c + 1;
  const bool conv = st->rho <= st->rtol * st->snorm;
  if (conv) st->status = 0;
  if (conv || st->cycles >= st->max_cycles) st->done = 1;
}

// Deferred decision of gmg_solve, after the first sweep of a cycle has taken
// the norm of its input, the previous cycle's result (the candidate, role 1)
// and speculatively swept it with the omega that acceptance would give.
// Same rule as k_cycle_finish: growth lowers omega (and, with rollback,
// discards the candidate), decay accepts it (map roles 0 and 1 swap) and
// raises omega.  Whenever omega did not come out as assumed, `redo` asks for
// the first sweep again from the accepted iterate.  The first pass of a
// solve has no candidate: it only points role 1 at the fourth buffer.
__global__ __launch_bounds__(256) void k_spec_finish(const double* p, long long n, SolveState* st,
                                                     OmegaRule rule) {
  if (st->done) return;
  const double rr = reduce_partials(p, n);
  if (threadIdx.x != 0) return;
  if (!st->pending) {
    st->pending = 1;
    st->map[1] = 3;
    st->redo = 0;
    st->omega_spec = fmin(rule.omega_max, rule.theta_inc * st->omega);
    return;
  }
  const double rn = sqrt(rr);
  const int c = st->cycles;
  if (c < GMG_MAX_HISTORY) {
    st->hist[c] = (st->snorm > 0.0) ? rn / st->snorm : 0.0;
    st->omegas[c] = st->omega;
  }
  st->last = rn;
  if (stop_non_finite(st, rn, c)) return;
  if (rn > st->rho) {  // growth
    st->omega = fmax(rule.omega_min, rule.theta_dec * st->omega);
    if (c < GMG_MAX_HISTORY) st->acc[c] = rule.rollback ? 0 : 1;
    if (!rule.rollback) {
      const int a = st->map[0];
      st->map[0] = st->map[1];
      st->map[1] = a;
      st->rho = rn;
    }
    st->redo = 1;
  } else {  // decay (or a tie)
    const int a = st->map[0];
    st->map[0] = st->map[1];
    st->map[1] = a;
    st->rho = rn;
    st->omega = fmin(rule.omega_max, rule.theta_inc * st->omega);
    st->accepted += 1;
    if (c < GMG_MAX_HISTORY) st->acc[c] = 1;
    st->redo = (st->omega != st->omega_spec) ? 1 : 0;
  }
  st->cycles = c + 1;
  st->omega_spec = fmin(rule.omega_max, rule.theta_inc * st->omega);
  const bool conv = st->rho <= st->rtol * st->snorm;
  if (conv) st->status = 0;
  if (conv || st->cycles >= st->max_cycles) st->done = 1;
}

__global__ void k_set_omega(SolveState* st, double omega) { st->omega = omega; }

__global__ __launch_bounds__(256) void k_sum_to(const double* p, long long n, double* out) {
  const double s = reduce_partials(p, n);
  if (threadIdx.x == 0) *out = s;
}

// Number of active cells (per-block partials, z-chunked).
__global__ __launch_bounds__(BT) void k_count_mask(Geom g, const uint8_t* __restrict__ mask,
                                                   double* partials, int kchunk) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
  double acc = 0.0;
  if (i < g.nx && j < g.ny)
    for (int k = k0; k < k1; ++k) acc += mask[(long long)k * g.sz + (long long)j * g.sy + i];
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double s = block_sum(acc, tid, BT);
  if (tid == 0)
    partials[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// Start of a refinement solve: ||sigma|| and the active-cell count.
__global__ __launch_bounds__(256) void k_ir_init(const double* ps, const double* pc, long long n,
                                                 IRState* ir, SolveState* inner, double rtol,
                                                 int max_outer, double inner_base, double target) {
  const double ss = reduce_partials(ps, n);
  __syncthreads();
  const double cnt = reduce_partials(pc, n);
  if (threadIdx.x == 0) {
    ir->snorm = sqrt(ss);
    ir->n_active = (int)cnt;
    ir->rtol = rtol;
    ir->outer = 0;
    ir->inner_total = 0;
    ir->max_outer = max_outer;
    ir->inner_base = ir->inner_rtol = inner_base;
    ir->target = target;
    ir->done = isfinite(ir->snorm) ? 0 : 1;
    ir->status = isfinite(ir->snorm) ? 5 : kStNonFinite;
    inner->done = 1;
  }
}

// Outer-step check on the FP64 residual norm: converged, out of steps, or the
// scale beta = ||r|| / sqrt(#active) of the next correction problem.
__global__ __launch_bounds__(256) void k_ir_check(const double* p, long long n, IRState* ir) {
  if (ir->done) return;
  const double rr = reduce_partials(p, n);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(rr);
  ir->rnorm = rn;
  if (ir->outer < GMG_MAX_HISTORY) ir->hist[ir->outer] = (ir->snorm > 0.0) ? rn / ir->snorm : 0.0;
  if (!isfinite(rn)) {  // NaN or Inf in x0 (sigma and L were checked before)
    ir->status = kStNonFinite;
    ir->done = 1;
  } else if (ir->snorm == 0.0 || rn <= ir->rtol * ir->snorm) {
    ir->status = 0;
    ir->done = 1;
  } else if (ir->outer >= ir->max_outer) {
    ir->done = 1;
  } else {
    ir->beta = rn / sqrt((double)max(ir->n_active, 1));
    ir->inner_rtol = ir_inner_tolerance(ir, rn);
  }
}

// b = fp32(r / beta) and the inner initial guess e = 0; partials of b^2.
__global__ __launch_bounds__(BT) void k_scale_cast(Geom g, const double* __restrict__ r,
                                                   const IRState* ir, float* __restrict__ b,
                                                   float* __restrict__ e, double* partials,
                                                   int kchunk) {
  if (ir->done) return;
  const double inv = 1.0 / ir->beta;
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
  double acc = 0.0;
  if (i < g.nx && j < g.ny)
    for (int k = k0; k < k1; ++k) {
      const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
      const float v = (float)(r[idx] * inv);
      b[idx] = v;
      e[idx] = 0.0f;
      acc += (double)v * (double)v;
    }
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double s = block_sum(acc, tid, BT);
  if (tid == 0)
    partials[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// x += beta * e in FP64; block (0,0,0) also books the step.
__global__ __launch_bounds__(BT) void k_ir_update(Geom g, double* __restrict__ x, Roles<float> E,
                                                  IRState* ir, const SolveState* inner) {
  if (ir->done) return;
  const float* e = E.get(0);
  const double beta = ir->beta;
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i < g.nx && j < g.ny) {
    const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
    x[idx] += beta * (double)e[idx];
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0 &&
      threadIdx.y == 0) {
    if (ir->outer < GMG_MAX_HISTORY) ir->inner[ir->outer] = inner->cycles;
    ir->inner_total += inner->cycles;
    ir->outer += 1;
  }
}

#include "gmg_pcg.h"
#include "gmg_split.h"

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------

namespace {

constexpr int kMaxLevels = 32;
constexpr int kPairTYDefault = 16;  // tile rows of the two-sweep pass by default
constexpr int kTailMaxCells = 32768;
constexpr long long kTailGlobalCells = 1LL << 20;  // coarsest level run by the tail from global memory
constexpr int kResChunk = 16;  // z-planes per block in the norm reductions

struct Level {
  Geom g;
  int c[3];        // factor to the next level; 0 on the coarsest
  void* L;         // [3][nz][ny][nx] in l_storage
  uint8_t* active;
  void* x[2];      // cycle dtype ping-pong iterates (levels >= 1)
  void* sigma;
  int kchunk;      // z-planes per workgroup of the fused sweep
  int ty;          // tile height of the fused sweep (rows of 64 cells)
  int pair_kc;     // > 0: two consecutive sweeps run as one two-sweep pass
                   // with this z-chunk; 0: separate sweeps
  int pair_ty;     // tile rows of the two-sweep pass (8 or 16)
  UBrick* ub;      // uniform-brick map (NULL: off); ubx x uby x ubz bricks
  int ubx, uby, ubz;
  S2TileMode* tm;  // face modes of the two-sweep pass's tiles (NULL: none)
  int tm_ty, tm_kc;  // the tiling they were found for (tm_kc 0: none yet)
};

size_t dsize(int dt) { return dt == GMG_F64 ? 8 : (dt == GMG_BF16 ? 2 : 4); }

Geom make_geom(const int n[3], const int per[3]) {
  Geom g;
  g.nx = n[0];
  g.ny = n[1];
  g.nz = n[2];
  g.px = per[0];
  g.py = per[1];
  g.pz = per[2];
  g.sy = n[0];
  g.sz = (long long)n[0] * n[1];
  g.n = g.sz * n[2];
  return g;
}

dim3 cell_grid(const Geom& g) { return dim3((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz); }
dim3 red_grid(const Geom& g) {
  return dim3((g.nx + BX - 1) / BX, (g.ny + BY - 1) / BY, (g.nz + kResChunk - 1) / kResChunk);
}
long long nblocks(dim3 d) { return (long long)d.x * d.y * d.z; }

// Fused-sweep tile height per precision (LDS budget: six 3-plane rings).
template <typename T> struct SweepTY { static constexpr int v = 8; };
template <> struct SweepTY<double> { static constexpr int v = 4; };

// z-chunk of the fused sweep: split z so that the workgroups fill whole
// rounds of the resident slots (256 CUs x workgroups per CU that fit the
// LDS budget of 160 KB), which avoids a partly filled last round; at least
// 2 planes per chunk.
constexpr int kCUs = 256;
// A level can run two consecutive sweeps as one pass: FP32 cycles of the
// red-black smoother with at least one smoothing step of two sweeps, and an
// even nx (the pass works on x-pairs).
bool pair_capable(const gmg_params& p, const Geom& g) {
  return p.pair_sweeps && p.cycle_dtype == GMG_F32 && p.smoother == GMG_SMOOTH_RBGS &&
         g.nx % 2 == 0 && g.n <= S2_MAX_CELLS &&
         (p.nu_pre >= 2 || p.nu_post >= 2 || p.nu_coarse >= 2);
}

// z-chunk of the two-sweep pass: one workgroup per CU (its register
// footprint allows one), as many chunks as fill the 256 CUs `per_cu` times
// (2 where tiles of uniform faces run faster than the others, so that the
// CUs balance them), at least 2 planes per chunk.
int pair_kchunk(const Geom& g, int ty, int per_cu = 1) {
  const long long tiles = (long long)((g.nx + S2_TX - 1) / S2_TX) * ((g.ny + ty - 1) / ty);
  const long long chunks = std::max<long long>(1, per_cu * kCUs / std::max<long long>(1, tiles));
  const int kc = (int)((g.nz + chunks - 1) / chunks);
  return std::max(std::min(2, g.nz), kc);
}

int sweep_kchunk(const Geom& g, int ty, int elem_bytes) {
  const long long tiles = (long long)((g.nx + SW_TX - 1) / SW_TX) * ((g.ny + ty - 1) / ty);
  const size_t lds = (size_t)elem_bytes * SW_EX * 3 * ((ty + 4) + 3 * (ty + 2) + (ty + 3) + (ty + 2));
  const long long per_cu = std::max<long long>(1, (long long)(160 * 1024 / lds));
  const long long slots = kCUs * per_cu;
  const long long chunks = std::max<long long>(1, slots / std::max<long long>(1, tiles));
  int kc = (int)((g.nz + chunks - 1) / chunks);
  return std::max(std::min(2, g.nz), kc);
}

}  // namespace

// A captured kernel sequence keyed by the caller pointers baked into it.
struct CapturedSeq {
  hipGraphExec_t exec;
  const void* k0;
  const void* k1;
};

struct gmg_handle {
  gmg_params p;
  hipStream_t s;
  int nlev;
  Level lev[kMaxLevels];
  int tail;      // first level cycled by k_tail (nlev: none)
  int tail_global;  // 1: the tail is the coarsest level alone, in global memory
  void* L0x;     // exact FP64 level-0 faces (dtype F64 with F32 cycles)
  void* w[3];    // level-0 work iterates (cycle dtype); the caller's x is the fourth
  double* spec_part;  // first-sweep residual partials of the deferred decision
  double* partials;  // 2 * maxpart
  long long maxpart;
  SolveState* st;
  SolveState* hst;   // pinned host mirror
  OmegaRule rule;
  // iterative refinement (dtype F64 with F32 cycles)
  IRState* ir;
  IRState* hir;      // pinned host mirror
  double* r64;       // FP64 outer residual
  float* b32;        // scaled, rounded correction right-hand side
  float* e32;        // correction (role 0 of the inner solve)
  // captured launch sequences, replayed with hipGraphLaunch
  hipStream_t cap;   // capture stream (the caller's may be the legacy stream)
  CapturedSeq cyc;   // one V-cycle of gmg_solve
  CapturedSeq irs;   // one outer step of gmg_solve_ir
  int ir_inner;      // max_inner / inner_rtol recorded in irs
  double ir_inner_rtol;
  // conjugate gradient (gmg_pcg on level 0; the PCG smoother on every level):
  // r, z, two direction buffers, q = B p and s = diag(-A) per level, in the
  // cycle precision, allocated on first use; one PCGState per level
  void* pcg[kMaxLevels][6];
  PCGState* pst;
  PCGState* hpst;    // pinned host mirror of level 0's state
  CapturedSeq pcgit; // one iteration of gmg_pcg
};

static const dim3 kBlock(BX, BY, 1);

// ---------------------------------------------------------------------------
// Typed enqueue helpers
// ---------------------------------------------------------------------------

template <typename T>
static Roles<T> level_roles(gmg_handle* h, int l, T* x0, const int* sel) {
  Roles<T> R{};
  if (l == 0) {
    R.p[0] = x0;
    R.p[1] = (T*)h->w[0];
    R.p[2] = (T*)h->w[1];
    R.sel = sel;
  } else {
    R.p[0] = (T*)h->lev[l].x[0];
    R.p[1] = (T*)h->lev[l].x[1];
    R.p[2] = (T*)h->lev[l].x[0];  // unused
    R.sel = nullptr;
  }
  return R;
}

// next ping-pong role: level 0 cycles 0 -> 1 -> 2 -> 1 -> 2 ... so that the
// accepted iterate (role 0) is never written; coarse levels alternate 0 <-> 1
static int next_role(int l, int r) { return l == 0 ? (r == 1 ? 2 : 1) : 1 - r; }

// Optional parts of a sweep launch: the input-residual partials, the omega
// to use (default: the solve state's), and a gate flag.
struct SweepOpt {
  double* res_part = nullptr;
  const double* omega = nullptr;
  const int* gate = nullptr;
};

template <typename T, typename TL, int TY>
static void launch_sweep(gmg_handle* h, int l, const Roles<T>& X, int rs, int rd, const T* sigma,
                         const T* xc, const int* done, int kchunk, const SweepOpt& o = {}) {
  const Level& lv = h->lev[l];
  const Geom gc = (xc && l + 1 < h->nlev) ? h->lev[l + 1].g : lv.g;
  const dim3 grid(((lv.g.nx + SW_TX - 1) / SW_TX) * ((lv.g.ny + TY - 1) / TY) *
                  ((lv.g.nz + kchunk - 1) / kchunk));
  const int cx = lv.c[0] ? lv.c[0] : 1, cy = lv.c[1] ? lv.c[1] : 1, cz = lv.c[2] ? lv.c[2] : 1;
  if (lv.g.nx % 2 == 0)
    hipLaunchKernelGGL((k_rb_sweep<T, TL, TY, 2>), grid, dim3(32 * TY), 0, h->s, lv.g, X, rs, rd,
                       sigma, (const TL*)lv.L, xc, lv.active, gc, cx, cy, cz, kchunk,
                       o.omega ? o.omega : &h->st->omega, done, o.res_part, o.gate);
  else
    hipLaunchKernelGGL((k_rb_sweep<T, TL, TY, 1>), grid, dim3(32 * TY), 0, h->s, lv.g, X, rs, rd,
                       sigma, (const TL*)lv.L, xc, lv.active, gc, cx, cy, cz, kchunk,
                       o.omega ? o.omega : &h->st->omega, done, o.res_part, o.gate);
}

// Workgroups of a level's sweep launch (partials written with res_part).
static long long sweep_blocks(const Level& lv, int ty) {
  return (long long)((lv.g.nx + SW_TX - 1) / SW_TX) * ((lv.g.ny + ty - 1) / ty) *
         ((lv.g.nz + lv.kchunk - 1) / lv.kchunk);
}

// Red-black sweep of level l as a red and a black half-sweep launch.
template <typename T, typename TL>
static void launch_split(gmg_handle* h, int l, const Roles<T>& X, int rs, int rd, const T* sigma,
                         const T* xc, const int* done) {
  const Level& lv = h->lev[l];
  const Geom gc = (xc && l + 1 < h->nlev) ? h->lev[l + 1].g : lv.g;
  const dim3 grid(((lv.g.nx + 1) / 2 + BX - 1) / BX, (lv.g.ny + BY - 1) / BY, lv.g.nz);
  const int cx = lv.c[0] ? lv.c[0] : 1, cy = lv.c[1] ? lv.c[1] : 1, cz = lv.c[2] ? lv.c[2] : 1;
  for (int colour = 0; colour < 2; ++colour)
    hipLaunchKernelGGL((k_half_sweep<T, TL>), grid, kBlock, 0, h->s, lv.g, X, rs, rd, sigma,
                       (const TL*)lv.L, xc, lv.active, gc, cx, cy, cz, colour, &h->st->omega,
                       done);
}

// Margin by which a later two-sweep-pass candidate of the autotuner must be
// faster than the one it has kept.
constexpr float kTuneMargin = 0.97f;

// With uniform_bricks 1 the two-sweep pass takes the uniform-brick map on
// levels of at least this many cells (2: on every level).  A workgroup checks
// its region's bricks before it starts (one dependent round trip to memory,
// about 2 us); on a 256^3 level the skipped face loads save far more (the
// pass about a quarter faster with a sphere of diameter 64, a third with no
// body), on 128^3 and smaller levels the check costs more than they save.
constexpr long long kUniformPassCells = 1LL << 23;

static const UBrick* pass_map(const gmg_handle* h, const Level& lv) {
  return (h->p.uniform_bricks == 2 || lv.g.n >= kUniformPassCells) ? lv.ub : nullptr;
}

// With uniform_bricks 1 a level has a uniform-brick map (read by its
// residual kernels, and by its two-sweep pass through the table of tile
// modes) when it has at least this many cells; with 2 every level has one.
// On smaller levels the map's checks lengthen kernels that are bound by
// latency, and rebuilding it costs each gmg_update_faces more than it saves
// (a 256 x 64 x 64 sequence of solves with a face update per step: 3.17 ms
// per step without the map, 3.45 with it on every level).
constexpr long long kMapCells = 1LL << 21;

static bool level_has_map(const gmg_params* p, const Geom& g) {
  return p->uniform_bricks == 2 || (p->uniform_bricks == 1 && g.n >= kMapCells);
}

static bool uses_tile_modes(const Level& lv) { return lv.tm != nullptr; }

// The face-mode table of level lv's pass at (ty, kchunk), if it was found
// for that tiling.
static const S2TileMode* pass_modes(const gmg_handle* h, const Level& lv, int ty, int kchunk) {
  return (uses_tile_modes(lv) && lv.tm_kc == kchunk && lv.tm_ty == ty) ? lv.tm : nullptr;
}

// Find the face modes of every level's current pass tiling (after the faces
// or a tiling changed; never inside a captured cycle).
static void refresh_pass_modes(gmg_handle* h) {
  for (int l = 0; l < h->nlev; ++l) {
    Level& lv = h->lev[l];
    lv.tm_kc = 0;
    if (!uses_tile_modes(lv) || lv.pair_kc <= 0) continue;
    const int ty = lv.pair_ty, kc = lv.pair_kc;
    const int nt = ((lv.g.nx + S2_TX - 1) / S2_TX) * ((lv.g.ny + ty - 1) / ty) *
                   ((lv.g.nz + kc - 1) / kc);
    if (ty == 16)
      hipLaunchKernelGGL((k_pass_modes<16>), dim3(nt), dim3(S2Cfg<16>::NTB), 0, h->s, lv.g, lv.ub,
                         lv.ubx, lv.uby, kc, lv.tm);
    else
      hipLaunchKernelGGL((k_pass_modes<8>), dim3(nt), dim3(S2Cfg<8>::NTB), 0, h->s, lv.g, lv.ub,
                         lv.ubx, lv.uby, kc, lv.tm);
    lv.tm_ty = ty;
    lv.tm_kc = kc;
  }
}

// Two consecutive sweeps of level l as one two-sweep pass (FP32 cycles, even
// nx): X[rd] = sweep(sweep(X[rs] (+ P x_c))), bitwise the result of two
// sweeps; rd != rs.
template <typename T, typename TL>
static void launch_pair(gmg_handle* h, int l, const Roles<T>& X, int rs, int rd, const T* sigma,
                        const T* xc, const int* done, int ty, int kchunk) {
  if constexpr (std::is_same<T, float>::value) {
    const Level& lv = h->lev[l];
    const Geom gc = (xc && l + 1 < h->nlev) ? h->lev[l + 1].g : lv.g;
    const int cx = lv.c[0] ? lv.c[0] : 1, cy = lv.c[1] ? lv.c[1] : 1, cz = lv.c[2] ? lv.c[2] : 1;
    auto go = [&](auto tyc) {
      constexpr int TY = decltype(tyc)::value;
      const S2TileMode* tm = pass_modes(h, lv, TY, kchunk);
      const UBrick* ub = tm ? nullptr : pass_map(h, lv);
      const dim3 grid(((lv.g.nx + S2_TX - 1) / S2_TX) * ((lv.g.ny + TY - 1) / TY) *
                      ((lv.g.nz + kchunk - 1) / kchunk));
      if (xc != nullptr)
        hipLaunchKernelGGL((k_rb_sweep2<T, TL, TY, true>), grid, dim3(S2Cfg<TY>::NTB), 0, h->s,
                           lv.g, X, rs, rd, sigma, (const TL*)lv.L, xc, lv.active, gc, cx, cy, cz,
                           kchunk, &h->st->omega, done, ub, lv.ubx, lv.uby, tm);
      else
        hipLaunchKernelGGL((k_rb_sweep2<T, TL, TY, false>), grid, dim3(S2Cfg<TY>::NTB), 0, h->s,
                           lv.g, X, rs, rd, sigma, (const TL*)lv.L, xc, lv.active, gc, cx, cy, cz,
                           kchunk, &h->st->omega, done, ub, lv.ubx, lv.uby, tm);
    };
    if (ty == 16)
      go(std::integral_constant<int, 16>{});
    else
      go(std::integral_constant<int, 8>{});
  }
}

// Workgroups of level l's two-sweep pass launch.
static long long pass_blocks(const Level& lv) {
  return (long long)((lv.g.nx + S2_TX - 1) / S2_TX) * ((lv.g.ny + lv.pair_ty - 1) / lv.pair_ty) *
         ((lv.g.nz + lv.pair_kc - 1) / lv.pair_kc);
}

// The deferred decision's first pass of level l (no correction): X[rd] =
// sweep(sweep(X[rs])) with the input-residual partials, omega and gate of o.
template <typename T, typename TL>
static void launch_pair_opt(gmg_handle* h, int l, const Roles<T>& X, int rs, int rd,
                            const T* sigma, const int* done, const SweepOpt& o) {
  if constexpr (std::is_same<T, float>::value) {
    const Level& lv = h->lev[l];
    auto go = [&](auto tyc) {
      constexpr int TY = decltype(tyc)::value;
      hipLaunchKernelGGL((k_rb_sweep2_res<T, TL, TY>), dim3(pass_blocks(lv)),
                         dim3(S2Cfg<TY>::NTB), 0, h->s, lv.g, X, rs, rd, sigma, (const TL*)lv.L,
                         lv.active, lv.pair_kc, o.omega ? o.omega : &h->st->omega, done,
                         o.res_part, o.gate,
                         pass_modes(h, lv, TY, lv.pair_kc) ? nullptr : pass_map(h, lv), lv.ubx,
                         lv.uby, pass_modes(h, lv, TY, lv.pair_kc));
    };
    if (lv.pair_ty == 16)
      go(std::integral_constant<int, 16>{});
    else
      go(std::integral_constant<int, 8>{});
  }
}

// One sweep of level l with the level's choice: the fused sweep with tiles
// of TY 4 or 8 rows (FP64 sweeps always use TY 4 for their LDS budget), or
// (ty 1) the split red and black launches.
template <typename T, typename TL>
static void enq_sweep(gmg_handle* h, int l, const Roles<T>& X, int rs, int rd, const T* sigma,
                      const T* xc, const int* done, const SweepOpt& o = {}) {
  const Level& lv = h->lev[l];
  if (lv.ty == 1 && o.res_part == nullptr && o.gate == nullptr && o.omega == nullptr)
    launch_split<T, TL>(h, l, X, rs, rd, sigma, xc, done);
  else if (sizeof(T) == 8 || lv.ty != 8)
    launch_sweep<T, TL, 4>(h, l, X, rs, rd, sigma, xc, done, lv.kchunk, o);
  else
    launch_sweep<T, TL, 8>(h, l, X, rs, rd, sigma, xc, done, lv.kchunk, o);
}

// nu sweeps of level l from role r (the first with the folded correction
// x_c), consecutive pairs as two-sweep passes where the level uses them;
// each launch writes the other role.  Returns the role of the result.
template <typename T, typename TL>
static int enq_sweeps(gmg_handle* h, int l, const Roles<T>& X, int r, const T* sigma, const T* xc,
                      const int* done, int nu) {
  const Level& lv = h->lev[l];
  for (int s = 0; s < nu;) {
    const int rd = next_role(l, r);
    const T* c = (s == 0) ? xc : nullptr;
    if (nu - s >= 2 && lv.pair_kc > 0) {
      launch_pair<T, TL>(h, l, X, r, rd, sigma, c, done, lv.pair_ty, lv.pair_kc);
      s += 2;
    } else {
      enq_sweep<T, TL>(h, l, X, r, rd, sigma, c, done);
      s += 1;
    }
    r = rd;
  }
  return r;
}

// z-blocks of a kernel that follows the nu sweeps of level l, per z-chunk of
// the two-sweep passes those sweeps ran as (planes_per_block fine planes per
// z-block of nzb), for chunk_top_first; 1 where the sweeps were not all
// passes or the chunks do not tile the z-blocks evenly.
static int zper_after_passes(const gmg_handle* h, int l, int nu, int planes_per_block, int nzb) {
  const Level& lv = h->lev[l];
  const int kc = lv.pair_kc;
  if (kc <= 0 || nu < 2 || nu % 2 != 0 || kc % planes_per_block != 0) return 1;
  const int per = kc / planes_per_block;
  return (per > 1 && nzb % per == 0 && (long long)per * planes_per_block * (nzb / per) == lv.g.nz)
             ? per
             : 1;
}

// Coarse planes per workgroup of level lv's fused residual + restriction.
static int restrict_planes(const Level& lv, const Level& lc) {
  const long long one = (long long)((lv.g.nx + BX - 1) / BX) * ((lv.g.ny + BY - 1) / BY) * lc.g.nz;
  return one >= kRestrictQuadBlocks ? 4 : (one >= kRestrictPairBlocks ? 2 : 1);
}

// zper: the pass's z-chunk in workgroups of this launch (chunk_top_first).
template <typename T, typename TL>
static void enq_restrict(gmg_handle* h, int l, const Roles<T>& X, int role, const T* sigma,
                         T* sigma_c, T* x_c, const int* done, int zper = 1) {
  const Level& lv = h->lev[l];
  const Level& lc = h->lev[l + 1];
  const int rc = restrict_planes(lv, lc);
  const dim3 grid((lv.g.nx + BX - 1) / BX, (lv.g.ny + BY - 1) / BY, (lc.g.nz + rc - 1) / rc);
  if (rc == 4)
    hipLaunchKernelGGL((k_restrict_residual<T, TL, 4>), grid, kBlock, 0, h->s, lv.g, X, role,
                       sigma, (const TL*)lv.L, lc.g, lv.c[0], lv.c[1], lv.c[2], sigma_c, x_c,
                       done, zper, lv.ub, lv.ubx, lv.uby);
  else if (rc == 2)
    hipLaunchKernelGGL((k_restrict_residual<T, TL, 2>), grid, kBlock, 0, h->s, lv.g, X, role,
                       sigma, (const TL*)lv.L, lc.g, lv.c[0], lv.c[1], lv.c[2], sigma_c, x_c,
                       done, zper, lv.ub, lv.ubx, lv.uby);
  else
    hipLaunchKernelGGL((k_restrict_residual<T, TL, 1>), grid, kBlock, 0, h->s, lv.g, X, role,
                       sigma, (const TL*)lv.L, lc.g, lv.c[0], lv.c[1], lv.c[2], sigma_c, x_c,
                       done, zper, lv.ub, lv.ubx, lv.uby);
}

// LDS bytes the tail needs when it starts at level lt.
template <typename T, typename TL>
static long long tail_bytes(const gmg_handle* h, int lt) {
  long long b = 0;
  for (int l = lt; l < h->nlev; ++l) b += tail_level_bytes<T, TL>(h->lev[l].g.n);
  return b;
}

// Work vectors (r, z, two direction buffers, q, s = diag(-A)) and state of
// the conjugate gradient on levels [0, nl), allocated on first use; s is
// computed once from the level's faces.
template <typename T, typename TL>
static gmg_status ensure_pcg(gmg_handle* h, int nl) {
  if (!h->pst) {
    HIP_TRY(hipMalloc(&h->pst, kMaxLevels * sizeof(PCGState)));
    HIP_TRY(hipMemsetAsync(h->pst, 0, kMaxLevels * sizeof(PCGState), h->s));
    HIP_TRY(hipHostMalloc((void**)&h->hpst, sizeof(PCGState), hipHostMallocDefault));
  }
  for (int l = 0; l < nl; ++l) {
    if (h->pcg[l][0]) continue;
    const Level& lv = h->lev[l];
    for (int b = 0; b < 6; ++b) HIP_TRY(hipMalloc(&h->pcg[l][b], lv.g.n * sizeof(T)));
    hipLaunchKernelGGL((k_pcg_diag<T, TL>), cell_grid(lv.g), kBlock, 0, h->s, lv.g,
                       (const TL*)lv.L, (T*)h->pcg[l][5]);
    HIP_TRY(hipGetLastError());
  }
  return GMG_OK;
}

// Start of a PCG run on level l from X[rs]: r, z, p and the run's state.
template <typename T, typename TL>
static void enq_pcg_start(gmg_handle* h, int l, const Roles<T>& X, int rs, const T* sigma,
                          double rtol, int max_it, const int* done) {
  const Level& lv = h->lev[l];
  const dim3 gr = red_grid(lv.g);
  T* const* b = (T* const*)h->pcg[l];
  hipLaunchKernelGGL((k_pcg_start<T, TL>), gr, kBlock, 0, h->s, lv.g, X, rs, sigma,
                     (const TL*)lv.L, (const T*)b[5], b[0], b[1], b[2], h->partials,
                     h->partials + h->maxpart, kResChunk, done);
  hipLaunchKernelGGL(k_pcg_begin, dim3(1), dim3(256), 0, h->s, h->pst + l, h->partials,
                     h->partials + h->maxpart, nblocks(gr), rtol, max_it, done);
}

// One PCG iteration on level l: X[dst] = X[src] + alpha p.  The direction
// buffers alternate with the iteration's parity (the first iteration of a
// run is even).
template <typename T, typename TL>
static void enq_pcg_iter(gmg_handle* h, int l, const Roles<T>& X, int src, int dst, int parity,
                         const int* done) {
  const Level& lv = h->lev[l];
  const dim3 gr = red_grid(lv.g);
  const long long np = nblocks(gr);
  T* const* b = (T* const*)h->pcg[l];
  PCGState* st = h->pst + l;
  hipLaunchKernelGGL((k_pcg_pq<T, TL>), gr, kBlock, 0, h->s, lv.g, (const T*)b[1],
                     (const T*)b[2 + parity], b[3 - parity], b[4], (const TL*)lv.L, st,
                     h->partials, kResChunk, done);
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(256), 0, h->s, st, h->partials, np, done);
  hipLaunchKernelGGL((k_pcg_xr<T>), gr, kBlock, 0, h->s, lv.g, X, src, dst, (const T*)b[3 - parity],
                     b[0], b[1], (const T*)b[4], (const T*)b[5], st, h->partials,
                     h->partials + h->maxpart, kResChunk, done);
  hipLaunchKernelGGL(k_pcg_next, dim3(1), dim3(256), 0, h->s, st, h->partials,
                     h->partials + h->maxpart, np, done);
}

// The PCG smoother: `iters` iterations restarted from X[rs], result in X[rd]
// (X[rs] itself when iters == 0).  Returns the role of the result.
template <typename T, typename TL>
static int enq_pcg_smooth(gmg_handle* h, int l, const Roles<T>& X, int rs, int rd,
                          const T* sigma, int iters, const int* done) {
  if (iters <= 0) return rs;
  enq_pcg_start<T, TL>(h, l, X, rs, sigma, 0.0, iters, done);
  for (int it = 0; it < iters; ++it) enq_pcg_iter<T, TL>(h, l, X, it == 0 ? rs : rd, rd, it & 1, done);
  return rd;
}

// Levels lt .. nlev-1 in one single-workgroup launch (gmg_tail.h).
template <typename T, typename TL>
static TailArgs<T, TL> tail_args(gmg_handle* h, int lt, const int* done, int* lds_bytes) {
  TailArgs<T, TL> a{};
  a.nl = h->nlev - lt;
  a.nu_pre = h->p.nu_pre;
  a.nu_post = h->p.nu_post;
  a.nu_coarse = h->p.nu_coarse;
  a.coarse_rtol = h->p.coarse_rtol;
  a.coarse_max = h->p.coarse_max;
  a.omega = &h->st->omega;
  a.done = done;
  a.sweeps = &h->st->coarse_sweeps;
  int off = 0;
  for (int q = 0; q < a.nl; ++q) {
    const Level& lv = h->lev[lt + q];
    TailLevel<T, TL>& t = a.lv[q];
    t.g = lv.g;
    t.x = (T*)lv.x[0];
    t.sigma = (T*)lv.sigma;
    t.L = (const TL*)lv.L;
    t.active = lv.active;
    t.cx = lv.c[0] ? lv.c[0] : 1;
    t.cy = lv.c[1] ? lv.c[1] : 1;
    t.cz = lv.c[2] ? lv.c[2] : 1;
    if (h->tail_global) continue;
    const long long n = lv.g.n;
    t.ox = off;
    t.os = t.ox + tail_round16(n * (long long)sizeof(T));
    t.oL = t.os + tail_round16(n * (long long)sizeof(T));
    t.oa = t.oL + tail_round16(3 * n * (long long)sizeof(TL));
    off = t.oa + tail_round16(n);
  }
  *lds_bytes = off;
  return a;
}

template <typename T, typename TL>
static void enq_tail(gmg_handle* h, int lt, const int* done) {
  int off = 0;
  const TailArgs<T, TL> a = tail_args<T, TL>(h, lt, done, &off);
  if (h->tail_global)
    hipLaunchKernelGGL((k_tail<T, TL, true>), dim3(1), dim3(kTailThreads), 0, h->s, a);
  else
    hipLaunchKernelGGL((k_tail<T, TL, false>), dim3(1), dim3(kTailThreads), off, h->s, a);
}

// First level of the tail: the first level >= 1 from which every level has
// at most tail_cells cells and all of them fit the tail's LDS budget and
// level count.  Failing that, a hierarchy of two or more levels with the
// red-black smoother runs its coarsest level alone through the tail in
// global memory (tail_global) if it has at most kTailGlobalCells cells;
// otherwise nlev (no tail).  Also lifts the kernel's dynamic-LDS limit.
template <typename T, typename TL>
static int plan_tail(gmg_handle* h) {
  h->tail_global = 0;
  if (h->p.smoother == GMG_SMOOTH_PCG || h->nlev < 2) return h->nlev;
  for (int l = 1; l < h->nlev; ++l) {
    if (h->lev[l].g.n > h->p.tail_cells || h->nlev - l > kTailMax ||
        tail_bytes<T, TL>(h, l) > kTailLds)
      continue;
    if (hipFuncSetAttribute((const void*)k_tail<T, TL, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kTailLds) != hipSuccess)
      break;
    return l;
  }
  if (h->lev[h->nlev - 1].g.n > kTailGlobalCells) return h->nlev;
  h->tail_global = 1;
  return h->nlev - 1;
}

// Deferred decision of gmg_solve (see k_spec_finish): the cycle's first
// sweep reads the candidate (level-0 role 1), writes role 2 and leaves the
// partials of its input residual in `part`; level-0 roles go through the
// solve state's map; the cycle's result is written to role 1.
struct SpecPlan {
  double* part;
  long long np;
  bool pass;  // the first smoothing step is a two-sweep pass
};

// V-cycle from level 0.  X0 is the level-0 role-0 buffer (with `sel`, the
// roles rotate on the device).  With a SpecPlan (and the mapped level-0
// roles R0), the first sweep is the speculative one and the decision on the
// previous cycle follows it.  Returns the level-0 role of the result.
template <typename T, typename TL>
static int enq_vcycle(gmg_handle* h, T* X0, const int* sel, const T* sigma0, const int* done,
                      const SpecPlan* sp = nullptr, const Roles<T>* R0 = nullptr) {
  const int nl = h->nlev;
  const gmg_params& p = h->p;
  int role[kMaxLevels];
  const int lt = h->tail;  // levels lt .. nl-1 run in one k_tail launch
  const bool pcg = p.smoother == GMG_SMOOTH_PCG;
  // descend: pre-smooth, then restrict the residual (coarse x starts at 0)
  for (int l = 0; l < lt; ++l) {
    const Roles<T> X = (l == 0 && R0) ? *R0 : level_roles<T>(h, l, X0, sel);
    const T* sg = (l == 0) ? sigma0 : (const T*)h->lev[l].sigma;
    const bool coarsest = (l == nl - 1);
    int r = 0;
    const int nsw = coarsest ? p.nu_coarse : p.nu_pre;
    if (l == 0 && sp) {
      // the first smoothing step (a two-sweep pass where level 0 uses them,
      // else one sweep) reads the candidate (role 1) with the speculative
      // omega and leaves its input's residual partials; the decision on the
      // previous cycle follows, and a gated step redoes it from the accepted
      // iterate (role 0) when that decision differs from the speculation
      SweepOpt first;
      first.res_part = sp->part;
      first.omega = &h->st->omega_spec;
      SweepOpt again;
      again.gate = &h->st->redo;
      int s = 0;
      if (sp->pass) {
        launch_pair_opt<T, TL>(h, 0, X, 1, 2, sg, done, first);
        hipLaunchKernelGGL(k_spec_finish, dim3(1), dim3(256), 0, h->s, sp->part, sp->np, h->st,
                           h->rule);
        launch_pair_opt<T, TL>(h, 0, X, 0, 2, sg, done, again);
        s = 2;
      } else {
        enq_sweep<T, TL>(h, 0, X, 1, 2, sg, nullptr, done, first);
        hipLaunchKernelGGL(k_spec_finish, dim3(1), dim3(256), 0, h->s, sp->part, sp->np, h->st,
                           h->rule);
        enq_sweep<T, TL>(h, 0, X, 0, 2, sg, nullptr, done, again);
        s = 1;
      }
      r = 2;
      while (s < nsw) {  // work roles 2 <-> 3
        const int rd = (r == 2) ? 3 : 2;
        if (nsw - s >= 2 && h->lev[0].pair_kc > 0) {
          launch_pair<T, TL>(h, 0, X, r, rd, sg, nullptr, done, h->lev[0].pair_ty,
                             h->lev[0].pair_kc);
          s += 2;
        } else {
          enq_sweep<T, TL>(h, 0, X, r, rd, sg, nullptr, done);
          s += 1;
        }
        r = rd;
      }
    } else if (pcg) {
      r = enq_pcg_smooth<T, TL>(h, l, X, r, next_role(l, r), sg, nsw, done);
    } else {
      r = enq_sweeps<T, TL>(h, l, X, r, sg, nullptr, done, nsw);
    }
    role[l] = r;
    if (coarsest) break;
    {
      const int rc = restrict_planes(h->lev[l], h->lev[l + 1]);
      enq_restrict<T, TL>(h, l, X, r, sg, (T*)h->lev[l + 1].sigma, (T*)h->lev[l + 1].x[0], done,
                          pcg ? 1
                              : zper_after_passes(h, l, nsw, rc * h->lev[l].c[2],
                                                  (h->lev[l + 1].g.nz + rc - 1) / rc));
    }
  }
  if (lt < nl) {
    enq_tail<T, TL>(h, lt, done);
    role[lt] = 0;  // the tail smooths in place in x[0]
  }
  // ascend: prolong + correct (folded into the first post-sweep), post-smooth
  const int top = (lt < nl) ? lt - 1 : nl - 2;
  for (int l = top; l >= 0; --l) {
    const Roles<T> X = (l == 0 && R0) ? *R0 : level_roles<T>(h, l, X0, sel);
    const T* sg = (l == 0) ? sigma0 : (const T*)h->lev[l].sigma;
    const Level& lv = h->lev[l];
    const T* xc = (const T*)h->lev[l + 1].x[role[l + 1]];
    int r = role[l];
    if (l == 0 && sp) {  // work roles 2 <-> 3, the last step writes the candidate role 1
      if (p.nu_post > 0) {
        for (int s = 0; s < p.nu_post;) {
          const bool pass = p.nu_post - s >= 2 && lv.pair_kc > 0;
          const int step = pass ? 2 : 1;
          const int rd = (s + step == p.nu_post) ? 1 : ((r == 2) ? 3 : 2);
          if (pass)
            launch_pair<T, TL>(h, 0, X, r, rd, sg, s == 0 ? xc : nullptr, done, lv.pair_ty,
                               lv.pair_kc);
          else
            enq_sweep<T, TL>(h, 0, X, r, rd, sg, s == 0 ? xc : nullptr, done);
          s += step;
          r = rd;
        }
      } else {
        const Level& lc = h->lev[1];
        hipLaunchKernelGGL((k_prolong<T>), cell_grid(lv.g), kBlock, 0, h->s, lv.g, X, r, 1,
                           lv.active, xc, lc.g, lv.c[0], lv.c[1], lv.c[2], done);
        r = 1;
      }
    } else if (p.nu_post > 0 && !pcg) {
      r = enq_sweeps<T, TL>(h, l, X, r, sg, xc, done, p.nu_post);
    } else {
      const int rd = (l == 0 && r == 0) ? 1 : r;  // never modify the accepted iterate
      const Level& lc = h->lev[l + 1];
      hipLaunchKernelGGL((k_prolong<T>), cell_grid(lv.g), kBlock, 0, h->s, lv.g, X, r, rd,
                         lv.active, xc, lc.g, lv.c[0], lv.c[1], lv.c[2], done);
      r = rd;
      if (pcg) r = enq_pcg_smooth<T, TL>(h, l, X, r, next_role(l, r), sg, p.nu_post, done);
    }
    role[l] = r;
  }
  return role[0];
}

// Level-0 residual-norm partials of role `role` into partials[off ...].
template <typename T, typename TL>
static long long enq_resnorm(gmg_handle* h, const Roles<T>& X, int role, const T* sigma,
                             const TL* L, T* r, long long off, const int* done) {
  const Level& lv = h->lev[0];
  const dim3 gr = red_grid(lv.g);
  const int zper = h->p.smoother == GMG_SMOOTH_RBGS
                       ? zper_after_passes(h, 0, h->nlev > 1 ? h->p.nu_post : h->p.nu_coarse,
                                           kResChunk, (int)gr.z)
                       : 1;
  // the map describes the level's stored faces: used when L is them
  const bool own = (const void*)L == lv.L;
  hipLaunchKernelGGL((k_residual<T, TL>), gr, kBlock, 0, h->s, lv.g, X, role, sigma, L, r,
                     h->partials + off, kResChunk, done, zper, own ? lv.ub : nullptr, lv.ubx,
                     lv.uby);
  return nblocks(gr);
}

#define DISPATCH_CYCLE(h, ...)                                     \
  do {                                                             \
    if ((h)->p.cycle_dtype == GMG_F64) {                           \
      typedef double T;                                            \
      typedef double TL;                                           \
      __VA_ARGS__;                                                 \
    } else if ((h)->p.l_storage == GMG_BF16) {                     \
      typedef float T;                                             \
      typedef uint16_t TL;                                         \
      __VA_ARGS__;                                                 \
    } else {                                                       \
      typedef float T;                                             \
      typedef float TL;                                            \
      __VA_ARGS__;                                                 \
    }                                                              \
  } while (0)

// ---------------------------------------------------------------------------
// Set-up
// ---------------------------------------------------------------------------

static bool can_coarsen(int n, int periodic, int min_coarse) {
  if (n % 2 != 0 || n / 2 < min_coarse) return false;
  if (periodic && (n / 2) % 2 != 0) return false;
  return true;
}

static gmg_status validate(const gmg_params* p) {
  if (!p) return fail(GMG_EINVAL, "params is NULL");
  for (int d = 0; d < 3; ++d) {
    if (p->n[d] < 1) return fail(GMG_ESHAPE, "n[d] must be >= 1");
    if (p->periodic[d] && (p->n[d] < 2 || p->n[d] % 2 != 0))
      return fail(GMG_ESHAPE, "a periodic direction needs an even size >= 2 (red-black colouring)");
  }
  const long long cells = (long long)p->n[0] * p->n[1] * p->n[2];
  if (cells > (1LL << 31) - 1) return fail(GMG_ESHAPE, "more than 2^31-1 cells");
  if (p->dtype != GMG_F32 && p->dtype != GMG_F64) return fail(GMG_EINVAL, "dtype must be F32 or F64");
  if (p->cycle_dtype != GMG_F32 && p->cycle_dtype != GMG_F64)
    return fail(GMG_EINVAL, "cycle_dtype must be F32 or F64");
  if (p->cycle_dtype == GMG_F64 && p->dtype != GMG_F64)
    return fail(GMG_EINVAL, "F64 cycles need F64 arrays");
  if (p->cycle_dtype == GMG_F64 && p->l_storage != GMG_F64)
    return fail(GMG_EINVAL, "F64 cycles need F64 face storage");
  if (p->cycle_dtype == GMG_F32 && p->l_storage != GMG_F32 && p->l_storage != GMG_BF16)
    return fail(GMG_EINVAL, "F32 cycles need F32 or BF16 face storage");
  if (p->min_coarse < 1 || p->max_levels < 0 || p->max_levels > kMaxLevels)
    return fail(GMG_EINVAL, "bad min_coarse / max_levels");
  if (p->nu_pre < 0 || p->nu_post < 0 || p->nu_coarse < 0 || p->nu_pre > 64 ||
      p->nu_post > 64 || p->nu_coarse > 256)
    return fail(GMG_EINVAL, "bad sweep counts");
  if (p->tail_cells < 0 || p->tail_cells > kTailMaxCells)
    return fail(GMG_EINVAL, "tail_cells must be in [0, 32768]");
  if (!(p->coarse_rtol >= 0.0 && p->coarse_rtol < 1.0))
    return fail(GMG_EINVAL, "coarse_rtol must be in [0, 1)");
  if (p->coarse_rtol > 0.0 && (p->coarse_max < 1 || p->coarse_max > 4096))
    return fail(GMG_EINVAL, "coarse_max must be in [1, 4096]");
  if (!(p->ir_target >= 0.0 && p->ir_target <= 1.0))
    return fail(GMG_EINVAL, "ir_target must be in [0, 1]");
  if (p->uniform_bricks < 0 || p->uniform_bricks > 2)
    return fail(GMG_EINVAL, "uniform_bricks must be 0, 1 or 2");
  if (p->smoother != GMG_SMOOTH_RBGS && p->smoother != GMG_SMOOTH_PCG)
    return fail(GMG_EINVAL, "smoother must be GMG_SMOOTH_RBGS or GMG_SMOOTH_PCG");
  if (p->deferred_norm != 0 && p->deferred_norm != 1)
    return fail(GMG_EINVAL, "deferred_norm must be 0 or 1");
  if (p->pair_sweeps != 0 && p->pair_sweeps != 1)
    return fail(GMG_EINVAL, "pair_sweeps must be 0 or 1");
  if (!(p->omega0 > 0) || !(p->omega_min > 0) || !(p->omega_max >= p->omega_min) ||
      !(p->theta_dec > 0) || !(p->theta_inc > 0) || !std::isfinite(p->omega_max) ||
      !std::isfinite(p->omega0) || !std::isfinite(p->theta_inc))
    return fail(GMG_EINVAL, "bad relaxation parameters");
  return GMG_OK;
}

static void free_handle(gmg_handle* h) {
  if (!h) return;
  for (int l = 0; l < h->nlev; ++l) {
    (void)hipFree(h->lev[l].L);
    (void)hipFree(h->lev[l].active);
    (void)hipFree(h->lev[l].ub);
    (void)hipFree(h->lev[l].tm);
    (void)hipFree(h->lev[l].x[0]);
    (void)hipFree(h->lev[l].x[1]);
    (void)hipFree(h->lev[l].sigma);
  }
  (void)hipFree(h->L0x);
  (void)hipFree(h->w[0]);
  (void)hipFree(h->w[1]);
  (void)hipFree(h->w[2]);
  (void)hipFree(h->spec_part);
  (void)hipFree(h->partials);
  (void)hipFree(h->st);
  if (h->hst) (void)hipHostFree(h->hst);
  (void)hipFree(h->ir);
  if (h->hir) (void)hipHostFree(h->hir);
  (void)hipFree(h->r64);
  (void)hipFree(h->b32);
  (void)hipFree(h->e32);
  if (h->cyc.exec) (void)hipGraphExecDestroy(h->cyc.exec);
  if (h->irs.exec) (void)hipGraphExecDestroy(h->irs.exec);
  if (h->pcgit.exec) (void)hipGraphExecDestroy(h->pcgit.exec);
  for (int l = 0; l < kMaxLevels; ++l)
    for (int b = 0; b < 6; ++b) (void)hipFree(h->pcg[l][b]);
  (void)hipFree(h->pst);
  if (h->hpst) (void)hipHostFree(h->hpst);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  delete h;
}

template <typename TI, typename TL>
static void enq_copy_faces(gmg_handle* h, const void* Lin, void* Lout) {
  const Level& lv = h->lev[0];
  hipLaunchKernelGGL((k_copy_faces<TI, TL>), cell_grid(lv.g), kBlock, 0, h->s, lv.g,
                     (const TI*)Lin, (TL*)Lout, &h->st->bad);
}

template <typename TL>
static void enq_build_levels(gmg_handle* h) {
  for (int l = 0; l + 1 < h->nlev; ++l) {
    const Level& lv = h->lev[l];
    const Level& lc = h->lev[l + 1];
    hipLaunchKernelGGL((k_restrict_faces<TL>), cell_grid(lc.g), kBlock, 0, h->s, lv.g,
                       (const TL*)lv.L, lc.g, lv.c[0], lv.c[1], lv.c[2], (TL*)lc.L);
  }
  for (int l = 0; l < h->nlev; ++l) {
    const Level& lv = h->lev[l];
    hipLaunchKernelGGL((k_active<TL>), cell_grid(lv.g), kBlock, 0, h->s, lv.g, (const TL*)lv.L,
                       lv.active);
    if (lv.ub)
      hipLaunchKernelGGL((k_uniform_bricks<TL>), dim3(lv.ubx, lv.uby, lv.ubz), kBlock, 0, h->s,
                         lv.g, (const TL*)lv.L, lv.active, lv.ub);
  }
}

// Level-0 faces from the caller's L (and the exact FP64 copy of a
// refinement handle), then every coarser level's faces and active mask.
static gmg_status enq_load_faces(gmg_handle* h, const void* L) {
  const gmg_params* p = &h->p;
  void* L0 = h->lev[0].L;
  if (p->dtype == GMG_F64) {
    if (p->l_storage == GMG_F64) enq_copy_faces<double, double>(h, L, L0);
    else if (p->l_storage == GMG_BF16) enq_copy_faces<double, uint16_t>(h, L, L0);
    else enq_copy_faces<double, float>(h, L, L0);
    if (h->L0x) enq_copy_faces<double, double>(h, L, h->L0x);
  } else {
    if (p->l_storage == GMG_BF16) enq_copy_faces<float, uint16_t>(h, L, L0);
    else enq_copy_faces<float, float>(h, L, L0);
  }
  HIP_TRY(hipGetLastError());
  if (p->l_storage == GMG_F64) enq_build_levels<double>(h);
  else if (p->l_storage == GMG_BF16) enq_build_levels<uint16_t>(h);
  else enq_build_levels<float>(h);
  refresh_pass_modes(h);
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

static gmg_status setup_impl(const gmg_params* p, const void* L, void* stream, gmg_handle* h) {
  h->p = *p;
  h->s = (hipStream_t)stream;
  // the PCG smoother has no relaxation factor, so a rejected cycle would
  // repeat identically: every cycle is accepted
  h->rule = OmegaRule{p->omega_min, p->omega_max, p->theta_dec, p->theta_inc,
                      p->smoother == GMG_SMOOTH_PCG ? 0 : p->rollback};
  // level plan (Sec. 3.2)
  int n[3] = {p->n[0], p->n[1], p->n[2]};
  int nl = 0;
  while (true) {
    Level& lv = h->lev[nl];
    lv.g = make_geom(n, p->periodic);
    bool ok[3];
    for (int d = 0; d < 3; ++d) ok[d] = can_coarsen(n[d], p->periodic[d], p->min_coarse);
    bool stop;
    int c[3];
    if (p->anisotropic) {
      for (int d = 0; d < 3; ++d) c[d] = ok[d] ? 2 : 1;
      stop = !(ok[0] || ok[1] || ok[2]);
    } else {
      // every dimension of the problem together; a direction of extent 1 on
      // the finest grid (2-D problems) is not a dimension and keeps factor 1
      stop = true;
      bool all_ok = true;
      for (int d = 0; d < 3; ++d) {
        const bool dim = p->n[d] > 1;
        c[d] = dim ? 2 : 1;
        if (dim) {
          stop = false;
          all_ok = all_ok && ok[d];
        }
      }
      stop = stop || !all_ok;
    }
    if ((p->max_levels && nl + 1 >= p->max_levels) || nl + 1 >= kMaxLevels) stop = true;
    ++nl;
    h->nlev = nl;
    if (stop) {
      lv.c[0] = lv.c[1] = lv.c[2] = 0;
      break;
    }
    for (int d = 0; d < 3; ++d) {
      lv.c[d] = c[d];
      n[d] /= c[d];
    }
  }
  // allocations
  const size_t cs = dsize(p->cycle_dtype), ls = dsize(p->l_storage);
  long long maxpart = 0;
  for (int l = 0; l < h->nlev; ++l) {
    Level& lv = h->lev[l];
    HIP_TRY(hipMalloc(&lv.L, 3 * lv.g.n * ls));
    HIP_TRY(hipMalloc(&lv.active, lv.g.n));
    lv.ubx = (lv.g.nx + BX - 1) / BX;
    lv.uby = (lv.g.ny + BY - 1) / BY;
    lv.ubz = (lv.g.nz + kUBZ - 1) / kUBZ;
    lv.ub = nullptr;
    lv.tm = nullptr;
    lv.tm_ty = lv.tm_kc = 0;
    if (level_has_map(p, lv.g)) {
      HIP_TRY(hipMalloc(&lv.ub, (size_t)lv.ubx * lv.uby * lv.ubz * sizeof(UBrick)));
      if (pair_capable(*p, lv.g))  // room for the most tiles: 64 x 8 columns, 1 plane
        HIP_TRY(hipMalloc(&lv.tm, (size_t)((lv.g.nx + S2_TX - 1) / S2_TX) *
                                      ((lv.g.ny + 7) / 8) * lv.g.nz * sizeof(S2TileMode)));
    }
    if (l > 0) {
      HIP_TRY(hipMalloc(&lv.x[0], lv.g.n * cs));
      HIP_TRY(hipMalloc(&lv.x[1], lv.g.n * cs));
      HIP_TRY(hipMalloc(&lv.sigma, lv.g.n * cs));
    }
    lv.ty = p->cycle_dtype == GMG_F64 ? SweepTY<double>::v : SweepTY<float>::v;
    lv.kchunk = sweep_kchunk(lv.g, lv.ty, p->cycle_dtype == GMG_F64 ? 8 : 4);
    // two-sweep passes: on by default at level 0, where a pass streams the
    // largest arrays; the autotuner decides for the other levels
    lv.pair_ty = kPairTYDefault;
    const bool mapped =
        p->uniform_bricks == 2 || (p->uniform_bricks == 1 && lv.g.n >= kUniformPassCells);
    lv.pair_kc =
        (l == 0 && pair_capable(*p, lv.g)) ? pair_kchunk(lv.g, lv.pair_ty, mapped ? 2 : 1) : 0;
  }
  maxpart = nblocks(red_grid(h->lev[0].g));
  h->maxpart = maxpart;
  HIP_TRY(hipMalloc(&h->partials, 2 * maxpart * sizeof(double)));
  HIP_TRY(hipMalloc(&h->w[0], h->lev[0].g.n * cs));
  HIP_TRY(hipMalloc(&h->w[1], h->lev[0].g.n * cs));
  if (p->dtype == p->cycle_dtype) {  // gmg_solve's deferred decision
    const Geom& g0 = h->lev[0].g;
    HIP_TRY(hipMalloc(&h->w[2], g0.n * cs));
    const long long maxblk = (long long)((g0.nx + SW_TX - 1) / SW_TX) * ((g0.ny + 3) / 4) * g0.nz;
    HIP_TRY(hipMalloc(&h->spec_part, maxblk * sizeof(double)));
  }
  HIP_TRY(hipMalloc(&h->st, sizeof(SolveState)));
  HIP_TRY(hipHostMalloc((void**)&h->hst, sizeof(SolveState), hipHostMallocDefault));
  std::memset(h->hst, 0, sizeof(SolveState));
  h->hst->omega = p->omega0;
  HIP_TRY(hipMemcpyAsync(h->st, h->hst, sizeof(SolveState), hipMemcpyHostToDevice, h->s));
  if (p->dtype == GMG_F64 && p->cycle_dtype == GMG_F32) {
    const long long n0 = h->lev[0].g.n;
    HIP_TRY(hipMalloc(&h->L0x, 3 * n0 * sizeof(double)));
    HIP_TRY(hipMalloc(&h->ir, sizeof(IRState)));
    HIP_TRY(hipHostMalloc((void**)&h->hir, sizeof(IRState), hipHostMallocDefault));
    HIP_TRY(hipMalloc(&h->r64, n0 * sizeof(double)));
    HIP_TRY(hipMalloc(&h->b32, n0 * sizeof(float)));
    HIP_TRY(hipMalloc(&h->e32, n0 * sizeof(float)));
  }
  GMG_TRY(enq_load_faces(h, L));
  DISPATCH_CYCLE(h, { h->tail = plan_tail<T, TL>(h); });
  if (p->coarse_rtol > 0.0 && p->smoother == GMG_SMOOTH_RBGS && h->nlev >= 2 &&
      h->tail == h->nlev)
    return fail(GMG_ESHAPE, "the coarsest-level rule (coarse_rtol > 0) needs a coarsest level of "
                            "at most 2^20 cells; set coarse_rtol = 0 for fixed sweeps");
  if (p->smoother == GMG_SMOOTH_PCG) DISPATCH_CYCLE(h, { GMG_TRY((ensure_pcg<T, TL>(h, h->nlev))); });
  HIP_TRY(hipMemcpyAsync(&h->hst->bad, &h->st->bad, sizeof(int), hipMemcpyDeviceToHost, h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  if (h->hst->bad) return fail(GMG_EINVAL, "a face coefficient is not finite (NaN or Inf)");
  return GMG_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

// Record the launches of `enqueue` (which must only enqueue work on h->s)
// into a graph on the capture stream, or reuse the one recorded for the same
// key pointers.  On success *exec is ready for hipGraphLaunch on any stream.
template <typename F>
static gmg_status captured(gmg_handle* h, CapturedSeq& cs, const void* k0, const void* k1,
                           F&& enqueue, hipGraphExec_t* exec) {
  if (cs.exec && cs.k0 == k0 && cs.k1 == k1) {
    *exec = cs.exec;
    return GMG_OK;
  }
  if (cs.exec) {
    HIP_TRY(hipGraphExecDestroy(cs.exec));
    cs.exec = nullptr;
  }
  if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  hipStream_t orig = h->s;
  h->s = h->cap;
  HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  gmg_status st = enqueue();
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap, &g);
  h->s = orig;
  if (st != GMG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(GMG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&cs.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) {
    cs.exec = nullptr;
    return fail(GMG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
  }
  cs.k0 = k0;
  cs.k1 = k1;
  *exec = cs.exec;
  return GMG_OK;
}

// Whether the deferred decision's first smoothing step is a two-sweep pass.
static bool spec_pass(const gmg_handle* h) {
  return h->p.cycle_dtype == GMG_F32 && h->p.nu_pre >= 2 && h->lev[0].pair_kc > 0;
}

// Whether gmg_solve defers each cycle's decision to the next cycle's first
// smoothing step (red-black smoother, at least one pre-sweep and two levels;
// the split sweep cannot leave partials).
static bool spec_ok(const gmg_handle* h) {
  return h->p.deferred_norm && h->p.smoother == GMG_SMOOTH_RBGS && h->p.nu_pre >= 1 &&
         h->nlev >= 2 && h->w[2] && h->spec_part && (spec_pass(h) || h->lev[0].ty != 1);
}

template <typename T, typename TL>
static gmg_status enq_solve_cycle(gmg_handle* h, T* xa, const T* sigma) {
  const Level& lv = h->lev[0];
  const long long np = nblocks(red_grid(lv.g));
  if (spec_ok(h)) {  // the cycle's norm is taken by the next cycle's first smoothing step
    const bool pass = spec_pass(h);
    const SpecPlan sp{h->spec_part,
                      pass ? pass_blocks(lv) : sweep_blocks(lv, sizeof(T) == 8 ? 4 : lv.ty), pass};
    const Roles<T> XM{{xa, (T*)h->w[0], (T*)h->w[1], (T*)h->w[2]}, nullptr, h->st->map};
    enq_vcycle<T, TL>(h, xa, nullptr, sigma, &h->st->done, &sp, &XM);
    HIP_TRY(hipGetLastError());
    return GMG_OK;
  }
  // otherwise: V-cycle, residual norm, decision
  const Roles<T> XS{{xa, (T*)h->w[0], (T*)h->w[1]}, &h->st->cur};
  const int f = enq_vcycle<T, TL>(h, xa, &h->st->cur, sigma, &h->st->done);
  enq_resnorm<T, TL>(h, XS, f, sigma, (const TL*)lv.L, nullptr, 0, &h->st->done);
  hipLaunchKernelGGL(k_cycle_finish, dim3(1), dim3(256), 0, h->s, h->partials, np, h->st, h->rule,
                     f);
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

template <typename TL>
static gmg_status ir_outer_step(gmg_handle* h, double* x, const double* sigma, int max_inner,
                                double inner_rtol) {
  const Level& lv = h->lev[0];
  const dim3 gr = red_grid(lv.g);
  const long long np = nblocks(gr);
  const Roles<double> X{{x, x, x}, nullptr};
  hipLaunchKernelGGL((k_residual<double, double>), gr, kBlock, 0, h->s, lv.g, X, 0, sigma,
                     (const double*)h->L0x, h->r64, h->partials, kResChunk, &h->ir->done, 1,
                     nullptr, 0, 0);
  hipLaunchKernelGGL(k_ir_check, dim3(1), dim3(256), 0, h->s, h->partials, np, h->ir);
  hipLaunchKernelGGL(k_scale_cast, gr, kBlock, 0, h->s, lv.g, (const double*)h->r64, h->ir,
                     h->b32, h->e32, h->partials + h->maxpart, kResChunk);
  hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(256), 0, h->s, h->partials + h->maxpart, np,
                     h->partials + h->maxpart, np, h->st, inner_rtol, max_inner, h->p.omega0,
                     &h->ir->done, (const double*)&h->ir->inner_rtol);
  const Roles<float> XS{{h->e32, (float*)h->w[0], (float*)h->w[1]}, &h->st->cur};
  for (int c = 0; c < max_inner; ++c) {
    const int f = enq_vcycle<float, TL>(h, h->e32, &h->st->cur, h->b32, &h->st->done);
    enq_resnorm<float, TL>(h, XS, f, h->b32, (const TL*)lv.L, nullptr, 0, &h->st->done);
    hipLaunchKernelGGL(k_cycle_finish, dim3(1), dim3(256), 0, h->s, h->partials, np, h->st,
                       h->rule, f);
  }
  hipLaunchKernelGGL(k_ir_update, cell_grid(lv.g), kBlock, 0, h->s, lv.g, x, XS, h->ir,
                     (const SolveState*)h->st);
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

// Forget recorded graphs (they embed the tile choice of every launch).
static gmg_status drop_graphs(gmg_handle* h) {
  if (h->cyc.exec) HIP_TRY(hipGraphExecDestroy(h->cyc.exec));
  if (h->irs.exec) HIP_TRY(hipGraphExecDestroy(h->irs.exec));
  if (h->pcgit.exec) HIP_TRY(hipGraphExecDestroy(h->pcgit.exec));
  h->cyc.exec = h->irs.exec = h->pcgit.exec = nullptr;
  return GMG_OK;
}

template <typename T, typename TL>
static gmg_status autotune_impl(gmg_handle* h, void* x, const void* sigma, int reps,
                                gmg_tune_report* rep) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int tys[2] = {8, 4};
  const int kcs[6] = {2, 4, 8, 16, 32, 64};
  for (int l = 0; l < h->nlev; ++l) {
    Level& lv = h->lev[l];
    T* a = (l == 0) ? (T*)x : (T*)lv.x[0];
    T* b = (l == 0) ? (T*)h->w[0] : (T*)lv.x[1];
    const T* sg = (l == 0) ? (const T*)sigma : (const T*)lv.sigma;
    const Roles<T> X{{a, b, a}, nullptr};
    rep->ty_default[l] = lv.ty;
    rep->kchunk_default[l] = lv.kchunk;
    float best = 1e30f, deft = 0.f;
    int bty = lv.ty, bkc = lv.kchunk;
    for (int it = -1; it <= 2 * 6; ++it) {
      // it == -1 times the default choice first, it == 12 the split sweep
      const int ty = (it < 0) ? lv.ty : (it == 12 ? 1 : tys[it / 6]);
      const int kc = (it < 0 || it == 12) ? lv.kchunk : kcs[it % 6];
      if (sizeof(T) == 8 && ty == 8) continue;
      if (kc > lv.g.nz) continue;
      auto run = [&]() {
        if (ty == 1)
          launch_split<T, TL>(h, l, X, 0, 1, sg, nullptr, nullptr);
        else if (ty == 4)
          launch_sweep<T, TL, 4>(h, l, X, 0, 1, sg, nullptr, nullptr, kc);
        else
          launch_sweep<T, TL, 8>(h, l, X, 0, 1, sg, nullptr, nullptr, kc);
      };
      run();  // warm-up
      HIP_TRY(hipEventRecord(e0, h->s));
      for (int r = 0; r < reps; ++r) run();
      HIP_TRY(hipEventRecord(e1, h->s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      ms /= reps;
      if (it < 0) deft = ms;
      if (ms < best) {
        best = ms;
        bty = ty;
        bkc = kc;
      }
    }
    lv.ty = bty;
    lv.kchunk = bkc;
    rep->ty[l] = bty;
    rep->kchunk[l] = bkc;
    rep->us[l] = 1e3 * best;
    rep->us_default[l] = 1e3 * deft;
    // two-sweep pass: kept where one pass beats two of the chosen sweeps.  A
    // level's passes run once without and (below the coarsest level) once
    // with the folded correction per cycle, so a candidate's cost is the mean
    // of the two (the coarse level's iterate buffer serves as the correction
    // operand; only the time matters here).
    rep->pair_kchunk[l] = 0;
    rep->pair_ty[l] = lv.pair_ty;
    rep->us_pair[l] = 0.0;
    if (std::is_same<T, float>::value && pair_capable(h->p, lv.g)) {
      const T* xc = (l + 1 < h->nlev) ? (const T*)h->lev[l + 1].x[0] : nullptr;
      float pbest = 1e30f;
      int pkc = 0, pty = lv.pair_ty;
      for (int ty : {16, 8}) {
        const int pkcs[8] = {pair_kchunk(lv.g, ty, pass_map(h, lv) ? 2 : 1), 4, 8, 16, 32, 64,
                             128, 256};
        for (int kc : pkcs) {
          if (kc > lv.g.nz) continue;
          float cost = 0.f;
          for (int fold = 0; fold < 2; ++fold) {
            const T* c = fold ? xc : nullptr;
            if (fold && c == nullptr) {
              cost *= 2.f;
              break;
            }
            launch_pair<T, TL>(h, l, X, 0, 1, sg, c, nullptr, ty, kc);  // warm-up
            HIP_TRY(hipEventRecord(e0, h->s));
            for (int r = 0; r < reps; ++r) launch_pair<T, TL>(h, l, X, 0, 1, sg, c, nullptr, ty, kc);
            HIP_TRY(hipEventRecord(e1, h->s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            cost += ms / reps;
          }
          const float ms = 0.5f * cost;  // mean time of one pass
          // a later candidate must beat the one kept by kTuneMargin: the
          // isolated times of close candidates change order from run to run
          // (and differ from their times inside a cycle), while the first
          // candidate of each height is the default rule's
          if (ms < kTuneMargin * pbest) {
            pbest = ms;
            pkc = kc;
            pty = ty;
          }
        }
      }
      lv.pair_kc = (pbest < 2.f * best) ? pkc : 0;
      lv.pair_ty = pty;
      rep->pair_kchunk[l] = lv.pair_kc;
      rep->pair_ty[l] = lv.pair_ty;
      rep->us_pair[l] = 1e3 * pbest;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  refresh_pass_modes(h);
  HIP_TRY(hipGetLastError());
  return drop_graphs(h);
}

// ---------------------------------------------------------------------------
// Residual without allocation
// ---------------------------------------------------------------------------

// Scratch of gmg_residual_noalloc: [0, P) partials of ||r||^2, [P, 2P)
// partials of ||sigma||^2 (P = kNoAllocPart, one per block of the reduction
// grid), [2P, 2P + 2) the two sums.  Every element a call reads it has
// written first, so nothing needs clearing between calls.
constexpr long long kNoAllocPart = 1LL << 18;
static __device__ __align__(256) double scratch[2 * kNoAllocPart + 2];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device
}  // namespace

// Device address of the current device's `scratch`, looked up once per
// device (the symbol's host-side name is not a device address).
static gmg_status scratch_address(double** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GMG_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GMG_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return GMG_OK;
}

// out = sqrt(sum of the n partials), on the device.
__global__ __launch_bounds__(256) void k_sum_sqrt_to(const double* p, long long n, double* out) {
  const double s = reduce_partials(p, n);
  if (threadIdx.x == 0) *out = sqrt(s);
}

extern "C" {

gmg_status gmg_default_params(gmg_params* p) {
  if (!p) return fail(GMG_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->n[0] = p->n[1] = p->n[2] = 0;
  p->dtype = GMG_F32;
  p->cycle_dtype = GMG_F32;
  p->l_storage = GMG_F32;
  p->anisotropic = 1;
  p->min_coarse = 4;
  p->max_levels = 0;
  p->nu_pre = 2;
  p->nu_post = 2;
  p->nu_coarse = 4;
  p->rollback = 1;
  p->graphs = 1;
  p->tail_cells = 4096;
  p->deferred_norm = 0;
  p->pair_sweeps = 1;
  p->omega0 = 1.0;
  p->omega_min = 0.1;
  p->omega_max = 1.0;
  p->theta_dec = 0.5;
  p->theta_inc = 1.2;
  p->coarse_rtol = 0.1;
  p->coarse_max = 64;
  p->ir_target = 0.5;
  p->uniform_bricks = 1;
  return GMG_OK;
}

gmg_status gmg_setup(const gmg_params* p, const void* L, void* stream, gmg_handle** out) {
  g_last_error.clear();
  if (!out || !L) return fail(GMG_EINVAL, "NULL L or out");
  *out = nullptr;
  GMG_TRY(validate(p));
  gmg_handle* h = new (std::nothrow) gmg_handle();
  if (!h) return fail(GMG_ENOMEM, "host allocation failed");
  std::memset((void*)h, 0, sizeof(gmg_handle));
  gmg_status s = setup_impl(p, L, stream, h);
  if (s != GMG_OK) {
    free_handle(h);
    return s;
  }
  *out = h;
  return GMG_OK;
}

gmg_status gmg_update_faces(gmg_handle* h, const void* L) {
  if (!h || !L) return fail(GMG_EINVAL, "NULL argument");
  h->hst->bad = 0;
  HIP_TRY(hipMemcpyAsync(&h->st->bad, &h->hst->bad, sizeof(int), hipMemcpyHostToDevice, h->s));
  GMG_TRY(enq_load_faces(h, L));
  for (int l = 0; l < h->nlev; ++l) {  // the PCG preconditioner diag(-A), where it exists
    if (!h->pcg[l][5]) continue;
    const Level& lv = h->lev[l];
    DISPATCH_CYCLE(h, {
      hipLaunchKernelGGL((k_pcg_diag<T, TL>), cell_grid(lv.g), kBlock, 0, h->s, lv.g,
                         (const TL*)lv.L, (T*)h->pcg[l][5]);
    });
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(&h->hst->bad, &h->st->bad, sizeof(int), hipMemcpyDeviceToHost, h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  if (h->hst->bad) return fail(GMG_EINVAL, "a face coefficient is not finite (NaN or Inf)");
  return GMG_OK;
}

gmg_status gmg_destroy(gmg_handle* h) {
  if (h) (void)hipStreamSynchronize(h->s);
  free_handle(h);
  return GMG_OK;
}

gmg_status gmg_num_levels(const gmg_handle* h, int32_t* nlevels) {
  if (!h || !nlevels) return fail(GMG_EINVAL, "NULL argument");
  *nlevels = h->nlev;
  return GMG_OK;
}

gmg_status gmg_level_shape(const gmg_handle* h, int32_t level, int32_t n[3], int32_t c[3]) {
  if (!h || !n || !c) return fail(GMG_EINVAL, "NULL argument");
  if (level < 0 || level >= h->nlev) return fail(GMG_EINVAL, "level out of range");
  const Level& lv = h->lev[level];
  n[0] = lv.g.nx;
  n[1] = lv.g.ny;
  n[2] = lv.g.nz;
  for (int d = 0; d < 3; ++d) c[d] = lv.c[d];
  return GMG_OK;
}

gmg_status gmg_level_faces(gmg_handle* h, int32_t level, void* L_out) {
  if (!h || !L_out) return fail(GMG_EINVAL, "NULL argument");
  if (level < 0 || level >= h->nlev) return fail(GMG_EINVAL, "level out of range");
  const Level& lv = h->lev[level];
  HIP_TRY(hipMemcpyAsync(L_out, lv.L, 3 * lv.g.n * dsize(h->p.l_storage),
                         hipMemcpyDeviceToDevice, h->s));
  return GMG_OK;
}

gmg_status gmg_residual(gmg_handle* h, const void* x, const void* sigma, void* r,
                        double* rnorm, double* snorm) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  const Level& lv = h->lev[0];
  const dim3 gr = red_grid(lv.g);
  double* pa = rnorm ? h->partials : nullptr;
  if (h->p.dtype == GMG_F64 && h->p.cycle_dtype == GMG_F32) {
    Roles<double> X{{(double*)x, (double*)x, (double*)x}, nullptr};
    hipLaunchKernelGGL((k_residual<double, double>), gr, kBlock, 0, h->s, lv.g, X, 0,
                       (const double*)sigma, (const double*)h->L0x, (double*)r, pa, kResChunk,
                       nullptr, 1, nullptr, 0, 0);
    if (snorm)
      hipLaunchKernelGGL((k_masked_sumsq<double>), gr, kBlock, 0, h->s, lv.g,
                         (const double*)sigma, lv.active, h->partials + h->maxpart, kResChunk);
  } else {
    DISPATCH_CYCLE(h, {
      Roles<T> X{{(T*)x, (T*)x, (T*)x}, nullptr};
      hipLaunchKernelGGL((k_residual<T, TL>), gr, kBlock, 0, h->s, lv.g, X, 0, (const T*)sigma,
                         (const TL*)lv.L, (T*)r, pa, kResChunk, nullptr, 1, lv.ub, lv.ubx,
                         lv.uby);
      if (snorm)
        hipLaunchKernelGGL((k_masked_sumsq<T>), gr, kBlock, 0, h->s, lv.g, (const T*)sigma,
                           lv.active, h->partials + h->maxpart, kResChunk);
    });
  }
  HIP_TRY(hipGetLastError());
  if (!rnorm && !snorm) return GMG_OK;
  // reduce both partial sets into the state's scratch, then read them back
  if (rnorm)
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(256), 0, h->s, h->partials, nblocks(gr),
                       &h->st->scr[0]);
  if (snorm)
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(256), 0, h->s, h->partials + h->maxpart,
                       nblocks(gr), &h->st->scr[1]);
  HIP_TRY(hipGetLastError());
  double tmp[2] = {0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(tmp, &h->st->scr[0], 2 * sizeof(double), hipMemcpyDeviceToHost, h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  if (rnorm) *rnorm = std::sqrt(tmp[0]);
  if (snorm) *snorm = std::sqrt(tmp[1]);
  return GMG_OK;
}

gmg_status gmg_residual_noalloc(gmg_handle* h, const void* x, const void* sigma, void* r,
                                double* rnorm, double* snorm) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  const Level& lv = h->lev[0];
  const dim3 gr = red_grid(lv.g);
  if (nblocks(gr) > kNoAllocPart)
    return fail(GMG_EINVAL, "gmg_residual_noalloc: level 0 needs " +
                                std::to_string(nblocks(gr)) + " reduction blocks, the scratch holds " +
                                std::to_string(kNoAllocPart));
  double* sc = nullptr;
  GMG_TRY(scratch_address(&sc));
  double* pr = rnorm ? sc : nullptr;
  double* ps = sc + kNoAllocPart;
  if (h->p.dtype == GMG_F64 && h->p.cycle_dtype == GMG_F32) {
    Roles<double> X{{(double*)x, (double*)x, (double*)x}, nullptr};
    hipLaunchKernelGGL((k_residual<double, double>), gr, kBlock, 0, h->s, lv.g, X, 0,
                       (const double*)sigma, (const double*)h->L0x, (double*)r, pr, kResChunk,
                       nullptr, 1, nullptr, 0, 0);
    if (snorm)
      hipLaunchKernelGGL((k_masked_sumsq<double>), gr, kBlock, 0, h->s, lv.g,
                         (const double*)sigma, lv.active, ps, kResChunk);
  } else {
    DISPATCH_CYCLE(h, {
      Roles<T> X{{(T*)x, (T*)x, (T*)x}, nullptr};
      hipLaunchKernelGGL((k_residual<T, TL>), gr, kBlock, 0, h->s, lv.g, X, 0, (const T*)sigma,
                         (const TL*)lv.L, (T*)r, pr, kResChunk, nullptr, 1, lv.ub, lv.ubx,
                         lv.uby);
      if (snorm)
        hipLaunchKernelGGL((k_masked_sumsq<T>), gr, kBlock, 0, h->s, lv.g, (const T*)sigma,
                           lv.active, ps, kResChunk);
    });
  }
  if (rnorm)
    hipLaunchKernelGGL(k_sum_sqrt_to, dim3(1), dim3(256), 0, h->s, pr, nblocks(gr), rnorm);
  if (snorm)
    hipLaunchKernelGGL(k_sum_sqrt_to, dim3(1), dim3(256), 0, h->s, ps, nblocks(gr), snorm);
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

gmg_status gmg_smooth(gmg_handle* h, int32_t level, void* x, const void* sigma,
                      int32_t sweeps) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  if (level < 0 || level >= h->nlev) return fail(GMG_EINVAL, "level out of range");
  if (sweeps < 0) return fail(GMG_EINVAL, "sweeps < 0");
  if (level == 0 && h->p.dtype != h->p.cycle_dtype)
    return fail(GMG_EINVAL, "level-0 smoothing needs dtype == cycle_dtype");
  const Level& lv = h->lev[level];
  DISPATCH_CYCLE(h, {
    // ping-pong between the caller's x (roles 0 and 2) and a work buffer of
    // that level (role 1), consecutive sweeps as two-sweep passes where the
    // level uses them
    T* work = (level == 0) ? (T*)h->w[0] : (T*)lv.x[1];
    Roles<T> X{{(T*)x, work, (T*)x}, nullptr};
    const int r = enq_sweeps<T, TL>(h, level, X, 0, (const T*)sigma, nullptr, nullptr, sweeps);
    if (r == 1)
      HIP_TRY(hipMemcpyAsync(x, work, lv.g.n * sizeof(T), hipMemcpyDeviceToDevice, h->s));
  });
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

gmg_status gmg_restrict_residual(gmg_handle* h, int32_t level, const void* x,
                                 const void* sigma, void* sigma_c, void* x_c) {
  if (!h || !x || !sigma || !sigma_c) return fail(GMG_EINVAL, "NULL argument");
  if (level < 0 || level + 1 >= h->nlev) return fail(GMG_EINVAL, "level has no coarser level");
  DISPATCH_CYCLE(h, {
    Roles<T> X{{(T*)x, (T*)x, (T*)x}, nullptr};
    enq_restrict<T, TL>(h, level, X, 0, (const T*)sigma, (T*)sigma_c, (T*)x_c, nullptr);
  });
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

gmg_status gmg_prolong_correct(gmg_handle* h, int32_t level, const void* x_c, void* x) {
  if (!h || !x || !x_c) return fail(GMG_EINVAL, "NULL argument");
  if (level < 0 || level + 1 >= h->nlev) return fail(GMG_EINVAL, "level has no coarser level");
  const Level& lv = h->lev[level];
  const Level& lc = h->lev[level + 1];
  DISPATCH_CYCLE(h, {
    Roles<T> X{{(T*)x, (T*)x, (T*)x}, nullptr};
    hipLaunchKernelGGL((k_prolong<T>), cell_grid(lv.g), kBlock, 0, h->s, lv.g, X, 0, 0,
                       lv.active, (const T*)x_c, lc.g, lv.c[0], lv.c[1], lv.c[2], nullptr);
  });
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

gmg_status gmg_get_omega(gmg_handle* h, double* omega) {
  if (!h || !omega) return fail(GMG_EINVAL, "NULL argument");
  HIP_TRY(hipMemcpyAsync(omega, &h->st->omega, sizeof(double), hipMemcpyDeviceToHost, h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  return GMG_OK;
}

gmg_status gmg_coarse_sweeps(gmg_handle* h, int32_t* sweeps) {
  if (!h || !sweeps) return fail(GMG_EINVAL, "NULL argument");
  HIP_TRY(hipMemcpyAsync(sweeps, &h->st->coarse_sweeps, sizeof(int32_t), hipMemcpyDeviceToHost,
                         h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  return GMG_OK;
}

gmg_status gmg_set_omega(gmg_handle* h, double omega) {
  if (!h) return fail(GMG_EINVAL, "NULL handle");
  if (!(omega > 0) || !std::isfinite(omega)) return fail(GMG_EINVAL, "omega must be > 0");
  hipLaunchKernelGGL(k_set_omega, dim3(1), dim3(1), 0, h->s, h->st, omega);
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

gmg_status gmg_vcycle(gmg_handle* h, void* x, const void* sigma, double* rnorm_after) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  if (h->p.dtype != h->p.cycle_dtype) return fail(GMG_EINVAL, "gmg_vcycle needs dtype == cycle_dtype");
  DISPATCH_CYCLE(h, {
    const int f = enq_vcycle<T, TL>(h, (T*)x, nullptr, (const T*)sigma, nullptr);
    if (f != 0)
      HIP_TRY(hipMemcpyAsync(x, h->w[f - 1], h->lev[0].g.n * sizeof(T), hipMemcpyDeviceToDevice,
                             h->s));
  });
  HIP_TRY(hipGetLastError());
  if (rnorm_after) return gmg_residual(h, x, sigma, nullptr, rnorm_after, nullptr);
  return GMG_OK;
}

gmg_status gmg_pcg(gmg_handle* h, void* x, const void* sigma, double rtol, int32_t max_iter,
                   gmg_pcg_info* info) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  if (h->p.dtype != h->p.cycle_dtype) return fail(GMG_EINVAL, "gmg_pcg needs dtype == cycle_dtype");
  if (!(rtol >= 0) || max_iter < 0) return fail(GMG_EINVAL, "bad rtol / max_iter");
  const Level& lv = h->lev[0];
  const long long np = nblocks(red_grid(lv.g));
  DISPATCH_CYCLE(h, {
    GMG_TRY((ensure_pcg<T, TL>(h, 1)));
    T* xa = (T*)x;
    const Roles<T> X{{xa, xa, xa}, nullptr};
    const int* done = &h->pst->done;
    hipLaunchKernelGGL((k_masked_sumsq<T>), red_grid(lv.g), kBlock, 0, h->s, lv.g,
                       (const T*)sigma, lv.active, h->partials, kResChunk);
    hipLaunchKernelGGL(k_pcg_snorm, dim3(1), dim3(256), 0, h->s, h->pst, h->partials, np);
    enq_pcg_start<T, TL>(h, 0, X, 0, (const T*)sigma, rtol, max_iter, nullptr);
    HIP_TRY(hipGetLastError());
    // iterations in pairs (even, odd), so that every replay starts on an
    // even iteration; kernels after the stopping test are no-ops
    auto pair = [&]() -> gmg_status {
      enq_pcg_iter<T, TL>(h, 0, X, 0, 0, 0, done);
      enq_pcg_iter<T, TL>(h, 0, X, 0, 0, 1, done);
      HIP_TRY(hipGetLastError());
      return GMG_OK;
    };
    int launched = 0, chunk = 8;
    while (true) {
      HIP_TRY(hipMemcpyAsync(h->hpst, h->pst, offsetof(PCGState, hist), hipMemcpyDeviceToHost,
                             h->s));
      HIP_TRY(hipStreamSynchronize(h->s));
      if (h->hpst->done || launched >= max_iter) break;
      const int pairs = std::max(1, std::min(chunk, (max_iter - launched + 1) / 2));
      if (h->p.graphs) {
        hipGraphExec_t ex = nullptr;
        GMG_TRY(captured(h, h->pcgit, xa, sigma, pair, &ex));
        for (int c = 0; c < pairs; ++c) HIP_TRY(hipGraphLaunch(ex, h->s));
      } else {
        for (int c = 0; c < pairs; ++c) GMG_TRY(pair());
      }
      launched += 2 * pairs;
      chunk = std::min(2 * chunk, 128);
    }
    HIP_TRY(hipMemcpyAsync(h->hpst, h->pst, sizeof(PCGState), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
  });
  const PCGState& s = *h->hpst;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = s.status;
    info->iterations = s.it;
    info->snorm = s.snorm;
    info->rnorm0 = s.rnorm0;
    info->rnorm = s.rnorm;
    for (int k = 0; k < std::min(s.it, GMG_MAX_HISTORY); ++k) info->history[k] = s.hist[k];
  }
  if (s.status == kStNonFinite)
    return fail(GMG_EINVAL, "residual norm not finite (NaN or Inf in sigma or x0)");
  return s.status == GMG_OK ? GMG_OK : fail(GMG_ENOCONV, "PCG did not reach the tolerance");
}

gmg_status gmg_solve(gmg_handle* h, void* x, const void* sigma, double rtol, int32_t max_cycles,
                     gmg_solve_info* info) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  if (h->p.dtype != h->p.cycle_dtype) return fail(GMG_EINVAL, "gmg_solve needs dtype == cycle_dtype");
  if (!(rtol >= 0) || max_cycles < 0) return fail(GMG_EINVAL, "bad rtol / max_cycles");
  const Level& lv = h->lev[0];
  const long long np = nblocks(red_grid(lv.g));
  const bool spec = spec_ok(h);
  int rounds = 0;
  DISPATCH_CYCLE(h, {
    T* xa = (T*)x;
    hipLaunchKernelGGL((k_start_norms<T, TL>), red_grid(lv.g), kBlock, 0, h->s, lv.g, xa,
                       (const T*)sigma, (const TL*)lv.L, h->partials, h->partials + h->maxpart,
                       kResChunk);
    hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(256), 0, h->s, h->partials, np,
                       h->partials + h->maxpart, np, h->st, rtol, (int)max_cycles, h->p.omega0,
                       nullptr, nullptr);
    HIP_TRY(hipGetLastError());
    int launched = 0, chunk = 2;
    while (true) {
      // The first round goes out right behind the start kernels, unpolled:
      // if the start already decided the solve (sigma = 0), its cycles find
      // `done` set and do nothing.
      if (launched > 0) {
        HIP_TRY(hipMemcpyAsync(h->hst, h->st, offsetof(SolveState, hist),
                               hipMemcpyDeviceToHost, h->s));
        HIP_TRY(hipStreamSynchronize(h->s));
      }
      // with the deferred decision the first pass decides nothing
      if ((launched > 0 && h->hst->done) || launched >= max_cycles + (spec ? 1 : 0)) break;
      if (launched > 0) {
        // size the next launch round from the observed contraction
        const double rho = h->hst->rho, tgt = rtol * h->hst->snorm;
        const double rate = std::pow(h->hst->rho / std::max(h->hst->rho0, 1e-300),
                                     1.0 / std::max(1, h->hst->cycles));
        if (tgt <= 0.0) {
          chunk = 16;  // rtol = 0: run to max_cycles
        } else if (rate > 0 && rate < 0.999 && rho > tgt) {
          chunk = (int)std::ceil(std::log(tgt / rho) / std::log(rate));
          chunk = std::max(1, std::min(chunk, 16));
        } else {
          chunk = 1;
        }
      }
      chunk = std::min(chunk, max_cycles + (spec ? 1 : 0) - launched);
      if (h->p.graphs) {
        hipGraphExec_t ex = nullptr;
        GMG_TRY(captured(h, h->cyc, xa, sigma,
                         [&]() { return enq_solve_cycle<T, TL>(h, xa, (const T*)sigma); }, &ex));
        for (int c = 0; c < chunk; ++c) HIP_TRY(hipGraphLaunch(ex, h->s));
      } else {
        for (int c = 0; c < chunk; ++c) GMG_TRY((enq_solve_cycle<T, TL>(h, xa, (const T*)sigma)));
      }
      launched += chunk;
      ++rounds;
    }
    HIP_TRY(hipMemcpyAsync(h->hst, h->st, sizeof(SolveState), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
    if (spec) {  // the accepted iterate is buffer map[0]: the caller's x or the fourth
      if (h->hst->map[0] == 3)
        HIP_TRY(hipMemcpyAsync(xa, h->w[2], lv.g.n * sizeof(T), hipMemcpyDeviceToDevice, h->s));
    } else {
      const int cur = h->hst->cur;
      if (cur != 0)
        HIP_TRY(hipMemcpyAsync(xa, h->w[cur - 1], lv.g.n * sizeof(T), hipMemcpyDeviceToDevice,
                               h->s));
    }
    HIP_TRY(hipStreamSynchronize(h->s));
  });
  const SolveState& s = *h->hst;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = s.status;
    info->cycles = s.cycles;
    info->accepted_cycles = s.accepted;
    info->launches = rounds;
    info->rnorm0 = s.rho0;
    info->rnorm = s.rho;
    info->snorm = s.snorm;
    info->omega = s.omega;
    const int nh = std::min(s.cycles, GMG_MAX_HISTORY);
    for (int c = 0; c < nh; ++c) {
      info->history[c] = s.hist[c];
      info->omegas[c] = s.omegas[c];
      info->accepted[c] = s.acc[c];
    }
  }
  if (s.status == kStNonFinite)
    return fail(GMG_EINVAL, "residual norm not finite (NaN or Inf in sigma or x0, or an "
                            "overflow); x holds the last accepted iterate");
  if (s.status != 0) return fail(GMG_ENOCONV, "max_cycles reached before rtol");
  return GMG_OK;
}

gmg_status gmg_solve_ir(gmg_handle* h, double* x, const double* sigma, double rtol,
                        int32_t max_outer, int32_t max_inner, double inner_rtol,
                        gmg_ir_info* info) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  if (h->p.dtype != GMG_F64 || h->p.cycle_dtype != GMG_F32)
    return fail(GMG_EINVAL, "gmg_solve_ir needs dtype F64 and cycle_dtype F32");
  if (!(rtol >= 0) || max_outer < 0 || max_inner < 0 || !(inner_rtol >= 0))
    return fail(GMG_EINVAL, "bad tolerances / step counts");
  const Level& lv = h->lev[0];
  const dim3 gr = red_grid(lv.g);
  const long long np = nblocks(gr);
  hipLaunchKernelGGL((k_masked_sumsq<double>), gr, kBlock, 0, h->s, lv.g, sigma, lv.active,
                     h->partials, kResChunk);
  hipLaunchKernelGGL(k_count_mask, gr, kBlock, 0, h->s, lv.g, lv.active, h->partials + h->maxpart,
                     kResChunk);
  hipLaunchKernelGGL(k_ir_init, dim3(1), dim3(256), 0, h->s, h->partials, h->partials + h->maxpart,
                     np, h->ir, h->st, rtol, (int)max_outer, inner_rtol, h->p.ir_target);
  HIP_TRY(hipGetLastError());
  auto step = [&]() {
    return h->p.l_storage == GMG_BF16 ? ir_outer_step<uint16_t>(h, x, sigma, max_inner, inner_rtol)
                                      : ir_outer_step<float>(h, x, sigma, max_inner, inner_rtol);
  };
  hipGraphExec_t ex = nullptr;
  if (h->p.graphs) {
    // the step depends on max_inner and inner_rtol too: re-record when they change
    if (h->irs.exec && (h->ir_inner != max_inner || h->ir_inner_rtol != inner_rtol)) {
      HIP_TRY(hipGraphExecDestroy(h->irs.exec));
      h->irs.exec = nullptr;
    }
    GMG_TRY(captured(h, h->irs, x, sigma, step, &ex));
    h->ir_inner = max_inner;
    h->ir_inner_rtol = inner_rtol;
  }
  for (int m = 0; m <= max_outer; ++m) {
    if (ex)
      HIP_TRY(hipGraphLaunch(ex, h->s));
    else
      GMG_TRY(step());
    HIP_TRY(hipMemcpyAsync(h->hir, h->ir, offsetof(IRState, hist), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
    if (h->hir->done) break;
  }
  HIP_TRY(hipMemcpyAsync(h->hir, h->ir, sizeof(IRState), hipMemcpyDeviceToHost, h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  const IRState& r = *h->hir;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = r.status;
    info->outer = r.outer;
    info->inner_total = r.inner_total;
    info->snorm = r.snorm;
    info->rnorm = r.rnorm;
    const int nh = std::min(r.outer + 1, GMG_MAX_HISTORY);
    for (int m = 0; m < nh; ++m) info->history[m] = r.hist[m];
    for (int m = 0; m < std::min(r.outer, GMG_MAX_HISTORY); ++m) info->inner_cycles[m] = r.inner[m];
  }
  if (r.status == kStNonFinite)
    return fail(GMG_EINVAL, "residual norm not finite (NaN or Inf in sigma or x0)");
  if (r.status != 0) return fail(GMG_ENOCONV, "max_outer reached before rtol");
  return GMG_OK;
}

gmg_status gmg_level_uniform(gmg_handle* h, int32_t level, int64_t* uniform,
                             int64_t* uniform_active, int64_t* total) {
  if (!h || !uniform || !total) return fail(GMG_EINVAL, "NULL argument");
  if (level < 0 || level >= h->nlev) return fail(GMG_EINVAL, "level out of range");
  const Level& lv = h->lev[level];
  *uniform = 0;
  *total = 0;
  if (uniform_active) *uniform_active = 0;
  if (!lv.ub) return GMG_OK;
  const size_t nb = (size_t)lv.ubx * lv.uby * lv.ubz;
  std::vector<UBrick> host(nb);
  HIP_TRY(hipMemcpyAsync(host.data(), lv.ub, nb * sizeof(UBrick), hipMemcpyDeviceToHost, h->s));
  HIP_TRY(hipStreamSynchronize(h->s));
  for (const UBrick& b : host) {
    *uniform += b.ok ? 1 : 0;
    if (uniform_active) *uniform_active += (b.ok && b.act) ? 1 : 0;
  }
  *total = (int64_t)nb;
  return GMG_OK;
}

gmg_status gmg_set_tiles(gmg_handle* h, int32_t level, int32_t ty, int32_t kchunk) {
  if (!h) return fail(GMG_EINVAL, "NULL handle");
  if (level < 0 || level >= h->nlev) return fail(GMG_EINVAL, "level out of range");
  if ((ty != 1 && ty != 4 && ty != 8) || (h->p.cycle_dtype == GMG_F64 && ty == 8))
    return fail(GMG_EINVAL, "ty must be 1 (split), 4 or 8 (1 or 4 for FP64 cycles)");
  if (kchunk < 1 || kchunk > h->lev[level].g.nz) return fail(GMG_EINVAL, "kchunk out of range");
  h->lev[level].ty = ty;
  h->lev[level].kchunk = kchunk;
  return drop_graphs(h);
}

gmg_status gmg_set_pair_sweeps(gmg_handle* h, int32_t level, int32_t ty, int32_t kchunk) {
  if (!h) return fail(GMG_EINVAL, "handle is NULL");
  if (level < 0 || level >= h->nlev) return fail(GMG_EINVAL, "level out of range");
  if (kchunk != 0 && ty != 8 && ty != 16) return fail(GMG_EINVAL, "ty must be 8 or 16");
  if (kchunk != 0 && !pair_capable(h->p, h->lev[level].g))
    return fail(GMG_EINVAL,
                "two-sweep passes need pair_sweeps = 1, FP32 cycles, the red-black smoother "
                "and an even nx");
  if (kchunk < 0 || kchunk > h->lev[level].g.nz) return fail(GMG_EINVAL, "kchunk out of range");
  h->lev[level].pair_kc = kchunk;
  if (kchunk != 0) h->lev[level].pair_ty = ty;
  refresh_pass_modes(h);
  HIP_TRY(hipGetLastError());
  return drop_graphs(h);
}

gmg_status gmg_autotune(gmg_handle* h, void* x, const void* sigma, int32_t reps,
                        gmg_tune_report* report) {
  if (!h || !x || !sigma || reps < 1) return fail(GMG_EINVAL, "bad autotune arguments");
  if (h->p.dtype != h->p.cycle_dtype)
    return fail(GMG_EINVAL, "gmg_autotune needs dtype == cycle_dtype (level-0 arrays)");
  gmg_tune_report local;
  gmg_tune_report* rep = report ? report : &local;
  std::memset(rep, 0, sizeof(*rep));
  rep->nlevels = h->nlev;
  gmg_status st = GMG_OK;
  DISPATCH_CYCLE(h, { st = autotune_impl<T, TL>(h, x, sigma, reps, rep); });
  if (st != GMG_OK) return st;
  HIP_TRY(hipStreamSynchronize(h->s));
  return GMG_OK;
}

const char* gmg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

#include "gmg_batch.h"
