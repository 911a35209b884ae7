// Coarse tail of the V-cycle in one workgroup.
//
// Below some size a level's sweep is pure latency: a fused-sweep launch on a
// 16^3 grid costs about as much as one on 128^3, and a V-cycle visits the
// small levels with a dozen launches.  Here one workgroup of kTailThreads
// threads runs everything from the first tail level down: pre-sweeps,
// residual restriction, the coarsest-level smoothing, prolongation +
// correction and post-sweeps, with workgroup barriers in place of kernel
// boundaries.  Tail levels (x, sigma, faces, active mask) are held in LDS for
// the whole launch and x and sigma go back to global memory at the end; a
// level too large for LDS (only ever the coarsest one, alone) is worked on
// in global memory by the same code.
//
// The coarsest level is smoothed either by nu_coarse sweeps or, with
// coarse_rtol > 0, in groups of nu_coarse sweeps until its residual norm has
// fallen to coarse_rtol times its value on entry (at most coarse_max): the paper's
// anisotropic coarsening (Sec. 3.2) reaches a coarsest grid on which the
// smoother alone removes the lowest wavenumbers, and this rule lets it do
// so.  The rule first removes the mean of the level's right-hand side over
// its active cells (zero in exact arithmetic on these singular levels; what
// rounding leaves there no sweep can remove), and its norms are FP64 sums in
// a fixed order.
//
// Arithmetic is that of the grid-wide kernels: the same relax_cell per cell,
// colour by colour (a colour's cells depend only on the other colour, so an
// in-place half-sweep equals the simultaneous one), the residual from
// stencil_Ax, and the restriction sum of each coarse cell taken in the order
// of the tiled restriction kernel (z first per fine column, then x-pairs,
// then y-pairs).  With one workgroup per problem the same body serves a batch
// of independent problems (k_tail_batch).
#pragma once

#include "gmg_device.h"

namespace gmg {

constexpr int kTailThreads = 1024;
constexpr int kTailMax = 8;                // levels the tail can hold
constexpr int kTailLds = 156 * 1024;       // LDS budget of the tail (bytes)

template <typename T, typename TL>
struct TailLevel {
  Geom g;
  T* x;             // global x (written back at the end)
  T* sigma;         // global sigma (read for the first level, written back)
  const TL* L;      // global faces
  const uint8_t* active;
  int cx, cy, cz;   // factors to the next level
  int ox, os, oL, oa;  // byte offsets of x, sigma, faces, mask in LDS
};

template <typename T, typename TL>
struct TailArgs {
  TailLevel<T, TL> lv[kTailMax];
  int nl;  // levels in the tail; the last is the coarsest
  int nu_pre, nu_post, nu_coarse;
  double coarse_rtol;  // > 0: the coarsest-level stopping rule (see above)
  int coarse_max;
  const double* omega;  // relaxation factor (device)
  const int* done;      // solve finished: the launch is a no-op (may be NULL)
  int* sweeps;          // receives the coarsest level's sweep count (may be NULL)
};

// LDS bytes of one level: x, sigma (T), three faces (TL), mask, each part
// rounded up to 16 bytes.
__host__ __device__ inline int tail_round16(long long b) { return (int)((b + 15) & ~15LL); }
template <typename T, typename TL>
__host__ __device__ inline int tail_level_bytes(long long n) {
  return 2 * tail_round16(n * (long long)sizeof(T)) + tail_round16(3 * n * (long long)sizeof(TL)) +
         tail_round16(n);
}

// a / b for 0 <= a < 2^22, b >= 1, from a float reciprocal and one fix-up.
__device__ __forceinline__ int tail_div(int a, int b, float rb) {
  int q = (int)((float)a * rb);
  const int r = a - q * b;
  if (r < 0) --q;
  else if (r >= b) ++q;
  return q;
}

template <typename T, typename TL>
struct TailView {  // one level in LDS
  Geom g;
  T* x;
  T* s;
  TL* L;
  uint8_t* a;
};

// GLOBAL: the level is used in place in global memory; otherwise it lives in
// LDS at its offsets.  A compile-time choice, so that the LDS pointers are
// known to be LDS pointers and the accesses become LDS instructions.
template <typename T, typename TL, bool GLOBAL>
__device__ __forceinline__ TailView<T, TL> tail_view(char* lds, const TailLevel<T, TL>& v) {
  if constexpr (GLOBAL)
    return TailView<T, TL>{v.g, v.x, v.sigma, const_cast<TL*>(v.L),
                           const_cast<uint8_t*>(v.active)};
  return TailView<T, TL>{v.g, (T*)(lds + v.ox), (T*)(lds + v.os), (TL*)(lds + v.oL),
                         (uint8_t*)(lds + v.oa)};
}

// One half-sweep of colour `colour` ((i + j + k) mod 2), in place: thread
// work items are x-pairs of a row, each holding exactly one cell per colour.
template <typename T, typename TL>
__device__ __forceinline__ void tail_half_sweep(const TailView<T, TL>& v, int colour, T omega) {
  const Geom& g = v.g;
  const int nx = g.nx, ny = g.ny;
  const int sy = nx, sz = nx * ny, n = sz * g.nz;
  const int pr = (nx + 1) >> 1;
  const int np = pr * ny * g.nz;
  const float rpr = 1.0f / (float)pr, rny = 1.0f / (float)ny;
  const TL* Lx = v.L;
  const TL* Ly = v.L + n;
  const TL* Lz = v.L + 2 * n;
  T* x = v.x;
  for (int p = threadIdx.x; p < np; p += kTailThreads) {
    const int row = tail_div(p, pr, rpr);
    const int m = p - row * pr;
    const int k = tail_div(row, ny, rny);
    const int j = row - k * ny;
    const int i = 2 * m + ((j + k + colour) & 1);
    if (i >= nx) continue;
    const int q = row * nx + i;
    // neighbours: wrap when periodic; outside a wall value and high face are 0
    const bool xe_in = i + 1 < nx || g.px, xw_in = i > 0 || g.px;
    const bool yn_in = j + 1 < ny || g.py, ys_in = j > 0 || g.py;
    const bool zt_in = k + 1 < g.nz || g.pz, zb_in = k > 0 || g.pz;
    const int qe = (i + 1 < nx) ? q + 1 : q - (nx - 1);
    const int qw = (i > 0) ? q - 1 : q + (nx - 1);
    const int qn = (j + 1 < ny) ? q + sy : q - (ny - 1) * sy;
    const int qs = (j > 0) ? q - sy : q + (ny - 1) * sy;
    const int qt = (k + 1 < g.nz) ? q + sz : q - (g.nz - 1) * sz;
    const int qb = (k > 0) ? q - sz : q + (g.nz - 1) * sz;
    x[q] = relax_cell<T>(x[q], xe_in ? x[qe] : T(0), xw_in ? x[qw] : T(0), yn_in ? x[qn] : T(0),
                         ys_in ? x[qs] : T(0), zt_in ? x[qt] : T(0), zb_in ? x[qb] : T(0),
                         ldL<T>(Lx, q), xe_in ? ldL<T>(Lx, qe) : T(0), ldL<T>(Ly, q),
                         yn_in ? ldL<T>(Ly, qn) : T(0), ldL<T>(Lz, q),
                         zt_in ? ldL<T>(Lz, qt) : T(0), v.s[q], omega);
  }
  __syncthreads();
}

template <typename T, typename TL>
__device__ __forceinline__ void tail_sweeps(const TailView<T, TL>& v, int nsw, T omega) {
  for (int s = 0; s < nsw; ++s) {
    tail_half_sweep<T, TL>(v, 0, omega);
    tail_half_sweep<T, TL>(v, 1, omega);
  }
}

// Sum over the cz fine planes of coarse plane K of the residual of fine
// column (i, j), active cells only.
template <typename T, typename TL>
__device__ __forceinline__ T tail_column_residual(const TailView<T, TL>& f, int cz, int i, int j,
                                                  int K) {
  const Geom& g = f.g;
  T acc = T(0);
  for (int dz = 0; dz < cz; ++dz) {
    const int k = K * cz + dz;
    const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
    const T xc = f.x[idx];
    T D;
    const T ax = stencil_Ax<T, TL>(g, f.x, f.L, idx, i, j, k, xc, D);
    if (D != T(0)) acc += f.s[idx] - ax;
  }
  return acc;
}

// sigma_c = R (sigma - A x) on the next level and x_c = 0.
template <typename T, typename TL>
__device__ __forceinline__ void tail_restrict(const TailView<T, TL>& f, const TailLevel<T, TL>& fl,
                                              const TailView<T, TL>& c) {
  const Geom& gc = c.g;
  const int ncell = (int)gc.n;
  const float rnx = 1.0f / (float)gc.nx, rny = 1.0f / (float)gc.ny;
  for (int q = threadIdx.x; q < ncell; q += kTailThreads) {
    const int row = tail_div(q, gc.nx, rnx);
    const int I = q - row * gc.nx;
    const int K = tail_div(row, gc.ny, rny);
    const int J = row - K * gc.ny;
    T r[2];
    for (int dy = 0; dy < fl.cy; ++dy) {
      const int j = J * fl.cy + dy;
      T a = tail_column_residual<T, TL>(f, fl.cz, I * fl.cx, j, K);
      if (fl.cx == 2) a += tail_column_residual<T, TL>(f, fl.cz, I * fl.cx + 1, j, K);
      r[dy] = a;
    }
    c.s[q] = (fl.cy == 2) ? r[0] + r[1] : r[0];
    c.x[q] = T(0);
  }
  __syncthreads();
}

// x += P x_c on active cells.
template <typename T, typename TL>
__device__ __forceinline__ void tail_prolong(const TailView<T, TL>& f, const TailLevel<T, TL>& fl,
                                             const TailView<T, TL>& c) {
  const Geom& g = f.g;
  const int ncell = (int)g.n;
  const float rnx = 1.0f / (float)g.nx, rny = 1.0f / (float)g.ny;
  for (int q = threadIdx.x; q < ncell; q += kTailThreads) {
    if (!f.a[q]) continue;
    const int row = tail_div(q, g.nx, rnx);
    const int i = q - row * g.nx;
    const int k = tail_div(row, g.ny, rny);
    const int j = row - k * g.ny;
    f.x[q] += c.x[(k / fl.cz) * (int)c.g.sz + (j / fl.cy) * (int)c.g.sy + i / fl.cx];
  }
  __syncthreads();
}

// The coarsest level is smoothed by a group of threads: the workgroup's
// first wavefront alone when the level has at most kWaveCells cells (its
// cells do not fill more, and between two half-sweeps a wavefront needs only
// its own memory operations completed: a fence, no barrier), else the whole
// workgroup.  The group's stride STRIDE names it.
constexpr int kWave = 64;
constexpr int kWaveCells = 256;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

template <int STRIDE>
__device__ __forceinline__ void grp_sync() {
  if constexpr (STRIDE == kWave)
    wave_sync();
  else
    __syncthreads();
}

// Sum over the wavefront, the same fixed order in every lane's result.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over the group, the result in every thread (red: one LDS double).
template <int STRIDE>
__device__ __forceinline__ double grp_sum(double v, double* red) {
  if constexpr (STRIDE == kWave) {
    return wave_sum(v);
  } else {
    const double s = block_sum(v, threadIdx.x, STRIDE);
    if (threadIdx.x == 0) *red = s;
    __syncthreads();
    const double out = *red;
    __syncthreads();  // *red is reused by the next sum
    return out;
  }
}

// Half-sweep of colour `colour` by the group, in place: work items are
// x-pairs of a row, each holding exactly one cell per colour.
template <typename T, typename TL, int STRIDE>
__device__ __forceinline__ void grp_half_sweep(const TailView<T, TL>& v, int colour, T omega) {
  const Geom& g = v.g;
  const int nx = g.nx, ny = g.ny;
  const int sy = nx, sz = nx * ny, n = sz * g.nz;
  const int pr = (nx + 1) >> 1;
  const int np = pr * ny * g.nz;
  const float rpr = 1.0f / (float)pr, rny = 1.0f / (float)ny;
  const TL* Lx = v.L;
  const TL* Ly = v.L + n;
  const TL* Lz = v.L + 2 * n;
  T* x = v.x;
  for (int p = threadIdx.x; p < np; p += STRIDE) {
    const int row = tail_div(p, pr, rpr);
    const int m = p - row * pr;
    const int k = tail_div(row, ny, rny);
    const int j = row - k * ny;
    const int i = 2 * m + ((j + k + colour) & 1);
    if (i >= nx) continue;
    const int q = row * nx + i;
    const bool xe_in = i + 1 < nx || g.px, xw_in = i > 0 || g.px;
    const bool yn_in = j + 1 < ny || g.py, ys_in = j > 0 || g.py;
    const bool zt_in = k + 1 < g.nz || g.pz, zb_in = k > 0 || g.pz;
    const int qe = (i + 1 < nx) ? q + 1 : q - (nx - 1);
    const int qw = (i > 0) ? q - 1 : q + (nx - 1);
    const int qn = (j + 1 < ny) ? q + sy : q - (ny - 1) * sy;
    const int qs = (j > 0) ? q - sy : q + (ny - 1) * sy;
    const int qt = (k + 1 < g.nz) ? q + sz : q - (g.nz - 1) * sz;
    const int qb = (k > 0) ? q - sz : q + (g.nz - 1) * sz;
    x[q] = relax_cell<T>(x[q], xe_in ? x[qe] : T(0), xw_in ? x[qw] : T(0), yn_in ? x[qn] : T(0),
                         ys_in ? x[qs] : T(0), zt_in ? x[qt] : T(0), zb_in ? x[qb] : T(0),
                         ldL<T>(Lx, q), xe_in ? ldL<T>(Lx, qe) : T(0), ldL<T>(Ly, q),
                         yn_in ? ldL<T>(Ly, qn) : T(0), ldL<T>(Lz, q),
                         zt_in ? ldL<T>(Lz, qt) : T(0), v.s[q], omega);
  }
  grp_sync<STRIDE>();
}

// Residual of cell q of a tail level (dtype arithmetic); `act` is D != 0.
template <typename T, typename TL>
__device__ __forceinline__ T tail_cell_residual(const TailView<T, TL>& v, int q, float rnx,
                                                float rny, bool& act) {
  const Geom& g = v.g;
  const int row = tail_div(q, g.nx, rnx);
  const int i = q - row * g.nx;
  const int k = tail_div(row, g.ny, rny);
  const int j = row - k * g.ny;
  T D;
  const T ax = stencil_Ax<T, TL>(g, v.x, v.L, q, i, j, k, v.x[q], D);
  act = D != T(0);
  return act ? v.s[q] - ax : T(0);
}

// ||sigma - A x||_2 over the active cells: FP64 squares of the dtype
// residuals summed per thread in cell order, then over the group.
template <typename T, typename TL, int STRIDE>
__device__ __forceinline__ double grp_resnorm(const TailView<T, TL>& v, double* red) {
  const Geom& g = v.g;
  const int ncell = (int)g.n;
  const float rnx = 1.0f / (float)g.nx, rny = 1.0f / (float)g.ny;
  double s2 = 0.0;
  for (int q = threadIdx.x; q < ncell; q += STRIDE) {
    bool act;
    const T r = tail_cell_residual<T, TL>(v, q, rnx, rny, act);
    if (act) s2 += (double)r * (double)r;
  }
  return sqrt(grp_sum<STRIDE>(s2, red));
}

// sigma -= its mean over the active cells (FP64 sum and mean, the
// difference rounded once to the dtype).  With walls and periodic
// directions only, every level is singular (constants are in the null
// space) and a right-hand side is solvable only with zero mean; the
// restricted residual has it in exact arithmetic, and this removes what
// rounding left, which the smoother could not reduce and which would drift
// the level's iterate along the null space.
template <typename T, typename TL, int STRIDE>
__device__ __forceinline__ void grp_project(const TailView<T, TL>& v, double* red) {
  const int ncell = (int)v.g.n;
  double s = 0.0, c = 0.0;
  for (int q = threadIdx.x; q < ncell; q += STRIDE)
    if (v.a[q]) {
      s += (double)v.s[q];
      c += 1.0;
    }
  s = grp_sum<STRIDE>(s, red);
  c = grp_sum<STRIDE>(c, red);
  const double mean = c > 0.0 ? s / c : 0.0;
  for (int q = threadIdx.x; q < ncell; q += STRIDE)
    if (v.a[q]) v.s[q] = (T)((double)v.s[q] - mean);
  grp_sync<STRIDE>();
}

// Smoothing of the coarsest level by one group: nu_coarse sweeps, or with
// coarse_rtol > 0 the right-hand side projected to zero mean, then sweeps in
// groups of max(1, nu_coarse), the residual norm checked after each, until
// it is at most coarse_rtol times its value on entry or coarse_max sweeps
// are done (the last group cut to fit).  Returns the number of sweeps.
template <typename T, typename TL, int STRIDE>
__device__ __forceinline__ int grp_coarsest(const TailView<T, TL>& v, int nu_coarse,
                                            double coarse_rtol, int coarse_max, T omega,
                                            double* red) {
  int n = 0;
  if (!(coarse_rtol > 0.0)) {
    for (; n < nu_coarse; ++n) {
      grp_half_sweep<T, TL, STRIDE>(v, 0, omega);
      grp_half_sweep<T, TL, STRIDE>(v, 1, omega);
    }
    return n;
  }
  grp_project<T, TL, STRIDE>(v, red);
  const double lim = coarse_rtol * grp_resnorm<T, TL, STRIDE>(v, red);
  const int group = nu_coarse > 1 ? nu_coarse : 1;
  while (n < coarse_max) {
    const int k = min(group, coarse_max - n);
    for (int s = 0; s < k; ++s) {
      grp_half_sweep<T, TL, STRIDE>(v, 0, omega);
      grp_half_sweep<T, TL, STRIDE>(v, 1, omega);
    }
    n += k;
    if (n < coarse_max && grp_resnorm<T, TL, STRIDE>(v, red) <= lim) break;
  }
  return n;
}

// Register-resident variant for the first wavefront on a level of at most
// 2 x 64 x-pairs: each lane owns up to two x-pairs, i.e. two cells of each
// colour, and keeps their indices, neighbour indices, faces and sigma in
// registers for the whole coarsest smoothing; a half-sweep then reads only
// the neighbours' x from LDS.  Every update is relax_cell on the operands
// grp_half_sweep passes it, so the iterates are bitwise the same.
constexpr int kRegPairs = 2 * kWave;

template <typename T>
struct RegCell {
  int q;       // cell index, -1: none
  int nb[6];   // x+1, x-1, y+1, y-1, z+1, z-1 (wrapped where periodic)
  int in;      // bit d: neighbour d is in the grid (or wrapped)
  T f[6];      // faces: low x, high x, low y, high y, low z, high z (0 beyond a wall)
  T sg;
};

template <typename T, typename TL>
__device__ __forceinline__ RegCell<T> reg_cell(const TailView<T, TL>& v, int p, int colour) {
  const Geom& g = v.g;
  const int nx = g.nx, ny = g.ny;
  const int sy = nx, sz = nx * ny, n = sz * g.nz;
  const int pr = (nx + 1) >> 1;
  RegCell<T> c;
  c.q = -1;
  if (p >= pr * ny * g.nz) return c;
  const int row = tail_div(p, pr, 1.0f / (float)pr);
  const int m = p - row * pr;
  const int k = tail_div(row, ny, 1.0f / (float)ny);
  const int j = row - k * ny;
  const int i = 2 * m + ((j + k + colour) & 1);
  if (i >= nx) return c;
  const int q = row * nx + i;
  c.q = q;
  const bool ok[6] = {i + 1 < nx || (bool)g.px, i > 0 || (bool)g.px,
                      j + 1 < ny || (bool)g.py, j > 0 || (bool)g.py,
                      k + 1 < g.nz || (bool)g.pz, k > 0 || (bool)g.pz};
  c.nb[0] = (i + 1 < nx) ? q + 1 : q - (nx - 1);
  c.nb[1] = (i > 0) ? q - 1 : q + (nx - 1);
  c.nb[2] = (j + 1 < ny) ? q + sy : q - (ny - 1) * sy;
  c.nb[3] = (j > 0) ? q - sy : q + (ny - 1) * sy;
  c.nb[4] = (k + 1 < g.nz) ? q + sz : q - (g.nz - 1) * sz;
  c.nb[5] = (k > 0) ? q - sz : q + (g.nz - 1) * sz;
  c.in = 0;
#pragma unroll
  for (int d = 0; d < 6; ++d) c.in |= ok[d] ? (1 << d) : 0;
  c.f[0] = ldL<T>(v.L, q);
  c.f[1] = ok[0] ? ldL<T>(v.L, c.nb[0]) : T(0);
  c.f[2] = ldL<T>(v.L + n, q);
  c.f[3] = ok[2] ? ldL<T>(v.L + n, c.nb[2]) : T(0);
  c.f[4] = ldL<T>(v.L + 2 * n, q);
  c.f[5] = ok[4] ? ldL<T>(v.L + 2 * n, c.nb[4]) : T(0);
  c.sg = T(0);
  return c;
}

// The six neighbour values of a cell (0 outside a wall) into nv.
template <typename T>
__device__ __forceinline__ void reg_nbrs(const T* x, const RegCell<T>& c, T (&nv)[6]) {
#pragma unroll
  for (int d = 0; d < 6; ++d) nv[d] = ((c.in >> d) & 1) ? x[c.nb[d]] : T(0);
}

template <typename T>
__device__ __forceinline__ void reg_relax(T* x, const RegCell<T>& c, T omega) {
  if (c.q < 0) return;
  T nv[6];
  reg_nbrs<T>(x, c, nv);
  x[c.q] = relax_cell<T>(x[c.q], nv[0], nv[1], nv[2], nv[3], nv[4], nv[5], c.f[0], c.f[1],
                         c.f[2], c.f[3], c.f[4], c.f[5], c.sg, omega);
}

// Squared residual sigma - A x of an owned active cell (0 otherwise).
template <typename T>
__device__ __forceinline__ double reg_res2(const T* x, const RegCell<T>& c) {
  if (c.q < 0) return 0.0;
  T nv[6];
  reg_nbrs<T>(x, c, nv);
  const T xc = x[c.q];
  T ax = T(0), d = T(0);
  ax += c.f[1] * (nv[0] - xc);
  ax += c.f[0] * (nv[1] - xc);
  d += c.f[0] + c.f[1];
  ax += c.f[3] * (nv[2] - xc);
  ax += c.f[2] * (nv[3] - xc);
  d += c.f[2] + c.f[3];
  ax += c.f[5] * (nv[4] - xc);
  ax += c.f[4] * (nv[5] - xc);
  d += c.f[4] + c.f[5];
  if (-d == T(0)) return 0.0;
  const T r = c.sg - ax;
  return (double)r * (double)r;
}

template <typename T, typename TL>
__device__ __forceinline__ int reg_coarsest(const TailView<T, TL>& v, int nu_coarse,
                                            double coarse_rtol, int coarse_max, T omega,
                                            double* red) {
  const int lane = threadIdx.x;
  RegCell<T> c[2][2];  // [colour][x-pair slot]
#pragma unroll
  for (int col = 0; col < 2; ++col)
#pragma unroll
    for (int it = 0; it < 2; ++it) c[col][it] = reg_cell<T, TL>(v, lane + kWave * it, col);
  const bool rule = coarse_rtol > 0.0;
  if (rule) grp_project<T, TL, kWave>(v, red);
#pragma unroll
  for (int col = 0; col < 2; ++col)
#pragma unroll
    for (int it = 0; it < 2; ++it)
      if (c[col][it].q >= 0) c[col][it].sg = v.s[c[col][it].q];
  auto sweep = [&]() {
#pragma unroll
    for (int col = 0; col < 2; ++col) {
      reg_relax<T>(v.x, c[col][0], omega);
      reg_relax<T>(v.x, c[col][1], omega);
      wave_sync();
    }
  };
  auto norm = [&]() {
    double a = 0.0;
#pragma unroll
    for (int col = 0; col < 2; ++col)
#pragma unroll
      for (int it = 0; it < 2; ++it) a += reg_res2<T>(v.x, c[col][it]);
    return sqrt(wave_sum(a));
  };
  int n = 0;
  if (!rule) {
    for (; n < nu_coarse; ++n) sweep();
    return n;
  }
  const double lim = coarse_rtol * norm();
  const int group = nu_coarse > 1 ? nu_coarse : 1;
  while (n < coarse_max) {
    const int k = min(group, coarse_max - n);
    for (int s2 = 0; s2 < k; ++s2) sweep();
    n += k;
    if (n < coarse_max && norm() <= lim) break;
  }
  return n;
}

// The coarsest level's smoothing (grp_coarsest) by the first wavefront or
// the workgroup; returns the number of sweeps to every thread.
template <typename T, typename TL>
__device__ __forceinline__ int tail_coarsest(const TailView<T, TL>& v, int nu_coarse,
                                             double coarse_rtol, int coarse_max, T omega,
                                             int* count) {
  __shared__ double red;
  const int pairs = ((v.g.nx + 1) >> 1) * v.g.ny * v.g.nz;
  if (pairs <= kRegPairs) {
    if (threadIdx.x < kWave) {
      const int n = reg_coarsest<T, TL>(v, nu_coarse, coarse_rtol, coarse_max, omega, &red);
      if (threadIdx.x == 0) *count = n;
    }
  } else if (v.g.n <= kWaveCells) {
    if (threadIdx.x < kWave) {
      const int n = grp_coarsest<T, TL, kWave>(v, nu_coarse, coarse_rtol, coarse_max, omega, &red);
      if (threadIdx.x == 0) *count = n;
    }
  } else {
    const int n =
        grp_coarsest<T, TL, kTailThreads>(v, nu_coarse, coarse_rtol, coarse_max, omega, &red);
    if (threadIdx.x == 0) *count = n;
  }
  __syncthreads();
  return *count;
}

// Copy n elements between global memory and LDS in 16-byte pieces, several
// in flight per thread (both ends 16-byte aligned), then the remaining bytes.
template <typename T>
__device__ __forceinline__ void tail_copy(T* dst, const T* src, int n) {
  const int nb = n * (int)sizeof(T);
  const int n16 = nb >> 4;
  uint4* d16 = reinterpret_cast<uint4*>(dst);
  const uint4* s16 = reinterpret_cast<const uint4*>(src);
  int q = threadIdx.x;
  for (; q + 3 * kTailThreads < n16; q += 4 * kTailThreads) {
    const uint4 a = s16[q], b = s16[q + kTailThreads], c = s16[q + 2 * kTailThreads],
                d = s16[q + 3 * kTailThreads];
    d16[q] = a;
    d16[q + kTailThreads] = b;
    d16[q + 2 * kTailThreads] = c;
    d16[q + 3 * kTailThreads] = d;
  }
  for (; q < n16; q += kTailThreads) d16[q] = s16[q];
  uint8_t* d1 = reinterpret_cast<uint8_t*>(dst);
  const uint8_t* s1 = reinterpret_cast<const uint8_t*>(src);
  for (int b = (n16 << 4) + (int)threadIdx.x; b < nb; b += kTailThreads) d1[b] = s1[b];
}

// The whole tail of one problem (see the top of this file).  GLOBAL: the
// tail is one level (the coarsest), used in place in global memory.
template <typename T, typename TL, bool GLOBAL>
__device__ __forceinline__ void tail_run(const TailArgs<T, TL>& a, char* tail_lds) {
  __shared__ int count;
  const T omega = (T)(*a.omega);
  const int last = a.nl - 1;
  // stage the levels in LDS (x and sigma of the first level come from the
  // restriction that precedes this launch; deeper levels are produced here)
  if constexpr (!GLOBAL) {
    for (int l = 0; l < a.nl; ++l) {
      const TailLevel<T, TL>& v = a.lv[l];
      const TailView<T, TL> w = tail_view<T, TL, false>(tail_lds, v);
      const int n = (int)v.g.n;
      tail_copy<TL>(w.L, v.L, 3 * n);
      tail_copy<uint8_t>(w.a, v.active, n);
      if (l == 0) {
        tail_copy<T>(w.x, v.x, n);
        tail_copy<T>(w.s, v.sigma, n);
      }
    }
    __syncthreads();
  }
  for (int l = 0; l < last; ++l) {
    const TailView<T, TL> f = tail_view<T, TL, GLOBAL>(tail_lds, a.lv[l]);
    tail_sweeps<T, TL>(f, a.nu_pre, omega);
    tail_restrict<T, TL>(f, a.lv[l], tail_view<T, TL, GLOBAL>(tail_lds, a.lv[l + 1]));
  }
  const int nc = tail_coarsest<T, TL>(tail_view<T, TL, GLOBAL>(tail_lds, a.lv[last]),
                                      a.nu_coarse, a.coarse_rtol, a.coarse_max, omega, &count);
  if (a.sweeps && threadIdx.x == 0) *a.sweeps = nc;
  for (int l = last - 1; l >= 0; --l) {
    const TailView<T, TL> f = tail_view<T, TL, GLOBAL>(tail_lds, a.lv[l]);
    tail_prolong<T, TL>(f, a.lv[l], tail_view<T, TL, GLOBAL>(tail_lds, a.lv[l + 1]));
    tail_sweeps<T, TL>(f, a.nu_post, omega);
  }
  if constexpr (!GLOBAL) {
    for (int l = 0; l < a.nl; ++l) {
      const TailLevel<T, TL>& v = a.lv[l];
      const TailView<T, TL> w = tail_view<T, TL, false>(tail_lds, v);
      tail_copy<T>(v.x, w.x, (int)v.g.n);
      tail_copy<T>(v.sigma, w.s, (int)v.g.n);
    }
  }
}

template <typename T, typename TL, bool GLOBAL>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T, TL> a) {
  if (a.done != nullptr && *a.done) return;
  extern __shared__ __align__(16) char tail_lds[];
  tail_run<T, TL, GLOBAL>(a, tail_lds);
}

// One workgroup per problem of a batch, each with its own tail.
template <typename T, typename TL, bool GLOBAL>
__global__ __launch_bounds__(kTailThreads) void k_tail_batch(
    const TailArgs<T, TL>* __restrict__ args) {
  const TailArgs<T, TL>& a = args[blockIdx.x];
  if (a.done != nullptr && *a.done) return;
  extern __shared__ __align__(16) char tail_lds[];
  tail_run<T, TL, GLOBAL>(a, tail_lds);
}

}  // namespace gmg
