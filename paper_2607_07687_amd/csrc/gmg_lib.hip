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
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <new>
#include <string>

#include "gmg_kernels.h"

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

__device__ __forceinline__ bool stopped(const int* done) { return done != nullptr && *done; }

// Which level-0 buffer a cycle kernel reads (src) and works on (dst).  With a
// selector, the accepted iterate is in xa when *sel == 0 and in xb otherwise,
// and the cycle's work buffer is the other one; without one, both are xb.
template <typename T>
__device__ __forceinline__ void pick(T* xa, T* xb, const int* sel, T*& src, T*& dst) {
  if (sel == nullptr) {
    src = xa;
    dst = xb;
  } else if (*sel) {
    src = xb;
    dst = xa;
  } else {
    src = xa;
    dst = xb;
  }
}

// r = sigma - A x on active cells (0 elsewhere); optional store of r and
// per-block partial sums of r^2 (FP64).
template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_residual(Geom g, const T* xa, const T* xb,
                                                 const int* sel, int use_dst,
                                                 const T* __restrict__ sigma,
                                                 const TL* __restrict__ L, T* r,
                                                 double* partials, const int* done) {
  if (stopped(done)) return;
  T *src, *dst;
  pick(const_cast<T*>(xa), const_cast<T*>(xb), sel, src, dst);
  const T* x = use_dst ? dst : src;
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  double acc = 0.0;
  if (i < g.nx && j < g.ny) {
    const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
    const T xc = x[idx];
    T D;
    const T ax = stencil_Ax<T, TL>(g, x, L, idx, i, j, k, xc, D);
    const T rv = (D != T(0)) ? sigma[idx] - ax : T(0);
    if (r) r[idx] = rv;
    acc = (double)rv * (double)rv;
  }
  if (partials) {
    const int tid = threadIdx.x + BX * threadIdx.y;
    const double s = block_sum(acc, tid, BT);
    if (tid == 0)
      partials[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
  }
}

// Sum of v^2 over active cells (mask != 0), per-block partials.
template <typename T>
__global__ __launch_bounds__(BT) void k_masked_sumsq(Geom g, const T* __restrict__ v,
                                                     const uint8_t* __restrict__ mask,
                                                     double* partials) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  double acc = 0.0;
  if (i < g.nx && j < g.ny) {
    const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
    if (mask[idx]) acc = (double)v[idx] * (double)v[idx];
  }
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double s = block_sum(acc, tid, BT);
  if (tid == 0)
    partials[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// One red-black half-sweep of colour `colour`: each thread owns the pair of
// x-cells (2p, 2p+1) of its row and updates the one with (i+j+k)%2 == colour
// from the residual of the pre-sweep iterate.  mode 0: in place on dst.
// mode 1: reads src, writes the updated colour AND copies the other colour
// into dst (first half-sweep of a cycle that keeps src for rollback).
template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_rb_half(Geom g, T* xa, T* xb, const int* sel, int mode,
                                                const T* __restrict__ sigma,
                                                const TL* __restrict__ L, int colour,
                                                const double* omega_p, const int* done) {
  if (stopped(done)) return;
  T *src, *dst;
  pick(xa, xb, sel, src, dst);
  const T* x = mode ? src : dst;
  const int p = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (j >= g.ny) return;
  const int par = (j + k + colour) & 1;
  const int i = 2 * p + par;
  const long long row = (long long)k * g.sz + (long long)j * g.sy;
  if (mode) {
    const int io = 2 * p + (par ^ 1);
    if (io < g.nx) dst[row + io] = src[row + io];
  }
  if (i >= g.nx) return;
  const long long idx = row + i;
  const T xc = x[idx];
  T D;
  const T ax = stencil_Ax<T, TL>(g, x, L, idx, i, j, k, xc, D);
  T xn = xc;
  if (D != T(0)) {
    const T omega = (T)(*omega_p);
    xn = xc + omega * (sigma[idx] - ax) / D;
  }
  dst[idx] = xn;
}

// Copy src -> dst (level-0 work buffer initialisation when no pre-sweep runs).
template <typename T>
__global__ __launch_bounds__(BT) void k_copy_sel(Geom g, T* xa, T* xb, const int* sel,
                                                 const int* done) {
  if (stopped(done)) return;
  T *src, *dst;
  pick(xa, xb, sel, src, dst);
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const long long idx = (long long)blockIdx.z * g.sz + (long long)j * g.sy + i;
  dst[idx] = src[idx];
}

// Fused residual + restriction: one thread per coarse cell J sums the fine
// residuals over its c-block and zeroes the coarse initial guess.
template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_restrict_residual(
    Geom gf, const T* xa, const T* xb, const int* sel, const T* __restrict__ sigma,
    const TL* __restrict__ L, Geom gc, int cx, int cy, int cz, T* __restrict__ sigma_c,
    T* __restrict__ x_c, const int* done) {
  if (stopped(done)) return;
  T *src, *dst;
  pick(const_cast<T*>(xa), const_cast<T*>(xb), sel, src, dst);
  const T* x = dst;
  const int I = blockIdx.x * BX + threadIdx.x;
  const int J = blockIdx.y * BY + threadIdx.y;
  const int K = blockIdx.z;
  if (I >= gc.nx || J >= gc.ny) return;
  T acc = T(0);
  for (int sz = 0; sz < cz; ++sz) {
    const int k = K * cz + sz;
    for (int sy = 0; sy < cy; ++sy) {
      const int j = J * cy + sy;
      for (int sx = 0; sx < cx; ++sx) {
        const int i = I * cx + sx;
        const long long idx = (long long)k * gf.sz + (long long)j * gf.sy + i;
        const T xc = x[idx];
        T D;
        const T ax = stencil_Ax<T, TL>(gf, x, L, idx, i, j, k, xc, D);
        if (D != T(0)) acc += sigma[idx] - ax;
      }
    }
  }
  const long long cidx = (long long)K * gc.sz + (long long)J * gc.sy + I;
  sigma_c[cidx] = acc;
  if (x_c) x_c[cidx] = T(0);
}

// Piecewise-constant prolongation + correction on active fine cells.
template <typename T>
__global__ __launch_bounds__(BT) void k_prolong(Geom gf, T* xa, T* xb, const int* sel,
                                                const uint8_t* __restrict__ active,
                                                const T* __restrict__ x_c, Geom gc, int cx,
                                                int cy, int cz, const int* done) {
  if (stopped(done)) return;
  T *src, *dst;
  pick(xa, xb, sel, src, dst);
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= gf.nx || j >= gf.ny) return;
  const long long idx = (long long)k * gf.sz + (long long)j * gf.sy + i;
  if (!active[idx]) return;
  const long long cidx = (long long)(k / cz) * gc.sz + (long long)(j / cy) * gc.sy + i / cx;
  dst[idx] += x_c[cidx];
}

// Level-0 face copy from the caller's dtype into storage, zeroing the low
// face at index 0 of every wall direction.
template <typename TI, typename TL>
__global__ __launch_bounds__(BT) void k_copy_faces(Geom g, const TI* __restrict__ Lin,
                                                   TL* __restrict__ Lout) {
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
  double s = 0.0;
  for (long long q = tid; q < n; q += blockDim.x) s += p[q];
  return block_sum(s, tid, blockDim.x);
}

// Start of a solve: ||sigma|| (partials a) and ||r(x0)|| (partials b).
__global__ __launch_bounds__(256) void k_solve_init(const double* pa, long long na,
                                                    const double* pb, long long nb,
                                                    SolveState* st, double rtol,
                                                    int max_cycles, double omega0) {
  const double ss = reduce_partials(pa, na);
  __syncthreads();
  const double rr = reduce_partials(pb, nb);
  if (threadIdx.x == 0) {
    st->snorm = sqrt(ss);
    st->rho = st->rho0 = st->last = sqrt(rr);
    st->omega = omega0;
    st->rtol = rtol;
    st->cur = 0;
    st->cycles = 0;
    st->accepted = 0;
    st->max_cycles = max_cycles;
    const bool conv = (st->snorm == 0.0) || (st->rho <= rtol * st->snorm);
    st->status = conv ? 0 : 5;
    st->done = (conv || max_cycles <= 0) ? 1 : 0;
  }
}

// End of a V-cycle: new residual norm, the adaptive-relaxation decision
// (Sec. 3.1) and the convergence flag.
__global__ __launch_bounds__(256) void k_cycle_finish(const double* p, long long n,
                                                      SolveState* st, OmegaRule rule) {
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
  int accept;
  if (rn > st->rho) {  // growth
    st->omega = fmax(rule.omega_min, rule.theta_dec * st->omega);
    accept = rule.rollback ? 0 : 1;
    if (c < GMG_MAX_HISTORY) st->acc[c] = rule.rollback ? 0 : 1;
    if (!rule.rollback) {
      st->cur ^= 1;
      st->rho = rn;
    }
  } else {
    st->cur ^= 1;
    st->rho = rn;
    st->omega = fmin(rule.omega_max, rule.theta_inc * st->omega);
    st->accepted += 1;
    accept = 1;
    if (c < GMG_MAX_HISTORY) st->acc[c] = 1;
  }
  (void)accept;
  st->cycles = c + 1;
  const bool conv = st->rho <= st->rtol * st->snorm;
  if (conv) st->status = 0;
  if (conv || st->cycles >= st->max_cycles) st->done = 1;
}

__global__ void k_set_omega(SolveState* st, double omega) { st->omega = omega; }

__global__ __launch_bounds__(256) void k_sum_to(const double* p, long long n, double* out) {
  const double s = reduce_partials(p, n);
  if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------

namespace {

constexpr int kMaxLevels = 32;

struct Level {
  Geom g;
  int c[3];      // factor to the next level; 0 on the coarsest
  void* L;       // [3][nz][ny][nx] in l_storage
  uint8_t* active;
  void* x;       // cycle dtype (levels >= 1)
  void* sigma;
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
dim3 pair_grid(const Geom& g) {
  const int np = (g.nx + 1) / 2;
  return dim3((np + BX - 1) / BX, (g.ny + BY - 1) / BY, g.nz);
}
long long nblocks(dim3 d) { return (long long)d.x * d.y * d.z; }

}  // namespace

struct gmg_handle {
  gmg_params p;
  hipStream_t s;
  int nlev;
  Level lev[kMaxLevels];
  void* L0x;     // exact FP64 level-0 faces (dtype F64 with F32 cycles)
  void* xwork;   // second level-0 iterate (cycle dtype)
  double* partials;  // 2 * maxpart
  long long maxpart;
  SolveState* st;
  SolveState* hst;   // pinned host mirror
  OmegaRule rule;
};

static const dim3 kBlock(BX, BY, 1);

// ---------------------------------------------------------------------------
// Typed enqueue helpers
// ---------------------------------------------------------------------------

template <typename T, typename TL>
static void enq_half(gmg_handle* h, int l, T* xa, T* xb, const int* sel, int mode,
                     const T* sigma, int colour, const int* done) {
  const Level& lv = h->lev[l];
  hipLaunchKernelGGL((k_rb_half<T, TL>), pair_grid(lv.g), kBlock, 0, h->s, lv.g, xa, xb, sel,
                     mode, sigma, (const TL*)lv.L, colour, &h->st->omega, done);
}

template <typename T, typename TL>
static void enq_sweeps(gmg_handle* h, int l, T* xa, T* xb, const int* sel, int& first_copy,
                       const T* sigma, int sweeps, const int* done) {
  for (int s = 0; s < sweeps; ++s)
    for (int c = 0; c < 2; ++c) {
      enq_half<T, TL>(h, l, xa, xb, sel, first_copy, sigma, c, done);
      first_copy = 0;
    }
}

// V-cycle from level 0 with the level-0 iterate selected by (xa, xb, sel);
// `copy` = 1 makes the first level-0 operation read src and fill dst.
template <typename T, typename TL>
static void enq_vcycle(gmg_handle* h, T* xa, T* xb, const int* sel, int copy,
                       const T* sigma0, const int* done) {
  const int nl = h->nlev;
  const gmg_params& p = h->p;
  // descend
  for (int l = 0; l < nl; ++l) {
    T* a = (l == 0) ? xa : (T*)h->lev[l].x;
    T* b = (l == 0) ? xb : (T*)h->lev[l].x;
    const int* sl = (l == 0) ? sel : nullptr;
    const T* sg = (l == 0) ? sigma0 : (const T*)h->lev[l].sigma;
    int fc = (l == 0) ? copy : 0;
    const bool coarsest = (l == nl - 1);
    enq_sweeps<T, TL>(h, l, a, b, sl, fc, sg, coarsest ? p.nu_coarse : p.nu_pre, done);
    if (fc) {  // no sweep ran on level 0: initialise the work buffer
      const Level& lv = h->lev[l];
      hipLaunchKernelGGL((k_copy_sel<T>), cell_grid(lv.g), kBlock, 0, h->s, lv.g, a, b, sl, done);
    }
    if (coarsest) break;
    const Level& lv = h->lev[l];
    const Level& lc = h->lev[l + 1];
    hipLaunchKernelGGL((k_restrict_residual<T, TL>), cell_grid(lc.g), kBlock, 0, h->s, lv.g,
                       (const T*)a, (const T*)b, sl, sg, (const TL*)lv.L, lc.g, lv.c[0], lv.c[1],
                       lv.c[2], (T*)lc.sigma, (T*)lc.x, done);
  }
  // ascend
  for (int l = nl - 2; l >= 0; --l) {
    T* a = (l == 0) ? xa : (T*)h->lev[l].x;
    T* b = (l == 0) ? xb : (T*)h->lev[l].x;
    const int* sl = (l == 0) ? sel : nullptr;
    const T* sg = (l == 0) ? sigma0 : (const T*)h->lev[l].sigma;
    const Level& lv = h->lev[l];
    const Level& lc = h->lev[l + 1];
    hipLaunchKernelGGL((k_prolong<T>), cell_grid(lv.g), kBlock, 0, h->s, lv.g, a, b, sl,
                       lv.active, (const T*)lc.x, lc.g, lv.c[0], lv.c[1], lv.c[2], done);
    int fc = 0;
    enq_sweeps<T, TL>(h, l, a, b, sl, fc, sg, p.nu_post, done);
  }
}

// Level-0 residual norm partials into partials[off ...].  use_dst selects the
// work buffer of (xa, xb, sel).  Returns the partial count.
template <typename T, typename TL>
static long long enq_resnorm(gmg_handle* h, const T* xa, const T* xb, const int* sel,
                             int use_dst, const T* sigma, const TL* L, T* r, long long off,
                             const int* done) {
  const Level& lv = h->lev[0];
  const dim3 gr = cell_grid(lv.g);
  hipLaunchKernelGGL((k_residual<T, TL>), gr, kBlock, 0, h->s, lv.g, xa, xb, sel, use_dst,
                     sigma, L, r, h->partials + off, done);
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
    (void)hipFree(h->lev[l].x);
    (void)hipFree(h->lev[l].sigma);
  }
  (void)hipFree(h->L0x);
  (void)hipFree(h->xwork);
  (void)hipFree(h->partials);
  (void)hipFree(h->st);
  if (h->hst) (void)hipHostFree(h->hst);
  delete h;
}

template <typename TI, typename TL>
static void enq_copy_faces(gmg_handle* h, const void* Lin, void* Lout) {
  const Level& lv = h->lev[0];
  hipLaunchKernelGGL((k_copy_faces<TI, TL>), cell_grid(lv.g), kBlock, 0, h->s, lv.g,
                     (const TI*)Lin, (TL*)Lout);
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
  }
}

static gmg_status setup_impl(const gmg_params* p, const void* L, void* stream, gmg_handle* h) {
  h->p = *p;
  h->s = (hipStream_t)stream;
  h->rule = OmegaRule{p->omega_min, p->omega_max, p->theta_dec, p->theta_inc, p->rollback};
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
      c[0] = c[1] = c[2] = 2;
      stop = !(ok[0] && ok[1] && ok[2]);
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
    if (l > 0) {
      HIP_TRY(hipMalloc(&lv.x, lv.g.n * cs));
      HIP_TRY(hipMalloc(&lv.sigma, lv.g.n * cs));
    }
  }
  maxpart = nblocks(cell_grid(h->lev[0].g));
  h->maxpart = maxpart;
  HIP_TRY(hipMalloc(&h->partials, 2 * maxpart * sizeof(double)));
  HIP_TRY(hipMalloc(&h->xwork, h->lev[0].g.n * cs));
  HIP_TRY(hipMalloc(&h->st, sizeof(SolveState)));
  HIP_TRY(hipHostMalloc((void**)&h->hst, sizeof(SolveState), hipHostMallocDefault));
  std::memset(h->hst, 0, sizeof(SolveState));
  h->hst->omega = p->omega0;
  HIP_TRY(hipMemcpyAsync(h->st, h->hst, sizeof(SolveState), hipMemcpyHostToDevice, h->s));
  // level-0 faces
  void* L0 = h->lev[0].L;
  if (p->dtype == GMG_F64) {
    if (p->l_storage == GMG_F64) enq_copy_faces<double, double>(h, L, L0);
    else if (p->l_storage == GMG_BF16) enq_copy_faces<double, uint16_t>(h, L, L0);
    else enq_copy_faces<double, float>(h, L, L0);
    if (p->cycle_dtype == GMG_F32) {
      HIP_TRY(hipMalloc(&h->L0x, 3 * h->lev[0].g.n * sizeof(double)));
      enq_copy_faces<double, double>(h, L, h->L0x);
    }
  } else {
    if (p->l_storage == GMG_BF16) enq_copy_faces<float, uint16_t>(h, L, L0);
    else enq_copy_faces<float, float>(h, L, L0);
  }
  HIP_TRY(hipGetLastError());
  if (p->l_storage == GMG_F64) enq_build_levels<double>(h);
  else if (p->l_storage == GMG_BF16) enq_build_levels<uint16_t>(h);
  else enq_build_levels<float>(h);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(h->s));
  return GMG_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

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
  p->omega0 = 1.0;
  p->omega_min = 0.1;
  p->omega_max = 1.0;
  p->theta_dec = 0.5;
  p->theta_inc = 1.2;
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
  const bool need = rnorm || snorm;
  const Level& lv = h->lev[0];
  const dim3 gr = cell_grid(lv.g);
  double* pa = rnorm ? h->partials : nullptr;
  if (h->p.dtype == GMG_F64 && h->p.cycle_dtype == GMG_F32) {
    hipLaunchKernelGGL((k_residual<double, double>), gr, kBlock, 0, h->s, lv.g,
                       (const double*)x, (const double*)x, nullptr, 0, (const double*)sigma,
                       (const double*)h->L0x, (double*)r, pa, nullptr);
    if (snorm)
      hipLaunchKernelGGL((k_masked_sumsq<double>), gr, kBlock, 0, h->s, lv.g,
                         (const double*)sigma, lv.active, h->partials + h->maxpart);
  } else {
    DISPATCH_CYCLE(h, {
      hipLaunchKernelGGL((k_residual<T, TL>), gr, kBlock, 0, h->s, lv.g, (const T*)x,
                         (const T*)x, nullptr, 0, (const T*)sigma, (const TL*)lv.L, (T*)r, pa,
                         nullptr);
      if (snorm)
        hipLaunchKernelGGL((k_masked_sumsq<T>), gr, kBlock, 0, h->s, lv.g, (const T*)sigma,
                           lv.active, h->partials + h->maxpart);
    });
  }
  HIP_TRY(hipGetLastError());
  if (!need) return GMG_OK;
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

gmg_status gmg_smooth(gmg_handle* h, int32_t level, void* x, const void* sigma,
                      int32_t sweeps) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  if (level < 0 || level >= h->nlev) return fail(GMG_EINVAL, "level out of range");
  if (sweeps < 0) return fail(GMG_EINVAL, "sweeps < 0");
  DISPATCH_CYCLE(h, {
    int fc = 0;
    enq_sweeps<T, TL>(h, level, (T*)x, (T*)x, nullptr, fc, (const T*)sigma, sweeps, nullptr);
  });
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

gmg_status gmg_restrict_residual(gmg_handle* h, int32_t level, const void* x,
                                 const void* sigma, void* sigma_c, void* x_c) {
  if (!h || !x || !sigma || !sigma_c) return fail(GMG_EINVAL, "NULL argument");
  if (level < 0 || level + 1 >= h->nlev) return fail(GMG_EINVAL, "level has no coarser level");
  const Level& lv = h->lev[level];
  const Level& lc = h->lev[level + 1];
  DISPATCH_CYCLE(h, {
    hipLaunchKernelGGL((k_restrict_residual<T, TL>), cell_grid(lc.g), kBlock, 0, h->s, lv.g,
                       (const T*)x, (const T*)x, nullptr, (const T*)sigma, (const TL*)lv.L, lc.g,
                       lv.c[0], lv.c[1], lv.c[2], (T*)sigma_c, (T*)x_c, nullptr);
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
    hipLaunchKernelGGL((k_prolong<T>), cell_grid(lv.g), kBlock, 0, h->s, lv.g, (T*)x, (T*)x,
                       nullptr, lv.active, (const T*)x_c, lc.g, lv.c[0], lv.c[1], lv.c[2],
                       nullptr);
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
  DISPATCH_CYCLE(h, { enq_vcycle<T, TL>(h, (T*)x, (T*)x, nullptr, 0, (const T*)sigma, nullptr); });
  HIP_TRY(hipGetLastError());
  if (rnorm_after) return gmg_residual(h, x, sigma, nullptr, rnorm_after, nullptr);
  return GMG_OK;
}

gmg_status gmg_solve(gmg_handle* h, void* x, const void* sigma, double rtol, int32_t max_cycles,
                     gmg_solve_info* info) {
  if (!h || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  if (h->p.dtype != h->p.cycle_dtype) return fail(GMG_EINVAL, "gmg_solve needs dtype == cycle_dtype");
  if (!(rtol >= 0) || max_cycles < 0) return fail(GMG_EINVAL, "bad rtol / max_cycles");
  const Level& lv = h->lev[0];
  const dim3 gr = cell_grid(lv.g);
  const long long np = nblocks(gr);
  int rounds = 0;
  DISPATCH_CYCLE(h, {
    T* xa = (T*)x;
    T* xb = (T*)h->xwork;
    hipLaunchKernelGGL((k_masked_sumsq<T>), gr, kBlock, 0, h->s, lv.g, (const T*)sigma, lv.active,
                       h->partials);
    enq_resnorm<T, TL>(h, xa, xa, nullptr, 0, (const T*)sigma, (const TL*)lv.L, nullptr,
                       h->maxpart, nullptr);
    hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(256), 0, h->s, h->partials, np,
                       h->partials + h->maxpart, np, h->st, rtol, (int)max_cycles, h->p.omega0);
    HIP_TRY(hipGetLastError());
    int launched = 0, chunk = 2;
    while (true) {
      HIP_TRY(hipMemcpyAsync(h->hst, h->st, offsetof(SolveState, hist), hipMemcpyDeviceToHost,
                             h->s));
      HIP_TRY(hipStreamSynchronize(h->s));
      if (h->hst->done || launched >= max_cycles) break;
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
      chunk = std::min(chunk, max_cycles - launched);
      for (int c = 0; c < chunk; ++c) {
        enq_vcycle<T, TL>(h, xa, xb, &h->st->cur, 1, (const T*)sigma, &h->st->done);
        enq_resnorm<T, TL>(h, xa, xb, &h->st->cur, 1, (const T*)sigma, (const TL*)lv.L, nullptr,
                           0, &h->st->done);
        hipLaunchKernelGGL(k_cycle_finish, dim3(1), dim3(256), 0, h->s, h->partials, np, h->st,
                           h->rule);
      }
      HIP_TRY(hipGetLastError());
      launched += chunk;
      ++rounds;
    }
    HIP_TRY(hipMemcpyAsync(h->hst, h->st, sizeof(SolveState), hipMemcpyDeviceToHost, h->s));
    HIP_TRY(hipStreamSynchronize(h->s));
    if (h->hst->cur == 1)
      HIP_TRY(hipMemcpyAsync(xa, xb, lv.g.n * sizeof(T), hipMemcpyDeviceToDevice, h->s));
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
  if (s.status != 0) return fail(GMG_ENOCONV, "max_cycles reached before rtol");
  return GMG_OK;
}

const char* gmg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
