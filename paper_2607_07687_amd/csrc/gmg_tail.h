// Coarse tail of the V-cycle in one workgroup.
//
// Below some size a level's sweep is pure latency: a fused-sweep launch on a
// 16^3 grid costs about as much as one on 128^3, and a V-cycle visits the
// small levels with a dozen launches.  Here one workgroup of kTailThreads
// threads runs everything from the first tail level down: pre-sweeps,
// residual restriction, the coarsest sweeps, prolongation + correction and
// post-sweeps, with workgroup barriers in place of kernel boundaries.  All
// tail levels (x, sigma, faces, active mask) are held in LDS for the whole
// launch; x and sigma go back to global memory at the end.
//
// Arithmetic is that of the grid-wide kernels: the same relax_cell per cell,
// colour by colour (a colour's cells depend only on the other colour, so an
// in-place half-sweep equals the simultaneous one), the residual from
// stencil_Ax, and the restriction sum of each coarse cell taken in the order
// of the tiled restriction kernel (z first per fine column, then x-pairs,
// then y-pairs).
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

template <typename T, typename TL>
__device__ __forceinline__ TailView<T, TL> tail_view(char* lds, const TailLevel<T, TL>& v) {
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

template <typename T, typename TL>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T, TL> a, const double* omega_p,
                                                       const int* done) {
  if (done != nullptr && *done) return;
  extern __shared__ __align__(16) char tail_lds[];
  const T omega = (T)(*omega_p);
  const int last = a.nl - 1;
  // stage every tail level in LDS (x and sigma of the first level come from
  // the restriction that precedes this launch; deeper levels are produced here)
  for (int l = 0; l < a.nl; ++l) {
    const TailLevel<T, TL>& v = a.lv[l];
    const TailView<T, TL> w = tail_view<T, TL>(tail_lds, v);
    const int n = (int)v.g.n;
    tail_copy<TL>(w.L, v.L, 3 * n);
    tail_copy<uint8_t>(w.a, v.active, n);
    if (l == 0) {
      tail_copy<T>(w.x, v.x, n);
      tail_copy<T>(w.s, v.sigma, n);
    }
  }
  __syncthreads();
  for (int l = 0; l < last; ++l) {
    const TailView<T, TL> f = tail_view<T, TL>(tail_lds, a.lv[l]);
    tail_sweeps<T, TL>(f, a.nu_pre, omega);
    tail_restrict<T, TL>(f, a.lv[l], tail_view<T, TL>(tail_lds, a.lv[l + 1]));
  }
  tail_sweeps<T, TL>(tail_view<T, TL>(tail_lds, a.lv[last]), a.nu_coarse, omega);
  for (int l = last - 1; l >= 0; --l) {
    const TailView<T, TL> f = tail_view<T, TL>(tail_lds, a.lv[l]);
    tail_prolong<T, TL>(f, a.lv[l], tail_view<T, TL>(tail_lds, a.lv[l + 1]));
    tail_sweeps<T, TL>(f, a.nu_post, omega);
  }
  for (int l = 0; l < a.nl; ++l) {
    const TailLevel<T, TL>& v = a.lv[l];
    const TailView<T, TL> w = tail_view<T, TL>(tail_lds, v);
    tail_copy<T>(v.x, w.x, (int)v.g.n);
    tail_copy<T>(v.sigma, w.s, (int)v.g.n);
  }
}

}  // namespace gmg
