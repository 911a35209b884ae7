// Device-side helpers shared by the GMG kernels: grid geometry, face loads
// for every storage format, the 7-point flux-form stencil, and deterministic
// block reductions for 64-lane CDNA wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmg {

// Geometry of one level.  n = nx*ny*nz cells; strides in elements.
struct Geom {
  int nx, ny, nz;
  int px, py, pz;  // 1 = periodic
  long long sy, sz, n;
};

// Face-coefficient loads: FP32, FP64, or BF16 kept as raw uint16 bits.
template <typename T> __device__ __forceinline__ T ldL(const float* p, long long i) { return (T)p[i]; }
template <typename T> __device__ __forceinline__ T ldL(const double* p, long long i) { return (T)p[i]; }
template <typename T> __device__ __forceinline__ T ldL(const uint16_t* p, long long i) {
  return (T)__uint_as_float(((uint32_t)p[i]) << 16);
}

// Stored-format conversions used when building the hierarchy.
template <typename TL> __device__ __forceinline__ TL to_storage(double v);
template <> __device__ __forceinline__ float to_storage<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ double to_storage<double>(double v) { return v; }
template <> __device__ __forceinline__ uint16_t to_storage<uint16_t>(double v) {
  // round to FP32 first, then FP32 -> BF16 round-to-nearest-even on the bits
  uint32_t u = __float_as_uint((float)v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Neighbour offsets along one direction for cell coordinate c of extent n:
// low neighbour (c-1, wrapping when periodic; self at a wall, where the low
// face is stored as 0) and high neighbour (c+1, wrapping; self at a wall with
// hi_ok = false so that the high face counts as 0).
struct Nb {
  long long lo, hi;
  bool hi_ok;
};
__device__ __forceinline__ Nb neighbours(int c, int n, int periodic, long long stride) {
  Nb r;
  r.lo = (c > 0) ? -stride : (periodic ? (long long)(n - 1) * stride : 0);
  if (c + 1 < n) {
    r.hi = stride;
    r.hi_ok = true;
  } else if (periodic) {
    r.hi = -(long long)(n - 1) * stride;
    r.hi_ok = true;
  } else {
    r.hi = 0;
    r.hi_ok = false;
  }
  return r;
}

// (A x)(I) in flux form and the diagonal D(I) = -(sum of the six faces).
// Summation order per direction: high face term, then low face term.
template <typename T, typename TL>
__device__ __forceinline__ T stencil_Ax(const Geom& g, const T* __restrict__ x,
                                        const TL* __restrict__ L, long long idx, int i,
                                        int j, int k, T xc, T& D) {
  T ax = T(0), s = T(0);
  {
    const Nb nb = neighbours(i, g.nx, g.px, 1);
    const T lm = ldL<T>(L, idx);
    const T lp = nb.hi_ok ? ldL<T>(L, idx + nb.hi) : T(0);
    ax += lp * (x[idx + nb.hi] - xc);
    ax += lm * (x[idx + nb.lo] - xc);
    s += lm + lp;
  }
  {
    const TL* Ly = L + g.n;
    const Nb nb = neighbours(j, g.ny, g.py, g.sy);
    const T lm = ldL<T>(Ly, idx);
    const T lp = nb.hi_ok ? ldL<T>(Ly, idx + nb.hi) : T(0);
    ax += lp * (x[idx + nb.hi] - xc);
    ax += lm * (x[idx + nb.lo] - xc);
    s += lm + lp;
  }
  {
    const TL* Lz = L + 2 * g.n;
    const Nb nb = neighbours(k, g.nz, g.pz, g.sz);
    const T lm = ldL<T>(Lz, idx);
    const T lp = nb.hi_ok ? ldL<T>(Lz, idx + nb.hi) : T(0);
    ax += lp * (x[idx + nb.hi] - xc);
    ax += lm * (x[idx + nb.lo] - xc);
    s += lm + lp;
  }
  D = -s;
  return ax;
}

// Relaxed Gauss-Seidel update of one cell from its six neighbour values
// (e, w: x+1, x-1; n, s: y+1, y-1; t, b: z+1, z-1), its six faces and sigma:
// x + omega (sigma - (A x)_off) / D with D = -(sum of faces); a cell with D = 0
// is left unchanged.  In FP32 the division is a multiplication by the
// hardware reciprocal of D (1 ulp), which costs a fraction of an IEEE
// division in the VALU-bound sweep kernels.  Every smoother calls this one
// function, so all of them round identically.
template <typename T>
__device__ __forceinline__ T relax_cell(T xc, T xe, T xw, T xn, T xs, T xt, T xb, T lxm, T lxp,
                                        T lym, T lyp, T lzm, T lzp, T sg, T omega) {
  T ax = T(0);
  ax += lxp * (xe - xc);
  ax += lxm * (xw - xc);
  ax += lyp * (xn - xc);
  ax += lym * (xs - xc);
  ax += lzp * (xt - xc);
  ax += lzm * (xb - xc);
  const T s = ((lxm + lxp) + (lym + lyp)) + (lzm + lzp);
  if (s == T(0)) return xc;
  if constexpr (sizeof(T) == 4)
    return xc + omega * (sg - ax) * __builtin_amdgcn_rcpf(-s);
  else
    return xc + omega * (sg - ax) / (-s);
}

// XCD-aware tile order.  The 8 XCDs of an MI355X each have their own L2 and
// receive workgroups round-robin (workgroup b runs on XCD b % 8).  Mapping
// hardware index b to logical tile t so that each XCD gets a contiguous range
// of tiles makes x- and y-neighbouring tiles share an L2, which then serves
// their halo re-reads.  A bijection on [0, nb).
constexpr int kXCDs = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb / kXCDs, r = nb % kXCDs;
  const int x = b % kXCDs, slot = b / kXCDs;
  return (x < r) ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

__device__ __forceinline__ bool stopped(const int* done) { return done != nullptr && *done; }

// Iterate buffers of a level by role.  Level 0 has three or four buffers
// whose roles change on the device: role 0 is the accepted iterate, the
// others are the cycle's work buffers.  With a selector, buffer
// (*sel + role) % 3 plays `role` (three buffers); with a map, buffer
// map[role] does (four buffers).  Coarse levels (and calls without either)
// use the buffers directly by role.
template <typename T>
struct Roles {
  T* p[4];
  const int* sel;
  const int* map;
  __device__ __forceinline__ T* get(int role) const {
    if (map != nullptr) return p[map[role]];
    const int base = (sel != nullptr) ? *sel : 0;
    return p[(base + role) % 3];
  }
};

// Sum of v over a block of `nthreads` (multiple of 64, <= 1024) threads,
// fixed order: wavefront shuffle tree, then wave partials in index order.
// The result is valid in thread 0 only.
__device__ __forceinline__ double block_sum(double v, int tid, int nthreads) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double wsum[16];
  const int lane = tid & 63, w = tid >> 6;
  if (lane == 0) wsum[w] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    const int nw = nthreads >> 6;
    for (int q = 0; q < nw; ++q) s += wsum[q];
  }
  return s;
}

}  // namespace gmg
