// Jacobi-preconditioned conjugate gradient (PCG) on the symmetric positive
// (semi)definite form (-A) x = -sigma over the active cells: the paper's
// general-purpose solver and, restarted at every smoothing step, the smoother
// of its GMG-PCG comparison (Sec. 3, Table 1).  Included by gmg_lib.hip after
// its kernels (uses Roles, stopped, reduce_partials and the 128 x 2 cell
// blocks).
//
// Vectors, in the cycle precision T: r = b - B x = A x - sigma (B = -A),
// z = r / s with s = diag(-A), the direction p (two buffers: the direction
// update reads the old p at neighbours), q = B p.  The scalars (r.z, p.q,
// alpha, beta, ||r||) live in a PCGState on the device, FP64.  One iteration
// is four launches:
//   k_pcg_pq    p' = z + beta p, q = B p' (p' evaluated at the neighbours on
//               the fly), partials of p'.q
//   k_pcg_alpha alpha = r.z / p'.q
//   k_pcg_xr    x += alpha p', r -= alpha q, z = r / s, partials of r.z, r.r
//   k_pcg_next  beta, ||r||, history, stopping test
// and a solve or smoothing run starts with k_pcg_start (r, z, p = z and their
// partials) and k_pcg_begin.
#pragma once

namespace gmg {

struct PCGState {
  double rz;      // r . z
  double pq;      // p . q
  double alpha;
  double beta;
  double rnorm;   // ||r|| over active cells
  double rnorm0;
  double snorm;   // ||sigma|| over active cells (solver only)
  double rtol;    // 0: no stopping test (smoother)
  int it, max_it, done, status;
  double hist[GMG_MAX_HISTORY];  // ||r|| / ||sigma|| after each iteration
};

// s = diag(-A): the sum of the six faces, in the order of stencil_Ax.
template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_pcg_diag(Geom g, const TL* __restrict__ L,
                                                 T* __restrict__ s) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  walk_column_v<T, TL>(g, [](long long) { return T(0); }, L, i, j, k, k + 1,
                       [&](long long idx, T, T D, T) { s[idx] = -D; });
}

// r = A x - sigma, z = r / s, p = z on active cells (0 elsewhere); FP64
// partials of r.z (pa) and r.r (pb) per block.
template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_pcg_start(Geom g, Roles<T> X, int role,
                                                  const T* __restrict__ sigma,
                                                  const TL* __restrict__ L,
                                                  const T* __restrict__ s, T* __restrict__ r,
                                                  T* __restrict__ z, T* __restrict__ p,
                                                  double* pa, double* pb, int kchunk,
                                                  const int* done) {
  if (stopped(done)) return;
  const T* __restrict__ x = X.get(role);
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
  const int k0 = blockIdx.z * kchunk;
  double arz = 0.0, arr = 0.0;
  walk_column_vs<T, TL>(g, [&](long long q) { return x[q]; },
                        [&](long long q) { return sigma[q]; }, L, i, j, k0,
                        min(g.nz, k0 + kchunk), [&](long long idx, T ax, T D, T, T sv) {
                         const T rv = (D != T(0)) ? ax - sv : T(0);
                         const T zv = (D != T(0)) ? rv / s[idx] : T(0);
                         r[idx] = rv;
                         z[idx] = zv;
                         p[idx] = zv;
                         arz += (double)rv * (double)zv;
                         arr += (double)rv * (double)rv;
                       });
  const int tid = threadIdx.x + BX * threadIdx.y;
  const long long blk = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const double srz = block_sum(arz, tid, BT);
  __syncthreads();
  const double srr = block_sum(arr, tid, BT);
  if (tid == 0) {
    pa[blk] = srz;
    pb[blk] = srr;
  }
}

// ||sigma|| of a solve (partials from k_masked_sumsq).
__global__ __launch_bounds__(256) void k_pcg_snorm(PCGState* st, const double* ps, long long n) {
  const double ss = reduce_partials(ps, n);
  if (threadIdx.x == 0) st->snorm = sqrt(ss);
}

// Start of a run: r.z, ||r||, beta = 0, counters and the stopping test.
__global__ __launch_bounds__(256) void k_pcg_begin(PCGState* st, const double* pa,
                                                   const double* pb, long long n, double rtol,
                                                   int max_it, const int* done) {
  if (stopped(done)) return;
  const double rz = reduce_partials(pa, n);
  __syncthreads();
  const double rr = reduce_partials(pb, n);
  if (threadIdx.x != 0) return;
  st->rz = rz;
  st->beta = 0.0;
  st->alpha = 0.0;
  st->rnorm = st->rnorm0 = sqrt(rr);
  st->rtol = rtol;
  st->it = 0;
  st->max_it = max_it;
  const bool bad = !isfinite(st->snorm) || !isfinite(st->rnorm);
  const bool conv = !bad && rtol > 0.0 && st->snorm > 0.0 && st->rnorm / st->snorm <= rtol;
  const bool zero_rhs = !bad && rtol > 0.0 && st->snorm == 0.0;
  st->done = (bad || conv || zero_rhs || max_it <= 0) ? 1 : 0;
  st->status = bad ? kStNonFinite : ((conv || zero_rhs) ? GMG_OK : GMG_ENOCONV);
}

// p' = z + beta p, q = B p' = -A p' on active cells; partials of p'.q.
template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_pcg_pq(Geom g, const T* __restrict__ z,
                                               const T* __restrict__ pold, T* __restrict__ pnew,
                                               T* __restrict__ q, const TL* __restrict__ L,
                                               const PCGState* st, double* pa, int kchunk,
                                               const int* done) {
  if (stopped(done)) return;
  const T beta = (T)st->beta;
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
  const int k0 = blockIdx.z * kchunk;
  double apq = 0.0;
  walk_column_v<T, TL>(g, [&](long long c) { return z[c] + beta * pold[c]; }, L, i, j, k0,
                       min(g.nz, k0 + kchunk), [&](long long idx, T ax, T D, T pv) {
                         const T qv = (D != T(0)) ? -ax : T(0);
                         pnew[idx] = pv;
                         q[idx] = qv;
                         apq += (double)pv * (double)qv;
                       });
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double s = block_sum(apq, tid, BT);
  if (tid == 0) pa[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = s;
}

// alpha = r.z / p.q (0 on breakdown, p.q = 0).
__global__ __launch_bounds__(256) void k_pcg_alpha(PCGState* st, const double* pa, long long n,
                                                   const int* done) {
  if (stopped(done)) return;
  const double pq = reduce_partials(pa, n);
  if (threadIdx.x != 0) return;
  st->pq = pq;
  st->alpha = (pq != 0.0) ? st->rz / pq : 0.0;
}

// X[rd] = X[rs] + alpha p, r -= alpha q, z = r / s; partials of r.z and r.r.
// The z-chunks go top first: k_pcg_pq, which runs before and after this
// kernel, goes bottom first, so each kernel starts on the planes the other
// touched last, the most likely to be still in the Infinity Cache.  Partials
// keep the chunk's index, so the reductions are unchanged.
template <typename T>
__global__ __launch_bounds__(BT) void k_pcg_xr(Geom g, Roles<T> X, int rs, int rd,
                                               const T* __restrict__ p, T* __restrict__ r,
                                               T* __restrict__ z, const T* __restrict__ q,
                                               const T* __restrict__ s, const PCGState* st,
                                               double* pa, double* pb, int kchunk,
                                               const int* done) {
  if (stopped(done)) return;
  const T alpha = (T)st->alpha;
  const T* xs = X.get(rs);
  T* xd = X.get(rd);
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
  const int zb = (int)gridDim.z - 1 - (int)blockIdx.z;
  const int k0 = zb * kchunk, k1 = min(g.nz, k0 + kchunk);
  double arz = 0.0, arr = 0.0;
  if (i < g.nx && j < g.ny) {
    for (int k = k0; k < k1; ++k) {
      const long long idx = (long long)k * g.sz + (long long)j * g.sy + i;
      xd[idx] = xs[idx] + alpha * p[idx];
      const T rv = r[idx] - alpha * q[idx];
      const T sv = s[idx];
      const T zv = (sv != T(0)) ? rv / sv : T(0);
      r[idx] = rv;
      z[idx] = zv;
      arz += (double)rv * (double)zv;
      arr += (double)rv * (double)rv;
    }
  }
  const int tid = threadIdx.x + BX * threadIdx.y;
  const long long blk = ((long long)zb * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const double srz = block_sum(arz, tid, BT);
  __syncthreads();
  const double srr = block_sum(arr, tid, BT);
  if (tid == 0) {
    pa[blk] = srz;
    pb[blk] = srr;
  }
}

// beta = r.z (new) / r.z (old), ||r||, history and the stopping test.
__global__ __launch_bounds__(256) void k_pcg_next(PCGState* st, const double* pa,
                                                  const double* pb, long long n,
                                                  const int* done) {
  if (stopped(done)) return;
  const double rz = reduce_partials(pa, n);
  __syncthreads();
  const double rr = reduce_partials(pb, n);
  if (threadIdx.x != 0) return;
  st->beta = (st->rz != 0.0) ? rz / st->rz : 0.0;
  st->rz = rz;
  st->rnorm = sqrt(rr);
  const int it = st->it;
  const double rel = (st->snorm > 0.0) ? st->rnorm / st->snorm : 0.0;
  if (it < GMG_MAX_HISTORY) st->hist[it] = rel;
  st->it = it + 1;
  if (!isfinite(st->rnorm)) {
    st->done = 1;
    st->status = kStNonFinite;
  } else if (st->rtol > 0.0 && rel <= st->rtol) {
    st->done = 1;
    st->status = GMG_OK;
  } else if (st->it >= st->max_it) {
    st->done = 1;
  }
}

}  // namespace gmg
