// Red-black sweep as two plain half-sweep launches, for levels where the
// fused sweep's plane march is latency-bound (its data fits L2 / Infinity
// Cache): W = sweep(S (+ P x_c)) as a red launch, then a black launch.  One
// thread per x-pair of a row updates the pair's cell of the launch's colour,
// reading its neighbours from global memory: the red launch reads the input
// (black cells), the black launch the red cells the red launch wrote.  The
// update is relax_cell on the same values as the fused sweep (the coarse
// correction added to every input value on active cells), so both give
// bitwise the same result.  Included by gmg_lib.hip (uses Roles, stopped and
// the 128 x 2 cell blocks).
#pragma once

namespace gmg {

template <typename T, typename TL>
__global__ __launch_bounds__(BT) void k_half_sweep(Geom g, Roles<T> X, int rs, int rd,
                                                   const T* __restrict__ sigma,
                                                   const TL* __restrict__ L,
                                                   const T* __restrict__ xc,
                                                   const uint8_t* __restrict__ active, Geom gc,
                                                   int cx, int cy, int cz, int colour,
                                                   const double* omega_p, const int* done) {
  if (stopped(done)) return;
  const int m = blockIdx.x * BX + threadIdx.x;  // x-pair of the row
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (j >= g.ny || 2 * m >= g.nx) return;
  const int i = 2 * m + ((j + k + colour) & 1);
  if (i >= g.nx) return;
  const T* S = X.get(rs);
  T* W = X.get(rd);
  const T omega = (T)(*omega_p);
  const int sx = cx >> 1, sy = cy >> 1, sz = cz >> 1;
  // input value at (ii, jj, kk): S plus the prolonged correction on active cells
  auto in = [&](int ii, int jj, int kk) -> T {
    const long long c = (long long)kk * g.sz + (long long)jj * g.sy + ii;
    T v = S[c];
    if (xc != nullptr && active[c])
      v += xc[(long long)(kk >> sz) * gc.sz + (long long)(jj >> sy) * gc.sy + (ii >> sx)];
    return v;
  };
  // neighbour value: the input (red launch) or the red result (black launch);
  // outside a wall 0
  auto nb = [&](int ii, int jj, int kk, bool inside) -> T {
    if (!inside) return T(0);
    if (colour == 0) return in(ii, jj, kk);
    return W[(long long)kk * g.sz + (long long)jj * g.sy + ii];
  };
  const bool e_in = i + 1 < g.nx || g.px, w_in = i > 0 || g.px;
  const bool n_in = j + 1 < g.ny || g.py, s_in = j > 0 || g.py;
  const bool t_in = k + 1 < g.nz || g.pz, b_in = k > 0 || g.pz;
  const int ie = (i + 1 < g.nx) ? i + 1 : 0, iw = (i > 0) ? i - 1 : g.nx - 1;
  const int jn = (j + 1 < g.ny) ? j + 1 : 0, js = (j > 0) ? j - 1 : g.ny - 1;
  const int kt = (k + 1 < g.nz) ? k + 1 : 0, kb = (k > 0) ? k - 1 : g.nz - 1;
  const long long q = (long long)k * g.sz + (long long)j * g.sy + i;
  const TL* Ly = L + g.n;
  const TL* Lz = L + 2 * g.n;
  const T lxp = e_in ? ldL<T>(L, (long long)k * g.sz + (long long)j * g.sy + ie) : T(0);
  const T lyp = n_in ? ldL<T>(Ly, (long long)k * g.sz + (long long)jn * g.sy + i) : T(0);
  const T lzp = t_in ? ldL<T>(Lz, (long long)kt * g.sz + (long long)j * g.sy + i) : T(0);
  W[q] = relax_cell<T>(in(i, j, k), nb(ie, j, k, e_in), nb(iw, j, k, w_in), nb(i, jn, k, n_in),
                       nb(i, js, k, s_in), nb(i, j, kt, t_in), nb(i, j, kb, b_in), ldL<T>(L, q), lxp,
                       ldL<T>(Ly, q), lyp, ldL<T>(Lz, q), lzp, sigma[q], omega);
}

}  // namespace gmg
