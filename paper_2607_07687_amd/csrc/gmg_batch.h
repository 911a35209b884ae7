// Batched mixed-precision solve of many independent Poisson problems of
// uneven sizes.
//
// Every problem keeps its own handle (hierarchy, buffers, device states).  The
// batched kernels below take descriptor tables instead of a single geometry:
// one launch covers, for instance, the fused sweep of level l of every problem
// that has a level l, tile by tile.  The grid-wide levels of a V-cycle run
// depth by depth in lockstep; the levels of each problem below its tail start
// (at most tail_cells cells, down to the coarsest) run in one launch of
// k_tail_batch, one workgroup per problem, which also applies the
// coarsest-level rule (coarse_rtol) per problem.  A problem without a tail
// (a single level) smooths its coarsest level during both the descent and
// the ascent (nu_pre + nu_post = nu_coarse sweeps).  Per-problem device flags
// turn converged problems into no-ops, so one refinement step of every
// problem (max_inner cycles, the new FP64 residual and its check) is one
// recorded graph.  The host launches a graph of the set-up and the first
// steps, then replays the one-step graph with a flag read-back between
// replays until every problem has finished, or max_outer steps.  Tile
// shapes: the separate sweep's z-chunk per level shape comes from
// gmg_batch_autotune; the two-sweep pass tiles follow the fixed rule in
// batch_build_tables.
//
// Included once, at the end of gmg_lib.hip.
#pragma once

namespace gmg {

// One (problem, level) of the batch, FP32 cycle arithmetic.
template <typename TL>
struct BLevel {
  Geom g, gc;          // level and next-coarser geometry (gc = g on the coarsest)
  int cx, cy, cz;      // factor to the next level (1 on the coarsest)
  int coarsest;
  int next_tail;       // level l+1 is run by the tail, which leaves its result in x[0]
  int vec2;            // nx even: 2-wide loads in the fused sweep
  const TL* L;
  const uint8_t* active;
  float* x[3];         // roles: level 0 (e, w0, w1) with sel; coarse levels (x0, x1, x0)
  const int* sel;
  const float* sigma;  // level 0: the scaled correction rhs b; coarse: restricted rhs
  float* sigma_next;   // restriction output (level l+1)
  float* x_next0;      // level l+1 iterate role 0 (zeroed by restriction)
  float* x_next1;      // level l+1 iterate role 1 (the prolongation source is the role
                       // that level's smoothing ended on)
  const int* done;     // the problem's inner-solve flag
  const double* omega;
};

// Level-0 (outer refinement) view of one problem.
template <typename TL>
struct BOuter {
  Geom g;
  const double* L0x;    // exact FP64 faces
  const TL* L;          // stored faces (inner operator)
  const uint8_t* active;
  double* x;            // caller FP64 iterate
  const double* sigma;  // caller FP64 rhs
  double* r64;
  float* b;
  float* e[3];          // inner roles (e, w0, w1)
  double* partA;        // residual partials
  double* partB;        // scaled-rhs partials
  int npart;
  IRState* ir;
  SolveState* st;
};

struct BTile {
  int d;               // descriptor index
  int i0, j0, k0, k1;  // origin, z-range (restriction: k0 = coarse plane)
  int slot;            // partial slot (residual tiles)
};

// Fused sweep of every tile; corr_role >= 0 folds the prolongation of the
// next level's iterate role corr_role into it (not on a problem's coarsest
// level, which has no next level).
template <typename TL, int TY>
__global__ __launch_bounds__(32 * TY) void k_b_sweep(const BLevel<TL>* __restrict__ lv,
                                                     const BTile* __restrict__ tiles, int rs,
                                                     int rd, int corr_role) {
  const BTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const BLevel<TL>& d = lv[t.d];
  if (*d.done) return;
  __shared__ SweepSmem<float, TY> sm;
  const Roles<float> X{{d.x[0], d.x[1], d.x[2]}, d.sel};
  const int cr = d.next_tail ? 0 : corr_role;
  const float* xc = (corr_role >= 0 && !d.coarsest) ? (cr ? d.x_next1 : d.x_next0) : nullptr;
  const float omega = (float)(*d.omega);
  if (d.vec2) {
    SweepArgs<float, TL, TY, 2> a{d.g, X.get(rs), d.sigma, d.L, xc, d.active, d.gc,
                                  d.cx, d.cy, d.cz};
    rb_sweep_tile<float, TL, TY, 2>(sm, a, X.get(rd), t.i0, t.j0, t.k0, t.k1, omega);
  } else {
    SweepArgs<float, TL, TY, 1> a{d.g, X.get(rs), d.sigma, d.L, xc, d.active, d.gc,
                                  d.cx, d.cy, d.cz};
    rb_sweep_tile<float, TL, TY, 1>(sm, a, X.get(rd), t.i0, t.j0, t.k0, t.k1, omega);
  }
}

// Two-sweep pass of every pass tile (two sweeps of one smoothing step in one
// launch, bitwise two fused sweeps).  PROL: the first post-smoothing pass,
// folding the prolongation of the next level's iterate role corr_role; on a
// problem's coarsest level it adds nothing (the mask then reads zero, and
// the level's own iterate stands in for the coarse one).
template <typename TL, int TY, bool PROL>
__global__ __launch_bounds__(S2Cfg<TY>::NTB) void k_b_sweep2(const BLevel<TL>* __restrict__ lv,
                                                             const BTile* __restrict__ tiles,
                                                             int rs, int rd, int corr_role) {
  const BTile t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const BLevel<TL>& d = lv[t.d];
  if (*d.done) return;
  __shared__ S2Smem<float, TY> sm;
  const Roles<float> X{{d.x[0], d.x[1], d.x[2]}, d.sel};
  const float omega = (float)(*d.omega);
  const bool corr = PROL && !d.coarsest;
  const int cr = d.next_tail ? 0 : corr_role;
  const float* xc = corr ? (cr ? d.x_next1 : d.x_next0) : X.get(rs);
  const S2Args<float, TL> a{d.g,      X.get(rs),       d.sigma,         d.L,
                            xc,       d.active,        corr ? d.gc : d.g, corr ? d.cx : 1,
                            corr ? d.cy : 1, corr ? d.cz : 1, corr ? 1 : 0};
  rb_sweep2_tile<float, TL, TY, PROL>(sm, a, X.get(rd), t.i0, t.j0, t.k0, t.k1, omega);
}

template <typename TL>
__global__ __launch_bounds__(BT) void k_b_restrict(const BLevel<TL>* __restrict__ lv,
                                                   const BTile* __restrict__ tiles, int role) {
  const BTile t = tiles[blockIdx.x];
  const BLevel<TL>& d = lv[t.d];
  if (*d.done) return;
  __shared__ float rows[1][BY][BX];
  const Roles<float> X{{d.x[0], d.x[1], d.x[2]}, d.sel};
  restrict_tile<float, TL>(rows, d.g, X.get(role), d.sigma, d.L, d.gc, d.cx, d.cy, d.cz,
                           d.sigma_next, d.x_next0, t.i0, t.j0, t.k0, t.k0 + 1);
}

// Inner-cycle residual norm partials of role `role` at level 0.
template <typename TL>
__global__ __launch_bounds__(BT) void k_b_resid32(const BOuter<TL>* __restrict__ ov,
                                                  const BTile* __restrict__ tiles, int role) {
  const BTile t = tiles[blockIdx.x];
  const BOuter<TL>& o = ov[t.d];
  if (o.st->done) return;
  const Roles<float> X{{o.e[0], o.e[1], o.e[2]}, &o.st->cur};
  const double acc = residual_column<float, TL>(o.g, X.get(role), o.b, o.L, (float*)nullptr,
                                                t.i0 + threadIdx.x, t.j0 + threadIdx.y, t.k0,
                                                t.k1);
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double s = block_sum(acc, tid, BT);
  if (tid == 0) o.partA[t.slot] = s;
}

template <typename TL>
__global__ __launch_bounds__(256) void k_b_cycle_finish(const BOuter<TL>* __restrict__ ov,
                                                        OmegaRule rule, int final_role) {
  const BOuter<TL>& o = ov[blockIdx.x];
  SolveState* st = o.st;
  if (st->done) return;
  const double rr = reduce_partials(o.partA, o.npart);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(rr);
  const int c = st->cycles;
  if (c < GMG_MAX_HISTORY) {
    st->hist[c] = (st->snorm > 0.0) ? rn / st->snorm : 0.0;
    st->omegas[c] = st->omega;
  }
  st->last = rn;
  if (stop_non_finite(st, rn, c)) return;
  const int next = (st->cur + final_role) % 3;
  if (rn > st->rho) {
    st->omega = fmax(rule.omega_min, rule.theta_dec * st->omega);
    if (c < GMG_MAX_HISTORY) st->acc[c] = rule.rollback ? 0 : 1;
    if (!rule.rollback) {
      st->cur = next;
      st->rho = rn;
    }
  } else {
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

// FP64 outer residual (r64 and partials A).
template <typename TL>
__global__ __launch_bounds__(BT) void k_b_resid64(const BOuter<TL>* __restrict__ ov,
                                                  const BTile* __restrict__ tiles) {
  const BTile t = tiles[blockIdx.x];
  const BOuter<TL>& o = ov[t.d];
  if (o.ir->done) return;
  const double acc = residual_column<double, double>(o.g, o.x, o.sigma, o.L0x, o.r64,
                                                     t.i0 + threadIdx.x, t.j0 + threadIdx.y,
                                                     t.k0, t.k1);
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double s = block_sum(acc, tid, BT);
  if (tid == 0) o.partA[t.slot] = s;
}

template <typename TL>
__global__ __launch_bounds__(256) void k_b_ir_check(const BOuter<TL>* __restrict__ ov) {
  const BOuter<TL>& o = ov[blockIdx.x];
  IRState* ir = o.ir;
  if (ir->done) return;
  const double rr = reduce_partials(o.partA, o.npart);
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

template <typename TL>
__global__ __launch_bounds__(BT) void k_b_scale_cast(const BOuter<TL>* __restrict__ ov,
                                                     const BTile* __restrict__ tiles) {
  const BTile t = tiles[blockIdx.x];
  const BOuter<TL>& o = ov[t.d];
  if (o.ir->done) return;
  const double inv = 1.0 / o.ir->beta;
  const int i = t.i0 + threadIdx.x, j = t.j0 + threadIdx.y;
  double acc = 0.0;
  if (i < o.g.nx && j < o.g.ny)
    for (int k = t.k0; k < t.k1; ++k) {
      const long long idx = (long long)k * o.g.sz + (long long)j * o.g.sy + i;
      const float v = (float)(o.r64[idx] * inv);
      o.b[idx] = v;
      o.e[0][idx] = 0.0f;
      acc += (double)v * (double)v;
    }
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double s = block_sum(acc, tid, BT);
  if (tid == 0) o.partB[t.slot] = s;
}

// Inner solve of the step, to the step's inner tolerance (ir_inner_tolerance).
template <typename TL>
__global__ __launch_bounds__(256) void k_b_solve_init(const BOuter<TL>* __restrict__ ov,
                                                      int max_inner, double omega0) {
  const BOuter<TL>& o = ov[blockIdx.x];
  if (o.ir->done) return;
  const double ss = reduce_partials(o.partB, o.npart);
  if (threadIdx.x == 0) {
    const double inner_rtol = o.ir->inner_rtol;
    SolveState* st = o.st;
    st->snorm = sqrt(ss);
    st->rho = st->rho0 = st->last = sqrt(ss);  // e = 0: the residual is b
    st->omega = omega0;
    st->rtol = inner_rtol;
    st->cur = 0;
    st->cycles = 0;
    st->accepted = 0;
    st->max_cycles = max_inner;
    const bool conv = (st->snorm == 0.0) || (st->rho <= inner_rtol * st->snorm);
    st->status = conv ? 0 : 5;
    st->done = (conv || max_inner <= 0) ? 1 : 0;
  }
}

// x += beta e in FP64 (role 0 of the inner solve is the accepted correction,
// whichever buffer holds it); block 0 books the step.
template <typename TL>
__global__ __launch_bounds__(BT) void k_b_ir_update(const BOuter<TL>* __restrict__ ov,
                                                    const BTile* __restrict__ tiles) {
  const BTile t = tiles[blockIdx.x];
  const BOuter<TL>& o = ov[t.d];
  IRState* ir = o.ir;
  if (ir->done) return;
  const Roles<float> E{{o.e[0], o.e[1], o.e[2]}, &o.st->cur};
  const float* e = E.get(0);
  const double beta = ir->beta;
  const int i = t.i0 + threadIdx.x, j = t.j0 + threadIdx.y;
  if (i < o.g.nx && j < o.g.ny)
    for (int k = t.k0; k < t.k1; ++k) {
      const long long idx = (long long)k * o.g.sz + (long long)j * o.g.sy + i;
      o.x[idx] += beta * (double)e[idx];
    }
  if (t.slot == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    if (ir->outer < GMG_MAX_HISTORY) ir->inner[ir->outer] = o.st->cycles;
    ir->inner_total += o.st->cycles;
    ir->outer += 1;
  }
}

template <typename TL>
__global__ __launch_bounds__(256) void k_b_ir_init(const BOuter<TL>* __restrict__ ov, double rtol,
                                                   int max_outer, double inner_base,
                                                   double target) {
  const BOuter<TL>& o = ov[blockIdx.x];
  // partials A hold ||sigma||^2 pieces, partials B the active-cell counts
  const double ss = reduce_partials(o.partA, o.npart);
  __syncthreads();
  const double cnt = reduce_partials(o.partB, o.npart);
  if (threadIdx.x == 0) {
    IRState* ir = o.ir;
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
    o.st->done = 1;
  }
}

// ||sigma||^2 and active-cell count partials of every problem.
template <typename TL>
__global__ __launch_bounds__(BT) void k_b_norm_count(const BOuter<TL>* __restrict__ ov,
                                                     const BTile* __restrict__ tiles) {
  const BTile t = tiles[blockIdx.x];
  const BOuter<TL>& o = ov[t.d];
  const int i = t.i0 + threadIdx.x, j = t.j0 + threadIdx.y;
  double s2 = 0.0, cnt = 0.0;
  if (i < o.g.nx && j < o.g.ny)
    for (int k = t.k0; k < t.k1; ++k) {
      const long long idx = (long long)k * o.g.sz + (long long)j * o.g.sy + i;
      if (o.active[idx]) {
        s2 += o.sigma[idx] * o.sigma[idx];
        cnt += 1.0;
      }
    }
  const int tid = threadIdx.x + BX * threadIdx.y;
  const double a = block_sum(s2, tid, BT);
  __syncthreads();
  const double b = block_sum(cnt, tid, BT);
  if (tid == 0) {
    o.partA[t.slot] = a;
    o.partB[t.slot] = b;
  }
}

// *all = 1 when every problem of the batch has finished (converged or out of
// refinement steps), else 0.  One block.
template <typename TL>
__global__ __launch_bounds__(256) void k_b_all_done(const BOuter<TL>* __restrict__ ov, int n,
                                                    int* __restrict__ all) {
  __shared__ int open;
  if (threadIdx.x == 0) open = 0;
  __syncthreads();
  int mine = 0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) mine |= ov[p].ir->done ? 0 : 1;
  if (mine) atomicOr(&open, 1);
  __syncthreads();
  if (threadIdx.x == 0) *all = open ? 0 : 1;
}

}  // namespace gmg

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct gmg_batch {
  int n;
  gmg_handle** h;
  hipStream_t s;
  int depth;        // max over the problems of the levels run by grid kernels
  void* tails;      // TailArgs<float, TL>[ntail]: problems with a tail, those
                    // staged in LDS first, then those run in global memory
  int ntail;
  int ntail_lds;    // of which staged in LDS
  int tail_lds;     // dynamic LDS of k_tail_batch (the largest tail)
  int storage;      // GMG_F32 or GMG_BF16
  gmg_params p0;
  // device descriptor tables
  void* lv;                 // BLevel<TL>[] for all (problem, level)
  void* ov;                 // BOuter<TL>[n]
  BTile* sweep_tiles;       // per depth, concatenated
  BTile* pair_tiles;        // two-sweep pass tiles per depth (depths where all allow it)
  BTile* rest_tiles;
  BTile* res_tiles;         // level-0 residual / update tiles
  std::vector<int> sweep_off, sweep_cnt, rest_off, rest_cnt;
  std::vector<int> pair_off, pair_cnt, pair_ty;  // pair_cnt 0: separate sweeps
  int res_cnt;
  // captured graphs (graph: setup and first check; step: one refinement step
  // of every problem) and what they were recorded for
  CapturedSeq graph, step;
  int* all_done;    // device flag written by k_b_all_done
  int* hall_done;   // pinned host copy
  std::vector<const void*> key;
  int g_outer, g_inner;
  double g_rtol, g_inner_rtol;
};

namespace {

template <typename TL>
gmg_status batch_build_tables(gmg_batch* b) {
  using namespace gmg;
  constexpr int TY = SweepTY<float>::v;
  std::vector<BLevel<TL>> lvs;
  std::vector<BOuter<TL>> ovs;
  std::vector<std::vector<BTile>> sw(b->depth), rt(b->depth);
  std::vector<BTile> rs;
  std::vector<int> lv_index(b->n * kMaxLevels, -1);
  std::vector<TailArgs<float, TL>> tails, gtails;
  int tail_lds = 0;
  for (int p = 0; p < b->n; ++p) {
    gmg_handle* h = b->h[p];
    const int lt = h->tail;  // levels lt .. nlev-1 run in the problem's tail
    for (int l = 0; l < h->nlev; ++l) {
      const Level& L = h->lev[l];
      BLevel<TL> d;
      std::memset((void*)&d, 0, sizeof(d));
      d.g = L.g;
      const bool coarsest = (l == h->nlev - 1);
      d.gc = coarsest ? L.g : h->lev[l + 1].g;
      d.cx = coarsest ? 1 : L.c[0];
      d.cy = coarsest ? 1 : L.c[1];
      d.cz = coarsest ? 1 : L.c[2];
      d.coarsest = coarsest ? 1 : 0;
      d.next_tail = (l + 1 == lt && lt < h->nlev) ? 1 : 0;
      d.vec2 = (L.g.nx % 2 == 0) ? 1 : 0;
      d.L = (const TL*)L.L;
      d.active = L.active;
      if (l == 0) {
        d.x[0] = h->e32;
        d.x[1] = (float*)h->w[0];
        d.x[2] = (float*)h->w[1];
        d.sel = &h->st->cur;
        d.sigma = h->b32;
      } else {
        d.x[0] = (float*)L.x[0];
        d.x[1] = (float*)L.x[1];
        d.x[2] = (float*)L.x[0];
        d.sel = nullptr;
        d.sigma = (const float*)L.sigma;
      }
      d.sigma_next = coarsest ? nullptr : (float*)h->lev[l + 1].sigma;
      d.x_next0 = coarsest ? nullptr : (float*)h->lev[l + 1].x[0];
      d.x_next1 = coarsest ? nullptr : (float*)h->lev[l + 1].x[1];
      d.done = &h->st->done;
      d.omega = &h->st->omega;
      const int di = (int)lvs.size();
      lv_index[p * kMaxLevels + l] = di;
      lvs.push_back(d);
      if (l >= lt) continue;  // the tail's level: no grid tiles
      // sweep tiles
      for (int kz = 0; kz < L.g.nz; kz += L.kchunk)
        for (int ty = 0; ty < L.g.ny; ty += TY)
          for (int tx = 0; tx < L.g.nx; tx += SW_TX)
            sw[l].push_back(BTile{di, tx, ty, kz, std::min(L.g.nz, kz + L.kchunk), 0});
      // restriction tiles (fine BX x BY tiles, one coarse plane each)
      if (!coarsest)
        for (int K = 0; K < h->lev[l + 1].g.nz; ++K)
          for (int ty = 0; ty < L.g.ny; ty += BY)
            for (int tx = 0; tx < L.g.nx; tx += BX) rt[l].push_back(BTile{di, tx, ty, K, K, 0});
    }
    if (lt < h->nlev) {
      int bytes = 0;
      (h->tail_global ? gtails : tails).push_back(tail_args<float, TL>(h, lt, &h->st->done, &bytes));
      tail_lds = std::max(tail_lds, bytes);
    }
    // level-0 residual / update tiles in the same order as the single-problem grid
    const Level& L0 = h->lev[0];
    int slot = 0;
    for (int kz = 0; kz < L0.g.nz; kz += kResChunk)
      for (int ty = 0; ty < L0.g.ny; ty += BY)
        for (int tx = 0; tx < L0.g.nx; tx += BX)
          rs.push_back(BTile{p, tx, ty, kz, std::min(L0.g.nz, kz + kResChunk), slot++});
    BOuter<TL> o;
    std::memset((void*)&o, 0, sizeof(o));
    o.g = L0.g;
    o.L0x = (const double*)h->L0x;
    o.L = (const TL*)L0.L;
    o.active = L0.active;
    o.r64 = h->r64;
    o.b = h->b32;
    o.e[0] = h->e32;
    o.e[1] = (float*)h->w[0];
    o.e[2] = (float*)h->w[1];
    o.partA = h->partials;
    o.partB = h->partials + h->maxpart;
    o.npart = slot;
    o.ir = h->ir;
    o.st = h->st;
    ovs.push_back(o);
  }
  // two-sweep pass tiles, at depths where every problem that reaches the
  // depth allows passes (even nx, at most 2^28 cells; FP32 cycles and the
  // red-black smoother hold for every batch): 64 x 16 tiles at depth 0 and
  // 64 x 8 below, with z-chunks sized so that a depth's tiles fill about two
  // rounds of the CUs.  Elsewhere the depth keeps separate sweeps.
  std::vector<std::vector<BTile>> pt(b->depth);
  b->pair_ty.assign(b->depth, 0);
  if (b->p0.pair_sweeps && (b->p0.nu_pre >= 2 || b->p0.nu_post >= 2)) {
    for (int l = 0; l < b->depth; ++l) {
      const int ty = (l == 0) ? 16 : 8;
      bool ok = true;
      long long xy = 0;
      for (int p = 0; p < b->n; ++p) {
        const gmg_handle* h = b->h[p];
        if (l >= h->tail) continue;
        const Geom& g = h->lev[l].g;
        if (g.nx % 2 != 0 || g.n > S2_MAX_CELLS) ok = false;
        xy += (long long)((g.nx + S2_TX - 1) / S2_TX) * ((g.ny + ty - 1) / ty);
      }
      if (!ok || xy == 0) continue;
      const int chunks = std::max(1, (int)std::lround(2.0 * kCUs / (double)xy));
      for (int p = 0; p < b->n; ++p) {
        const gmg_handle* h = b->h[p];
        if (l >= h->tail) continue;
        const Geom& g = h->lev[l].g;
        const int di = lv_index[p * kMaxLevels + l];
        const int kc = std::min(g.nz, std::max(2, (g.nz + chunks - 1) / chunks));
        for (int kz = 0; kz < g.nz; kz += kc)
          for (int y0 = 0; y0 < g.ny; y0 += ty)
            for (int x0 = 0; x0 < g.nx; x0 += S2_TX)
              pt[l].push_back(BTile{di, x0, y0, kz, std::min(g.nz, kz + kc), 0});
      }
      // longest tiles first: problems with different nz get z-chunks of
      // different length, and the short ones then fill the last round of the
      // CUs (tiles are independent: a pass reads one role and writes another)
      std::stable_sort(pt[l].begin(), pt[l].end(), [](const BTile& u, const BTile& v) {
        return u.k1 - u.k0 > v.k1 - v.k0;
      });
      b->pair_ty[l] = ty;
    }
  }
  // flatten
  std::vector<BTile> swf, rtf, ptf;
  b->pair_off.assign(b->depth, 0);
  b->pair_cnt.assign(b->depth, 0);
  for (int l = 0; l < b->depth; ++l) {
    b->pair_off[l] = (int)ptf.size();
    b->pair_cnt[l] = (int)pt[l].size();
    ptf.insert(ptf.end(), pt[l].begin(), pt[l].end());
  }
  b->sweep_off.assign(b->depth, 0);
  b->sweep_cnt.assign(b->depth, 0);
  b->rest_off.assign(b->depth, 0);
  b->rest_cnt.assign(b->depth, 0);
  for (int l = 0; l < b->depth; ++l) {
    b->sweep_off[l] = (int)swf.size();
    b->sweep_cnt[l] = (int)sw[l].size();
    swf.insert(swf.end(), sw[l].begin(), sw[l].end());
    b->rest_off[l] = (int)rtf.size();
    b->rest_cnt[l] = (int)rt[l].size();
    rtf.insert(rtf.end(), rt[l].begin(), rt[l].end());
  }
  b->res_cnt = (int)rs.size();
  HIP_TRY(hipMalloc(&b->lv, lvs.size() * sizeof(BLevel<TL>)));
  HIP_TRY(hipMalloc(&b->ov, ovs.size() * sizeof(BOuter<TL>)));
  HIP_TRY(hipMalloc(&b->sweep_tiles, std::max<size_t>(1, swf.size()) * sizeof(BTile)));
  HIP_TRY(hipMalloc(&b->pair_tiles, std::max<size_t>(1, ptf.size()) * sizeof(BTile)));
  HIP_TRY(hipMalloc(&b->rest_tiles, std::max<size_t>(1, rtf.size()) * sizeof(BTile)));
  HIP_TRY(hipMalloc(&b->res_tiles, std::max<size_t>(1, rs.size()) * sizeof(BTile)));
  HIP_TRY(hipMemcpy(b->lv, lvs.data(), lvs.size() * sizeof(BLevel<TL>), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->ov, ovs.data(), ovs.size() * sizeof(BOuter<TL>), hipMemcpyHostToDevice));
  if (!swf.empty())
    HIP_TRY(hipMemcpy(b->sweep_tiles, swf.data(), swf.size() * sizeof(BTile), hipMemcpyHostToDevice));
  if (!rtf.empty())
    HIP_TRY(hipMemcpy(b->rest_tiles, rtf.data(), rtf.size() * sizeof(BTile), hipMemcpyHostToDevice));
  if (!ptf.empty())
    HIP_TRY(hipMemcpy(b->pair_tiles, ptf.data(), ptf.size() * sizeof(BTile), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->res_tiles, rs.data(), rs.size() * sizeof(BTile), hipMemcpyHostToDevice));
  b->ntail_lds = (int)tails.size();
  tails.insert(tails.end(), gtails.begin(), gtails.end());
  b->ntail = (int)tails.size();
  b->tail_lds = tail_lds;
  if (b->ntail) {
    HIP_TRY(hipMalloc(&b->tails, tails.size() * sizeof(TailArgs<float, TL>)));
    HIP_TRY(hipMemcpy(b->tails, tails.data(), tails.size() * sizeof(TailArgs<float, TL>),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipFuncSetAttribute((const void*)k_tail_batch<float, TL, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kTailLds));
  }
  return GMG_OK;
}

template <typename TL>
gmg_status batch_set_caller(gmg_batch* b, double* const* xs, const double* const* sigmas) {
  using namespace gmg;
  // patch the caller pointers into the outer descriptors
  std::vector<BOuter<TL>> ovs(b->n);
  HIP_TRY(hipMemcpy(ovs.data(), b->ov, b->n * sizeof(BOuter<TL>), hipMemcpyDeviceToHost));
  for (int p = 0; p < b->n; ++p) {
    ovs[p].x = xs[p];
    ovs[p].sigma = sigmas[p];
  }
  HIP_TRY(hipMemcpy(b->ov, ovs.data(), b->n * sizeof(BOuter<TL>), hipMemcpyHostToDevice));
  return GMG_OK;
}

// The two-sweep pass of depth l on every pass tile: X[rd] = sweep(sweep(X[rs])).
template <typename TL, bool PROL>
void batch_pass(const gmg_batch* b, hipStream_t s, const gmg::BLevel<TL>* lv, int l, int rs,
                int rd, int corr_role) {
  using namespace gmg;
  auto go = [&](auto tyc) {
    constexpr int TY = decltype(tyc)::value;
    hipLaunchKernelGGL((k_b_sweep2<TL, TY, PROL>), dim3(b->pair_cnt[l]), dim3(S2Cfg<TY>::NTB),
                       0, s, lv, b->pair_tiles + b->pair_off[l], rs, rd, corr_role);
  };
  if (b->pair_ty[l] == 16)
    go(std::integral_constant<int, 16>{});
  else
    go(std::integral_constant<int, 8>{});
}

// With `head`: the right-hand-side norms and active counts, the refinement
// state, the first FP64 residual and its check.  Then `steps` refinement steps
// (scale and round the residual, max_inner cycles, x += beta e, the new
// residual and its check).  With `all`, k_b_all_done writes there at the end.
template <typename TL>
gmg_status batch_enqueue_solve(gmg_batch* b, hipStream_t s, bool head, double rtol,
                               int max_outer, int steps, int max_inner, double inner_rtol,
                               int* all) {
  using namespace gmg;
  constexpr int TY = SweepTY<float>::v;
  const gmg_params& p = b->p0;
  const BLevel<TL>* lv = (const BLevel<TL>*)b->lv;
  const BOuter<TL>* ov = (const BOuter<TL>*)b->ov;
  const dim3 rblk(BX, BY, 1);
  if (head) {
    hipLaunchKernelGGL(k_b_norm_count<TL>, dim3(b->res_cnt), rblk, 0, s, ov, b->res_tiles);
    hipLaunchKernelGGL(k_b_ir_init<TL>, dim3(b->n), dim3(256), 0, s, ov, rtol, max_outer,
                       inner_rtol, p.ir_target);
    hipLaunchKernelGGL(k_b_resid64<TL>, dim3(b->res_cnt), rblk, 0, s, ov, b->res_tiles);
    hipLaunchKernelGGL(k_b_ir_check<TL>, dim3(b->n), dim3(256), 0, s, ov);
  }
  const OmegaRule rule = b->h[0]->rule;
  for (int m = 0; m < steps; ++m) {
    hipLaunchKernelGGL(k_b_scale_cast<TL>, dim3(b->res_cnt), rblk, 0, s, ov, b->res_tiles);
    hipLaunchKernelGGL(k_b_solve_init<TL>, dim3(b->n), dim3(256), 0, s, ov, max_inner, p.omega0);
    for (int c = 0; c < max_inner; ++c) {
      int role[kMaxLevels];
      // consecutive sweeps of a smoothing step run as two-sweep passes where
      // the depth has pass tiles (each pass moves the iterate one role on)
      for (int l = 0; l < b->depth; ++l) {  // descent
        int r = 0;
        for (int q = 0; q < p.nu_pre;) {
          const int rd = next_role(l, r);
          if (b->pair_cnt[l] && p.nu_pre - q >= 2) {
            batch_pass<TL, false>(b, s, lv, l, r, rd, -1);
            q += 2;
          } else {
            if (b->sweep_cnt[l])
              hipLaunchKernelGGL((k_b_sweep<TL, TY>), dim3(b->sweep_cnt[l]), dim3(32 * TY), 0, s,
                                 lv, b->sweep_tiles + b->sweep_off[l], r, rd, -1);
            q += 1;
          }
          r = rd;
        }
        role[l] = r;
        if (b->rest_cnt[l])
          hipLaunchKernelGGL(k_b_restrict<TL>, dim3(b->rest_cnt[l]), rblk, 0, s, lv,
                             b->rest_tiles + b->rest_off[l], r);
      }
      if (b->ntail_lds)
        hipLaunchKernelGGL((k_tail_batch<float, TL, false>), dim3(b->ntail_lds),
                           dim3(kTailThreads), b->tail_lds, s,
                           (const TailArgs<float, TL>*)b->tails);
      if (b->ntail > b->ntail_lds)
        hipLaunchKernelGGL((k_tail_batch<float, TL, true>), dim3(b->ntail - b->ntail_lds),
                           dim3(kTailThreads), 0, s,
                           (const TailArgs<float, TL>*)b->tails + b->ntail_lds);
      for (int l = b->depth - 1; l >= 0; --l) {  // ascent (coarsest levels finish smoothing)
        int r = role[l];
        // the prolongation source: the role level l+1's smoothing ended on
        const int cr = (l + 1 < b->depth) ? role[l + 1] : 0;
        for (int q = 0; q < p.nu_post;) {
          const int rd = next_role(l, r);
          if (b->pair_cnt[l] && p.nu_post - q >= 2) {
            if (q == 0)
              batch_pass<TL, true>(b, s, lv, l, r, rd, cr);
            else
              batch_pass<TL, false>(b, s, lv, l, r, rd, -1);
            q += 2;
          } else {
            if (b->sweep_cnt[l])
              hipLaunchKernelGGL((k_b_sweep<TL, TY>), dim3(b->sweep_cnt[l]), dim3(32 * TY), 0, s,
                                 lv, b->sweep_tiles + b->sweep_off[l], r, rd, q == 0 ? cr : -1);
            q += 1;
          }
          r = rd;
        }
        role[l] = r;
      }
      hipLaunchKernelGGL(k_b_resid32<TL>, dim3(b->res_cnt), rblk, 0, s, ov, b->res_tiles, role[0]);
      hipLaunchKernelGGL(k_b_cycle_finish<TL>, dim3(b->n), dim3(256), 0, s, ov, rule, role[0]);
    }
    hipLaunchKernelGGL(k_b_ir_update<TL>, dim3(b->res_cnt), rblk, 0, s, ov, b->res_tiles);
    hipLaunchKernelGGL(k_b_resid64<TL>, dim3(b->res_cnt), rblk, 0, s, ov, b->res_tiles);
    hipLaunchKernelGGL(k_b_ir_check<TL>, dim3(b->n), dim3(256), 0, s, ov);
  }
  if (all) hipLaunchKernelGGL(k_b_all_done<TL>, dim3(1), dim3(256), 0, s, ov, b->n, all);
  HIP_TRY(hipGetLastError());
  return GMG_OK;
}

void free_batch(gmg_batch* b) {
  if (!b) return;
  if (b->h)
    for (int p = 0; p < b->n; ++p) free_handle(b->h[p]);
  delete[] b->h;
  (void)hipFree(b->lv);
  (void)hipFree(b->ov);
  (void)hipFree(b->sweep_tiles);
  (void)hipFree(b->pair_tiles);
  (void)hipFree(b->rest_tiles);
  (void)hipFree(b->res_tiles);
  (void)hipFree(b->tails);
  if (b->graph.exec) (void)hipGraphExecDestroy(b->graph.exec);
  if (b->step.exec) (void)hipGraphExecDestroy(b->step.exec);
  (void)hipFree(b->all_done);
  (void)hipHostFree(b->hall_done);
  delete b;
}

}  // namespace

extern "C" {

gmg_status gmg_batch_setup(const gmg_params* params, const void* const* L, int32_t nprob,
                           void* stream, gmg_batch** out) {
  g_last_error.clear();
  if (!params || !L || !out || nprob <= 0) return fail(GMG_EINVAL, "bad batch arguments");
  *out = nullptr;
  const gmg_params& p0 = params[0];
  for (int p = 0; p < nprob; ++p) {
    GMG_TRY(validate(&params[p]));
    const gmg_params& q = params[p];
    if (!L[p]) return fail(GMG_EINVAL, "NULL L in batch");
    if (q.dtype != GMG_F64 || q.cycle_dtype != GMG_F32)
      return fail(GMG_EINVAL, "batch problems need dtype F64 and cycle_dtype F32");
    if (q.smoother != GMG_SMOOTH_RBGS)
      return fail(GMG_EINVAL, "the batched solve uses the red-black smoother only");
    if (q.l_storage != p0.l_storage || q.nu_pre != p0.nu_pre || q.nu_post != p0.nu_post ||
        q.nu_coarse != p0.nu_coarse || q.rollback != p0.rollback || q.omega0 != p0.omega0 ||
        q.omega_min != p0.omega_min || q.omega_max != p0.omega_max ||
        q.theta_dec != p0.theta_dec || q.theta_inc != p0.theta_inc ||
        q.coarse_rtol != p0.coarse_rtol || q.coarse_max != p0.coarse_max ||
        q.ir_target != p0.ir_target)
      return fail(GMG_EINVAL,
                  "batch problems must share storage, sweeps, the coarse rule, the omega rule "
                  "and ir_target");
  }
  gmg_batch* b = new (std::nothrow) gmg_batch();
  if (!b) return fail(GMG_ENOMEM, "host allocation failed");
  b->n = nprob;
  b->s = (hipStream_t)stream;
  b->p0 = p0;
  b->storage = p0.l_storage;
  b->h = new (std::nothrow) gmg_handle*[nprob]();
  if (!b->h) {
    delete b;
    return fail(GMG_ENOMEM, "host allocation failed");
  }
  b->depth = 0;
  for (int p = 0; p < nprob; ++p) {
    gmg_handle* h = new (std::nothrow) gmg_handle();
    if (!h) {
      free_batch(b);
      return fail(GMG_ENOMEM, "host allocation failed");
    }
    std::memset((void*)h, 0, sizeof(gmg_handle));
    b->h[p] = h;
    const gmg_status st = setup_impl(&params[p], L[p], stream, h);
    if (st != GMG_OK) {
      free_batch(b);
      return st;
    }
    if (h->tail == h->nlev && params[p].nu_coarse != params[p].nu_pre + params[p].nu_post) {
      free_batch(b);
      return fail(GMG_EINVAL, "a batch problem without a tail (a single level) needs "
                              "nu_coarse == nu_pre + nu_post");
    }
    b->depth = std::max(b->depth, h->tail);
  }
  const gmg_status st = (b->storage == GMG_BF16) ? batch_build_tables<uint16_t>(b)
                                                 : batch_build_tables<float>(b);
  if (st != GMG_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return GMG_OK;
}

gmg_status gmg_batch_autotune(gmg_batch* b, int32_t reps) {
  if (!b || reps < 1) return fail(GMG_EINVAL, "bad batch autotune arguments");
  // one timing per distinct level shape; the batched sweep uses ty = 8
  std::vector<std::array<int, 4>> done_keys;  // nx, ny, nz, kchunk
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int kcs[6] = {2, 4, 8, 16, 32, 64};
  for (int p = 0; p < b->n; ++p) {
    gmg_handle* h = b->h[p];
    for (int l = 0; l < h->nlev; ++l) {
      Level& lv = h->lev[l];
      int found = -1;
      for (size_t q = 0; q < done_keys.size(); ++q)
        if (done_keys[q][0] == lv.g.nx && done_keys[q][1] == lv.g.ny && done_keys[q][2] == lv.g.nz)
          found = (int)q;
      if (found >= 0) {
        lv.kchunk = done_keys[found][3];
        continue;
      }
      float* a = (l == 0) ? h->e32 : (float*)lv.x[0];
      float* c = (l == 0) ? (float*)h->w[0] : (float*)lv.x[1];
      const float* sg = (l == 0) ? h->b32 : (const float*)lv.sigma;
      const Roles<float> X{{a, c, a}, nullptr};
      float best = 1e30f;
      int bkc = lv.kchunk;
      for (int q = 0; q < 6; ++q) {
        const int kc = kcs[q];
        if (kc > lv.g.nz) continue;
        auto run = [&]() {
          if (b->storage == GMG_BF16)
            launch_sweep<float, uint16_t, 8>(h, l, X, 0, 1, sg, nullptr, nullptr, kc);
          else
            launch_sweep<float, float, 8>(h, l, X, 0, 1, sg, nullptr, nullptr, kc);
        };
        run();
        HIP_TRY(hipEventRecord(e0, h->s));
        for (int r = 0; r < reps; ++r) run();
        HIP_TRY(hipEventRecord(e1, h->s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          bkc = kc;
        }
      }
      lv.kchunk = bkc;
      done_keys.push_back({lv.g.nx, lv.g.ny, lv.g.nz, bkc});
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(hipGetLastError());
  // rebuild the descriptor tables with the new z-chunks; drop the graph
  (void)hipFree(b->lv);
  (void)hipFree(b->ov);
  (void)hipFree(b->sweep_tiles);
  (void)hipFree(b->pair_tiles);
  (void)hipFree(b->rest_tiles);
  (void)hipFree(b->res_tiles);
  (void)hipFree(b->tails);
  b->lv = b->ov = b->tails = nullptr;
  b->sweep_tiles = b->pair_tiles = b->rest_tiles = b->res_tiles = nullptr;
  if (b->graph.exec) {
    HIP_TRY(hipGraphExecDestroy(b->graph.exec));
    b->graph.exec = nullptr;
  }
  if (b->step.exec) {
    HIP_TRY(hipGraphExecDestroy(b->step.exec));
    b->step.exec = nullptr;
  }
  b->key.clear();
  return (b->storage == GMG_BF16) ? batch_build_tables<uint16_t>(b) : batch_build_tables<float>(b);
}

gmg_status gmg_batch_destroy(gmg_batch* b) {
  if (b) (void)hipStreamSynchronize(b->s);
  free_batch(b);
  return GMG_OK;
}

gmg_status gmg_batch_solve_ir(gmg_batch* b, double* const* x, const double* const* sigma,
                              double rtol, int32_t max_outer, int32_t max_inner,
                              double inner_rtol, gmg_ir_info* infos) {
  if (!b || !x || !sigma) return fail(GMG_EINVAL, "NULL argument");
  if (!(rtol >= 0) || max_outer < 0 || max_inner < 0 || !(inner_rtol >= 0))
    return fail(GMG_EINVAL, "bad tolerances / step counts");
  for (int p = 0; p < b->n; ++p)
    if (!x[p] || !sigma[p]) return fail(GMG_EINVAL, "NULL x / sigma in batch");
  std::vector<const void*> key;
  for (int p = 0; p < b->n; ++p) {
    key.push_back(x[p]);
    key.push_back(sigma[p]);
  }
  const bool same = b->graph.exec && key == b->key && b->g_outer == max_outer &&
                    b->g_inner == max_inner && b->g_rtol == rtol &&
                    b->g_inner_rtol == inner_rtol;
  if (!same) {
    GMG_TRY((b->storage == GMG_BF16 ? batch_set_caller<uint16_t>(b, x, sigma)
                                    : batch_set_caller<float>(b, x, sigma)));
    if (b->graph.exec) {
      HIP_TRY(hipGraphExecDestroy(b->graph.exec));
      b->graph.exec = nullptr;
    }
    if (b->step.exec) {
      HIP_TRY(hipGraphExecDestroy(b->step.exec));
      b->step.exec = nullptr;
    }
  }
  const bool bf = b->storage == GMG_BF16;
  if (b->p0.graphs) {
    if (!b->all_done) HIP_TRY(hipMalloc((void**)&b->all_done, sizeof(int)));
    if (!b->hall_done)
      HIP_TRY(hipHostMalloc((void**)&b->hall_done, sizeof(int), hipHostMallocDefault));
    if (!b->graph.exec || !b->step.exec) {
      // record the set-up and one refinement step of every problem as graphs
      gmg_handle* h0 = b->h[0];
      hipGraphExec_t ex = nullptr;
      auto rec = [&](CapturedSeq& cs, bool head, int steps) {
        return captured(h0, cs, nullptr, nullptr,
                        [&]() {
                          return bf ? batch_enqueue_solve<uint16_t>(b, h0->s, head, rtol,
                                                                    max_outer, steps, max_inner,
                                                                    inner_rtol, b->all_done)
                                    : batch_enqueue_solve<float>(b, h0->s, head, rtol, max_outer,
                                                                 steps, max_inner, inner_rtol,
                                                                 b->all_done);
                        },
                        &ex);
      };
      GMG_TRY(rec(b->graph, true, 0));
      GMG_TRY(rec(b->step, false, 1));
      b->key = key;
      b->g_outer = max_outer;
      b->g_inner = max_inner;
      b->g_rtol = rtol;
      b->g_inner_rtol = inner_rtol;
    }
    // replay the step until every problem has finished; each step graph ends
    // with the flag, and max_outer replays finish every problem regardless
    HIP_TRY(hipGraphLaunch(b->graph.exec, b->s));
    for (int m = 0;; ++m) {
      HIP_TRY(hipMemcpyAsync(b->hall_done, b->all_done, sizeof(int), hipMemcpyDeviceToHost, b->s));
      HIP_TRY(hipStreamSynchronize(b->s));
      if (*b->hall_done || m >= max_outer) break;
      HIP_TRY(hipGraphLaunch(b->step.exec, b->s));
    }
  } else {
    GMG_TRY((bf ? batch_enqueue_solve<uint16_t>(b, b->s, true, rtol, max_outer, max_outer,
                                                max_inner, inner_rtol, nullptr)
                : batch_enqueue_solve<float>(b, b->s, true, rtol, max_outer, max_outer, max_inner,
                                             inner_rtol, nullptr)));
  }
  HIP_TRY(hipStreamSynchronize(b->s));
  bool all_ok = true;
  int first_bad = -1;
  for (int p = 0; p < b->n; ++p) {
    gmg_handle* h = b->h[p];
    HIP_TRY(hipMemcpy(h->hir, h->ir, sizeof(IRState), hipMemcpyDeviceToHost));
    const IRState& r = *h->hir;
    if (r.status != 0) all_ok = false;
    if (r.status == kStNonFinite && first_bad < 0) first_bad = p;
    if (infos) {
      gmg_ir_info* info = &infos[p];
      std::memset(info, 0, sizeof(*info));
      info->status = r.status;
      info->outer = r.outer;
      info->inner_total = r.inner_total;
      info->snorm = r.snorm;
      info->rnorm = r.rnorm;
      const int nh = std::min(r.outer + 1, GMG_MAX_HISTORY);
      for (int m = 0; m < nh; ++m) info->history[m] = r.hist[m];
      for (int m = 0; m < std::min(r.outer, GMG_MAX_HISTORY); ++m)
        info->inner_cycles[m] = r.inner[m];
    }
  }
  if (first_bad >= 0)
    return fail(GMG_EINVAL, "residual norm not finite (NaN or Inf in sigma or x0) in problem " +
                                std::to_string(first_bad));
  if (!all_ok) return fail(GMG_ENOCONV, "some problems reached max_outer before rtol");
  return GMG_OK;
}

}  // extern "C"
