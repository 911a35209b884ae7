// libunet.so: the 3-D U-Net warm start of the GMG solver, for gfx950.
//
// C ABI and layouts: include/unet.h.  Convolutions are implicit GEMMs on the
// CDNA4 BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation):
//   forward:  M = voxels, N = output channels, K = taps * input channels;
//   dgrad:    the forward kernel on flipped, transposed weights;
//   wgrad:    M = output channels, N = taps * input channels, K = voxels, split
//             over voxel chunks into FP32 partials that a second kernel sums
//             in a fixed order (deterministic).
// Everything else (pooling, upsampling, ReLU backward, the 1x1x1 head, the
// masked MSE, Adam) is elementwise or a small reduction and HBM-bound.

#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/unet.h"

namespace {

thread_local std::string g_err;

unet_status ufail(unet_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define UHIP(expr)                                                                       \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ufail(e_ == hipErrorOutOfMemory ? UNET_ENOMEM : UNET_EHIP,                  \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                   \
  } while (0)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}
__device__ __forceinline__ bf16x8 zero8() {
  uint4 v = make_uint4(0, 0, 0, 0);
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

struct Vox {
  int n, d, h, w;
};
__device__ __forceinline__ Vox vox_of(long long v, const unet_shape& s) {
  Vox r;
  r.w = (int)(v % s.w);
  long long t = v / s.w;
  r.h = (int)(t % s.h);
  t /= s.h;
  r.d = (int)(t % s.d);
  r.n = (int)(t / s.d);
  return r;
}
__device__ __forceinline__ long long vox_index(const Vox& a, const unet_shape& s) {
  return (((long long)a.n * s.d + a.d) * s.h + a.h) * s.w + a.w;
}

// Neighbour of voxel a at tap t (27 taps in (kd, kh, kw) order, or 1 tap = a
// itself); returns -1 outside the grid (zero padding).
__device__ __forceinline__ long long tap_nbr(const Vox& a, const unet_shape& s, int taps, int t) {
  if (taps == 1) return vox_index(a, s);
  Vox b = a;
  b.d += t / 9 - 1;
  b.h += (t / 3) % 3 - 1;
  b.w += t % 3 - 1;
  if (b.d < 0 || b.d >= s.d || b.h < 0 || b.h >= s.h || b.w < 0 || b.w >= s.w) return -1;
  return vox_index(b, s);
}

// ---------------------------------------------------------------------------
// MFMA lane layout (16x16x32 BF16):
//   A[m][k]: lane l holds m = l % 16, k = 8 (l / 16) + j, j = 0..7
//   B[k][n]: lane l holds n = l % 16, k = 8 (l / 16) + j
//   D[m][n]: lane l, element r holds m = 4 (l / 16) + r, n = l % 16
// ---------------------------------------------------------------------------

__global__ void k_mfma_selfcheck(const uint16_t* A, const uint16_t* B, float* out) {
  const int l = threadIdx.x;
  uint16_t a[8], b[8];
  for (int j = 0; j < 8; ++j) {
    a[j] = A[(l % 16) * 32 + 8 * (l / 16) + j];
    b[j] = B[(8 * (l / 16) + j) * 16 + (l % 16)];
  }
  bf16x8 av, bv;
  __builtin_memcpy(&av, a, 16);
  __builtin_memcpy(&bv, b, 16);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) out[(4 * (l / 16) + r) * 16 + (l % 16)] = acc[r];
}

// ---------------------------------------------------------------------------
// Implicit-GEMM convolution forward: each wave computes 16 MB voxels (MB
// blocks of 16) x NB*16 output channels, the workgroup's output channels
// starting at 16 NB blockIdx.y; K steps of 32 = 4 lane groups x 8
// consecutive input channels of one tap.  Every output's K order is the same
// for every (MB, NB), so the split does not change a bit of the result.
// ---------------------------------------------------------------------------

template <int MB, int NB>
__global__ __launch_bounds__(256) void k_conv_fwd(unet_shape s, const uint16_t* __restrict__ x,
                                                  int xld, int xoff, int cin,
                                                  const uint16_t* __restrict__ w,
                                                  const float* __restrict__ bias, int taps,
                                                  uint16_t* __restrict__ y, int yld, int yoff,
                                                  float* __restrict__ yf, int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long nvox = (long long)s.n * s.d * s.h * s.w;
  const long long vbase = ((long long)blockIdx.x * 4 + wave) * (16 * MB);
  const int co0 = blockIdx.y * (16 * NB);  // this workgroup's output channels
  const int K = taps * cin;
  const int ksteps = (K + 31) / 32;
  // Each of the lane's four voxels: its index (the host keeps voxel counts
  // below 2^31) and a mask of the taps that land inside the grid (bit t for
  // tap t in (kd, kh, kw) order; zero padding elsewhere).  A tap's neighbour
  // is then the voxel index plus an offset that is the same for every voxel.
  int vi[MB];
  uint32_t vm[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const long long v = vbase + mb * 16 + (lane & 15);
    const bool ok = v < nvox;
    const Vox a = vox_of(ok ? v : 0, s);
    vi[mb] = ok ? (int)v : 0;
    uint32_t m = 0;
    if (taps == 1) {
      m = 1u;
    } else {
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int dd = a.d + t / 9 - 1, dh = a.h + (t / 3) % 3 - 1, dw = a.w + t % 3 - 1;
        const bool in = dd >= 0 && dd < s.d && dh >= 0 && dh < s.h && dw >= 0 && dw < s.w;
        m |= (in ? 1u : 0u) << t;
      }
    }
    vm[mb] = ok ? m : 0u;
  }
  const int hw = s.h * s.w;
  // k / cin for k < 27 cin by a multiply and shift, exact for cin <= 384
  const uint32_t rcin = ((1u << 22) + (uint32_t)cin - 1) / (uint32_t)cin;
  const int kl = 8 * (lane >> 4);
  // Operands of K step ks.  Every load is issued (at the voxel itself or
  // at a clamped k when the value is padding), and padding is zeroed after
  // the load, so that no branch sits between the loads of a step and the
  // next step's loads can be in flight while this step's MFMAs run.
  auto load = [&](int ks, bf16x8 (&a)[MB], bf16x8 (&b)[NB]) {
    const int k = ks * 32 + kl;
    const bool kin = k < K;
    const int kk = kin ? k : K - 8;
    const int t = (int)(((uint32_t)kk * rcin) >> 22), ci = kk - t * cin;
    const int off = (taps == 1) ? 0 : (t / 9 - 1) * hw + ((t / 3) % 3 - 1) * s.w + (t % 3 - 1);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const bool use = kin && ((vm[mb] >> t) & 1u);
      const bf16x8 v = ld8(x + (long long)(use ? vi[mb] + off : vi[mb]) * xld + xoff + ci);
      a[mb] = use ? v : zero8();
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 v = ld8(w + (long long)(co0 + nb * 16 + (lane & 15)) * K + kk);
      b[nb] = kin ? v : zero8();
    }
  };
  f32x4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 a0[MB], b0[NB], a1[MB], b1[NB];
  load(0, a0, b0);
  for (int ks = 0; ks < ksteps; ++ks) {
    load(ks + 1 < ksteps ? ks + 1 : ks, a1, b1);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[mb], b0[nb], acc[mb][nb], 0, 0, 0);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) a0[mb] = a1[mb];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b0[nb] = b1[nb];
  }
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = co0 + nb * 16 + (lane & 15);
      const float bb = bias ? bias[co] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long v = vbase + mb * 16 + 4 * (lane >> 4) + r;
        if (v >= nvox) continue;
        float val = acc[mb][nb][r] + bb;
        if (relu) val = fmaxf(val, 0.f);
        if (yf)
          yf[v * yld + yoff + co] = val;
        else
          y[v * yld + yoff + co] = f2bf(val);
      }
    }
}

// The 3x3x3 convolution of CIN (8 to 64) input channels on grids with w a
// multiple of 64 and h of 4 (TW = 64: output tiles of 64 (w) x 4 (h) voxels
// of one plane, one row per wave), or w = 32 and h a multiple of 8 (TW = 32:
// 32 x 8 tiles, two rows per wave, contiguous as the rows are the whole grid
// width).  The tile's input neighbourhood ((TW + 2) x (TH + 2) x 3 voxels,
// zeros outside the grid) is staged in LDS once, and every tap's A operand is
// then read from LDS instead of being gathered from global memory 27 times.
// The K steps, the operands and the MFMA order are those of k_conv_fwd, so
// the output is bitwise the same.
template <int CIN, int NB, int TW = 64>
__global__ __launch_bounds__(256) void k_conv_fwd_tile(unet_shape s,
                                                       const uint16_t* __restrict__ x, int xld,
                                                       int xoff, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       uint16_t* __restrict__ y, int yld,
                                                       int yoff, float* __restrict__ yf,
                                                       int relu) {
  static_assert(CIN == 8 || CIN == 16 || CIN == 32 || CIN == 64,
                "tiled conv: 8, 16, 32 or 64 input channels (64: 152 KB of LDS)");
  static_assert(TW == 64 || TW == 32, "tiled conv: tiles 64 or 32 wide");
  constexpr int kTW = TW, kTH = 256 / TW, kRW = 64 / TW;  // kRW: rows per wave
  constexpr int kSW = kTW + 2, kSH = kTH + 2, kSlots = 3 * kSH * kSW;
  __shared__ __align__(16) uint16_t tile[kSlots * CIN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int co0 = blockIdx.y * (16 * NB);  // this workgroup's output channels
  const int tw = s.w / kTW, th = s.h / kTH;
  int b = blockIdx.x;
  const int w0 = (b % tw) * kTW;
  b /= tw;
  const int h0 = (b % th) * kTH;
  b /= th;
  const int d0 = b % s.d, n0 = b / s.d;
  // stage the neighbourhood: 16-byte pieces of 8 channels, four loads in
  // flight per thread before their stores
  constexpr int P8 = CIN / 8, NP = kSlots * P8;
  for (int p0 = threadIdx.x; p0 < NP; p0 += 4 * 256) {
    uint4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = min(p0 + u * 256, NP - 1);
      const int slot = p / P8, c8 = p - slot * P8;
      const int sw = slot % kSW, sh = (slot / kSW) % kSH, sd = slot / (kSW * kSH);
      const int dd = d0 - 1 + sd, hh = h0 - 1 + sh, ww = w0 - 1 + sw;
      const bool in = dd >= 0 && dd < s.d && hh >= 0 && hh < s.h && ww >= 0 && ww < s.w;
      const long long vox = in ? (((long long)n0 * s.d + dd) * s.h + hh) * s.w + ww : 0;
      const uint4 g = *reinterpret_cast<const uint4*>(x + vox * xld + xoff + c8 * 8);
      v[u] = in ? g : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = p0 + u * 256;
      if (p < NP) *reinterpret_cast<uint4*>(tile + p * 8) = v[u];
    }
  }
  __syncthreads();
  constexpr int K = 27 * CIN;
  constexpr int ksteps = (K + 31) / 32;
  const int kl = 8 * (lane >> 4);
  // Operands of K step ks: A (4 voxel blocks) from the LDS tile, B (NB
  // output blocks) from the weights.  Steps past the end read step ksteps - 1
  // (never used).
  auto load_a = [&](int ks, bf16x8 (&a)[4]) {
    const int k = min(ks, ksteps - 1) * 32 + kl;
    const bool kin = k < K;
    const int kk = kin ? k : K - 8;
    const int t = kk / CIN, ci = kk % CIN;
    const int dd = t / 9, dh = (t / 3) % 3, dw = t % 3;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      // the wave's voxel mb * 16 + (lane & 15): row l / TW of its rows
      const int l = mb * 16 + (lane & 15), row = l / kTW, wl = l % kTW;
      const int slot = (dd * kSH + kRW * wave + row + dh) * kSW + wl + dw;
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(tile + slot * CIN + ci);
      a[mb] = kin ? v : zero8();
    }
  };
  auto load_b = [&](int ks, bf16x8 (&b)[NB]) {
    const int k = min(ks, ksteps - 1) * 32 + kl;
    const bool kin = k < K;
    const int kk = kin ? k : K - 8;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 v = ld8(w + (long long)(co0 + nb * 16 + (lane & 15)) * K + kk);
      b[nb] = kin ? v : zero8();
    }
  };
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // weights PF steps ahead, activations one step ahead; MFMA order as in
  // k_conv_fwd (K steps in order)
  constexpr int PF = 4;
  bf16x8 bq[PF][NB], aq[2][4];
#pragma unroll
  for (int u = 0; u < PF; ++u) load_b(u, bq[u]);
  load_a(0, aq[0]);
  for (int ks = 0; ks < ksteps; ks += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int k = ks + u;
      if (k < ksteps) {
        load_a(k + 1, aq[(u + 1) & 1]);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aq[u & 1][mb], bq[u][nb],
                                                                  acc[mb][nb], 0, 0, 0);
        load_b(k + PF, bq[u]);
      }
    }
  }
  const long long vbase = (((long long)n0 * s.d + d0) * s.h + h0 + kRW * wave) * s.w + w0;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = co0 + nb * 16 + (lane & 15);
      const float bv = bias ? bias[co] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long v = vbase + mb * 16 + 4 * (lane >> 4) + r;
        float val = acc[mb][nb][r] + bv;
        if (relu) val = fmaxf(val, 0.f);
        if (yf)
          yf[v * yld + yoff + co] = val;
        else
          y[v * yld + yoff + co] = f2bf(val);
      }
    }
}

// wflip[c][t'][o] = w[o][taps-1-t'][c]
__global__ void k_flip_weights(const uint16_t* __restrict__ w, uint16_t* __restrict__ wf, int cout,
                               int cin, int taps) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)cout * cin * taps;
  if (i >= n) return;
  const int o = (int)(i % cout);
  long long r = i / cout;
  const int tp = (int)(r % taps);
  const int c = (int)(r / taps);
  wf[((long long)c * taps + tp) * cout + o] = w[((long long)o * taps + (taps - 1 - tp)) * cin + c];
}

// ---------------------------------------------------------------------------
// Weight gradient: block = (k-tile of 64, voxel chunk); 4 waves, wave q owns
// k-block q (16 values of k) and every 16-channel output block.  Each step
// stages 32 voxels of dy (as [o][v]) and of the im2col input (as [k][v]) in
// LDS so that every MFMA operand is one 16-byte LDS read.
// ---------------------------------------------------------------------------

template <int OB>
__global__ __launch_bounds__(256) void k_conv_wgrad(unet_shape s, const uint16_t* __restrict__ x,
                                                    int xld, int xoff, int cin,
                                                    const uint16_t* __restrict__ dy, int dld,
                                                    int doff, int taps, long long vchunk,
                                                    long long rs, float* __restrict__ ws) {
  constexpr int COUT = OB * 16;
  __shared__ uint16_t sdy[COUT][40];  // [o][v], padded rows
  __shared__ uint16_t sx[64][40];     // [k][v]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int K = taps * cin;
  const int k0 = blockIdx.x * 64;
  const long long nvox = (long long)s.n * s.d * s.h * s.w;
  const long long v0 = (long long)blockIdx.y * vchunk;
  const long long v1 = min(nvox, v0 + vchunk);
  f32x4 acc[OB];
#pragma unroll
  for (int ob = 0; ob < OB; ++ob) acc[ob] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long long vs = v0; vs < v1; vs += 32) {
    // stage dy: 32 voxels x COUT channels, 8 channels per item
    for (int q = tid; q < 32 * (COUT / 8); q += 256) {
      const int vv = q / (COUT / 8), oc = (q % (COUT / 8)) * 8;
      const long long v = vs + vv;
      uint16_t buf[8];
      if (v < v1) {
        const uint4 raw = *reinterpret_cast<const uint4*>(dy + v * dld + doff + oc);
        __builtin_memcpy(buf, &raw, 16);
      } else {
        for (int e = 0; e < 8; ++e) buf[e] = 0;
      }
      for (int e = 0; e < 8; ++e) sdy[oc + e][vv] = buf[e];
    }
    // stage im2col: 32 voxels x 64 k, 8 consecutive k (one tap) per item
    for (int q = tid; q < 32 * 8; q += 256) {
      const int vv = q >> 3, kc = (q & 7) * 8;
      const long long v = vs + vv;
      const int k = k0 + kc;
      uint16_t buf[8];
      long long nb_v = -1;
      int ci = 0;
      if (v < v1 && k < K) {
        const int t = k / cin;
        ci = k - t * cin;
        nb_v = tap_nbr(vox_of(v, s), s, taps, t);
      }
      if (nb_v >= 0) {
        const uint4 raw = *reinterpret_cast<const uint4*>(x + nb_v * xld + xoff + ci);
        __builtin_memcpy(buf, &raw, 16);
      } else {
        for (int e = 0; e < 8; ++e) buf[e] = 0;
      }
      for (int e = 0; e < 8; ++e) sx[kc + e][vv] = buf[e];
    }
    __syncthreads();
    const int vl = 8 * (lane >> 4);
    bf16x8 bv;
    __builtin_memcpy(&bv, &sx[wave * 16 + (lane & 15)][vl], 16);
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      bf16x8 av;
      __builtin_memcpy(&av, &sdy[ob * 16 + (lane & 15)][vl], 16);
      acc[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ob], 0, 0, 0);
    }
    __syncthreads();
  }
  // partial dW of this chunk: ws[chunk * rs + o K + k]
  float* out = ws + (long long)blockIdx.y * rs;
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = ob * 16 + 4 * (lane >> 4) + r;
      const int k = k0 + wave * 16 + (lane & 15);
      if (k < K) out[(long long)o * K + k] = acc[ob][r];
    }
}

// Per-chunk channel sums of dy (bias gradient partials): wsb[chunk * rs + o].
__global__ __launch_bounds__(256) void k_bias_partial(unet_shape s, const uint16_t* __restrict__ dy,
                                                      int dld, int doff, int cout, long long vchunk,
                                                      long long rs, float* __restrict__ wsb) {
  const long long nvox = (long long)s.n * s.d * s.h * s.w;
  const long long v0 = (long long)blockIdx.x * vchunk, v1 = min(nvox, v0 + vchunk);
  for (int o = threadIdx.x; o < cout; o += blockDim.x) {
    float acc = 0.f;
    for (long long v = v0; v < v1; ++v) acc += bf2f(dy[v * dld + doff + o]);
    wsb[(long long)blockIdx.x * rs + o] = acc;
  }
}

// out[i] = sum over c of ws[c * n + i] (i < n), in two levels when there are
// more than 64 chunks: workgroup (64 outputs, group g) sums chunks
// [64 g, 64 g + 64), each wave 16 of them in order, the four wave sums added
// in wave order, into tmp[g * n + i]; k_sum_split then adds the groups in
// order.  The order depends only on the chunk count: deterministic.
__global__ __launch_bounds__(256) void k_sum_groups(const float* __restrict__ ws, long long n,
                                                    int nchunks, float* __restrict__ tmp) {
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long i = (long long)blockIdx.x * 64 + lane;
  const int c0 = blockIdx.y * 64 + wave * 16, c1 = min(nchunks, c0 + 16);
  float acc = 0.f;
  if (i < n)
    for (int c = c0; c < c1; ++c) acc += ws[(long long)c * n + i];
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && i < n)
    tmp[(long long)blockIdx.y * n + i] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// Sum of the nchunks rows of ws (row length n) in row order; entries below nw
// go to dw, the rest to db.
__global__ void k_sum_split(const float* __restrict__ ws, long long n, int nchunks, long long nw,
                            float* __restrict__ dw, float* __restrict__ db) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int c = 0; c < nchunks; ++c) acc += ws[(long long)c * n + i];
  if (i < nw)
    dw[i] = acc;
  else
    db[i - nw] = acc;
}

// ---------------------------------------------------------------------------
// Weight gradient, row-tiled form.  Workgroup = one voxel chunk (sample n, a
// range of d planes, a block of 4 h rows, a w segment of WS voxels) x one
// channel part (OT outputs x CT inputs).  The workgroup walks its planes in
// order.  Each input plane's rows h0-1 .. h0+4 (w0-1 .. w0+WS, zeros outside
// the grid) are staged channel-major in a 3-slot LDS ring, so that the 8
// voxels a lane feeds to the MFMA are contiguous and the three w taps of one
// (d, h) tap row come from one 16-byte and one 4-byte LDS read, shifted by 0,
// 1 or 2 elements in registers.  The plane's dy rows are staged the same way.
// A unit is 32 voxels (a row of 32, or two rows of 16).  Wave q owns one
// 16 x 16 (output, input) channel block and all 27 taps for units
// q / P, q / P + 4 / P, ... of every plane, plus the bias sums (an MFMA
// against ones) when its input block is the part's first and the part starts
// at input channel 0.  Waves that share a channel block add their sums in
// wave order at the end.  Output: the chunk's row of ws, ws[chunk * rs + ...]
// with dW at o * 27 cin + t cin + c and the bias sums at cout * 27 cin + o.
// The next plane's loads are issued before the current plane's MFMAs.
// ---------------------------------------------------------------------------

struct WgradRowsArgs {
  unet_shape s;
  const uint16_t* x;
  int xld, xoff, cin;
  const uint16_t* dy;
  int dld, doff, cout;
  int nws, nhb, nds, dper, ncp;  // w segments, 4-row blocks, d ranges, planes per range, input parts
  long long rs;                  // ws row stride (floats)
  float* ws;
};

__device__ __forceinline__ uint32_t pack_lo(uint32_t a, uint32_t b) {
  return (a & 0xFFFFu) | (b << 16);
}
__device__ __forceinline__ uint32_t pack_hi(uint32_t a, uint32_t b) {
  return (a >> 16) | (b & 0xFFFF0000u);
}
__device__ __forceinline__ bf16x8 as_bf16x8(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const uint4 v = make_uint4(a, b, c, d);
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

// Four voxels x 8 channels (one 16-byte load per voxel) written channel-major:
// row e of dst (pitch elements apart) receives the 4 voxels' channel e.
__device__ __forceinline__ void store_quad_t(uint16_t* dst, int pitch, const uint4 (&r)[4]) {
  const uint32_t v0[4] = {r[0].x, r[0].y, r[0].z, r[0].w};
  const uint32_t v1[4] = {r[1].x, r[1].y, r[1].z, r[1].w};
  const uint32_t v2[4] = {r[2].x, r[2].y, r[2].z, r[2].w};
  const uint32_t v3[4] = {r[3].x, r[3].y, r[3].z, r[3].w};
#pragma unroll
  for (int e2 = 0; e2 < 4; ++e2) {
    *reinterpret_cast<uint2*>(dst + (2 * e2) * pitch) =
        make_uint2(pack_lo(v0[e2], v1[e2]), pack_lo(v2[e2], v3[e2]));
    *reinterpret_cast<uint2*>(dst + (2 * e2 + 1) * pitch) =
        make_uint2(pack_hi(v0[e2], v1[e2]), pack_hi(v2[e2], v3[e2]));
  }
}

template <int CT, int OT, int WS>
__global__ __launch_bounds__(256, 2) void k_wgrad_rows(WgradRowsArgs a) {
  constexpr int CTP = CT < 16 ? 16 : CT;       // staged input channels (8 padded to 16)
  constexpr int NCB = CTP / 16;                // 16-channel input blocks
  constexpr int P = (OT / 16) * NCB;           // channel blocks per workgroup
  constexpr int RPW = 4 / P;                   // waves per channel block
  constexpr int RU = 32 / WS;                  // rows per 32-voxel unit
  constexpr int U = 4 / RU;                    // units per plane
  constexpr int XQ = (WS + 5) / 4;             // 4-voxel groups per staged row (WS + 2)
  constexpr int XP = WS == 32 ? 40 : 24;       // staged row pitch (elements)
  constexpr int XO = 8 * XP + 8;               // 8-channel group stride
  constexpr int XR = 2 * NCB * XO;             // one staged row, all channels
  constexpr int XPL = 6 * XR;                  // one plane slot (6 rows)
  constexpr int DP = 40, DO = 8 * DP + 8, DU = (OT / 8) * DO;
  constexpr int NX = 6 * XQ * (CT / 8);        // x staging items per plane
  constexpr int ND = 4 * (WS / 4) * (OT / 8);  // dy staging items per plane
  constexpr int SM = 3 * XPL + U * DU;         // LDS elements (ring, then dy rows)
  // the final sums pass TG taps of every wave at a time through LDS
  constexpr int TG = 4 * 9 * 4 * 64 * 4 <= SM * 2 ? 9 : (4 * 3 * 4 * 64 * 4 <= SM * 2 ? 3 : 1);
  static_assert(P >= 1 && P <= 4 && 4 % P == 0, "channel blocks per workgroup");
  static_assert(NX <= 256 && ND <= 256, "one staging item per thread");
  static_assert(4 * TG * 4 * 64 * 4 <= SM * 2, "final sums fit in LDS");
  __shared__ __align__(16) uint16_t smem[SM];
  uint16_t* const xs = smem;
  uint16_t* const ds = smem + 3 * XPL;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int D = a.s.d, H = a.s.h, W = a.s.w;
  // chunks grouped per XCD: dispatch order sends block b to XCD b % 8
  const int nchunk = gridDim.x;
  int chunk = blockIdx.x;
  if ((nchunk & 7) == 0) chunk = (blockIdx.x & 7) * (nchunk >> 3) + (blockIdx.x >> 3);
  int t = chunk;
  const int wsg = t % a.nws;
  t /= a.nws;
  const int hb = t % a.nhb;
  t /= a.nhb;
  const int dsi = t % a.nds;
  const int n = t / a.nds;
  const int c0 = (blockIdx.y % a.ncp) * CT, o0 = (blockIdx.y / a.ncp) * OT;
  const int w0 = wsg * WS, h0 = hb * 4;
  const int d0 = dsi * a.dper, d1 = min(D, d0 + a.dper);
  const long long plane = (long long)H * W;
  const long long nbase = (long long)n * D * plane;

  // staging items: x (staged row, 8-channel group, 4-voxel group), dy (row, group, 4 voxels)
  const bool xitem = tid < NX;
  const int xq = tid % XQ, xoc = (tid / XQ) % (CT / 8), xrow = tid / (XQ * (CT / 8));
  const int xh = h0 - 1 + xrow;
  const bool xrow_ok = xitem && xh >= 0 && xh < H;
  const bool ditem = tid < ND;
  const int dq = tid % (WS / 4), doc = (tid / (WS / 4)) % (OT / 8), drow = tid / ((WS / 4) * (OT / 8));
  uint4 rx[4], rd[4];
  auto load_x = [&](int p) {
    const bool ok = xrow_ok && p >= 0 && p < D;
    const long long vrow = nbase + (long long)p * plane + (long long)xh * W;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int w = w0 - 1 + 4 * xq + j;
      rx[j] = make_uint4(0, 0, 0, 0);
      if (ok && w >= 0 && w < W && 4 * xq + j < WS + 2)
        rx[j] = *reinterpret_cast<const uint4*>(a.x + (vrow + w) * a.xld + a.xoff + c0 + 8 * xoc);
    }
  };
  auto store_x = [&](int slot) {
    if (xitem) store_quad_t(xs + slot * XPL + xrow * XR + xoc * XO + 4 * xq, XP, rx);
  };
  auto load_dy = [&](int p) {
    const long long v = nbase + (long long)p * plane + (long long)(h0 + drow) * W + w0 + 4 * dq;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      rd[j] = make_uint4(0, 0, 0, 0);
      if (ditem) rd[j] = *reinterpret_cast<const uint4*>(a.dy + (v + j) * a.dld + a.doff + o0 + 8 * doc);
    }
  };
  auto store_dy = [&]() {
    if (ditem) store_quad_t(ds + (drow / RU) * DU + doc * DO + (drow % RU) * WS + 4 * dq, DP, rd);
  };

  if (CT == 8) {  // padded input channels 8..15 stay zero
    for (int i = tid; i < 3 * 6 * (XO / 8); i += 256) {
      const int sr = i / (XO / 8), off = i % (XO / 8);
      *reinterpret_cast<uint4*>(xs + sr * XR + XO + 8 * off) = make_uint4(0, 0, 0, 0);
    }
  }
  load_x(d0 - 1);
  store_x(0);
  load_x(d0);
  store_x(1);
  load_x(d0 + 1);
  store_x(2);
  load_dy(d0);
  store_dy();
  __syncthreads();
  if (d0 + 1 < d1) {
    load_x(d0 + 2);
    load_dy(d0 + 1);
  }

  const int cblk = wave % P, rsub = wave / P;
  const int ob = cblk / NCB, cb = cblk % NCB;
  const int g = lane >> 4, l16 = lane & 15;
  const int oo = ob * 16 + l16;
  const int aoff = (oo >> 3) * DO + (oo & 7) * DP + 8 * g;
  const int ci = cb * 16 + l16;
  const int boff = (ci >> 3) * XO + (ci & 7) * XP + (RU == 2 ? 8 * (g & 1) : 8 * g);
  const int grow = RU == 2 ? (g >> 1) : 0;
  const bool do_bias = cb == 0 && c0 == 0;
  const bf16x8 ones = as_bf16x8(0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u);
  f32x4 acc[27], bacc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 27; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int d = d0; d < d1; ++d) {
    for (int u = rsub; u < U; u += RPW) {
      const bf16x8 av = ld8(ds + u * DU + aoff);
      if (do_bias) bacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, ones, bacc, 0, 0, 0);
      const int lr = u * RU + grow;  // row of the 4-row block
#pragma unroll
      for (int kd = 0; kd < 3; ++kd) {
        const uint16_t* xb = xs + ((d + kd - d0) % 3) * XPL + boff + lr * XR;
#pragma unroll
        for (int kh = 0; kh < 3; ++kh) {
          const uint16_t* pb = xb + kh * XR;
          const uint4 q = *reinterpret_cast<const uint4*>(pb);
          const uint32_t q4 = *reinterpret_cast<const uint32_t*>(pb + 8);
          const int tp = 9 * kd + 3 * kh;
          acc[tp] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, as_bf16x8(q.x, q.y, q.z, q.w),
                                                            acc[tp], 0, 0, 0);
          acc[tp + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              av,
              as_bf16x8(__builtin_amdgcn_alignbit(q.y, q.x, 16), __builtin_amdgcn_alignbit(q.z, q.y, 16),
                        __builtin_amdgcn_alignbit(q.w, q.z, 16), __builtin_amdgcn_alignbit(q4, q.w, 16)),
              acc[tp + 1], 0, 0, 0);
          acc[tp + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, as_bf16x8(q.y, q.z, q.w, q4),
                                                                acc[tp + 2], 0, 0, 0);
        }
      }
    }
    if (d + 1 < d1) {
      __syncthreads();
      store_x((d + 3 - d0) % 3);  // plane d + 2 replaces plane d - 1
      store_dy();                 // plane d + 1
      __syncthreads();
      if (d + 2 < d1) {
        load_x(d + 3);
        load_dy(d + 2);
      }
    }
  }

  // Final sums: each wave parks TG taps of its tiles in LDS; the threads add
  // the RPW waves of each channel block in wave order and store the chunk's
  // row (16 consecutive input channels per lane group).
  float* const red = reinterpret_cast<float*>(smem);
  const int K = 27 * a.cin;
  float* const row = a.ws + (long long)chunk * a.rs;
#pragma unroll
  for (int grp = 0; grp < 27 / TG; ++grp) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TG; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[((wave * TG + i) * 4 + e) * 64 + lane] = acc[TG * grp + i][e];
    __syncthreads();
    for (int idx = tid; idx < P * TG * 4 * 64; idx += 256) {
      const int ln = idx & 63, e = (idx >> 6) & 3, i = (idx >> 8) % TG, cbk = (idx >> 8) / TG;
      float v = 0.f;
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) v += red[(((cbk + P * rr) * TG + i) * 4 + e) * 64 + ln];
      const int c = (cbk % NCB) * 16 + (ln & 15);
      const int o = o0 + (cbk / NCB) * 16 + 4 * (ln >> 4) + e;
      if (c < CT) row[(long long)o * K + (TG * grp + i) * a.cin + c0 + c] = v;
    }
  }
  if (c0 == 0) {  // bias sums: blocks whose input block is the first
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) red[(wave * 4 + e) * 64 + lane] = bacc[e];
    __syncthreads();
    if (tid < (OT / 16) * 16) {
      const int obk = tid >> 4, e = tid & 3, gg = (tid >> 2) & 3;
      float v = 0.f;
#pragma unroll
      for (int rr = 0; rr < RPW; ++rr) v += red[((obk * NCB + P * rr) * 4 + e) * 64 + 16 * gg];
      row[(long long)a.cout * K + o0 + obk * 16 + 4 * gg + e] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Elementwise and small kernels
// ---------------------------------------------------------------------------

__global__ void k_relu_bwd(long long nvox, int c, const uint16_t* __restrict__ y, int yld, int yoff,
                           const uint16_t* __restrict__ dy, int dld, int doff,
                           uint16_t* __restrict__ out, int old, int ooff) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  const float g = bf2f(dy[v * dld + doff + ch]);
  out[v * old + ooff + ch] = (bf2f(y[v * yld + yoff + ch]) > 0.f) ? f2bf(g) : (uint16_t)0;
}

// coarse voxel V = (n, D, H, W) of a fine grid (2D, 2H, 2W)
__global__ void k_pool_fwd(unet_shape f, int c, const uint16_t* __restrict__ x, int xld, int xoff,
                           uint16_t* __restrict__ y, int yld, int yoff) {
  unet_shape cs{f.n, f.d / 2, f.h / 2, f.w / 2};
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncv = (long long)cs.n * cs.d * cs.h * cs.w;
  if (i >= ncv * c) return;
  const long long V = i / c;
  const int ch = (int)(i - V * c);
  const Vox a = vox_of(V, cs);
  float acc = 0.f;
  for (int q = 0; q < 8; ++q) {
    const Vox b{a.n, 2 * a.d + (q >> 2), 2 * a.h + ((q >> 1) & 1), 2 * a.w + (q & 1)};
    acc += bf2f(x[vox_index(b, f) * xld + xoff + ch]);
  }
  y[V * yld + yoff + ch] = f2bf(acc * 0.125f);
}

__global__ void k_pool_bwd(unet_shape f, int c, const uint16_t* __restrict__ dy, int dld, int doff,
                           uint16_t* __restrict__ dx, int xld, int xoff, int accumulate) {
  unet_shape cs{f.n, f.d / 2, f.h / 2, f.w / 2};
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nfv = (long long)f.n * f.d * f.h * f.w;
  if (i >= nfv * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  const Vox a = vox_of(v, f);
  const Vox b{a.n, a.d / 2, a.h / 2, a.w / 2};
  float g = 0.125f * bf2f(dy[vox_index(b, cs) * dld + doff + ch]);
  if (accumulate) g += bf2f(dx[v * xld + xoff + ch]);
  dx[v * xld + xoff + ch] = f2bf(g);
}

__global__ void k_up_fwd(unet_shape cs, int c, const uint16_t* __restrict__ x, int xld, int xoff,
                         uint16_t* __restrict__ y, int yld, int yoff) {
  const unet_shape f{cs.n, 2 * cs.d, 2 * cs.h, 2 * cs.w};
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nfv = (long long)f.n * f.d * f.h * f.w;
  if (i >= nfv * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  const Vox a = vox_of(v, f);
  const Vox b{a.n, a.d / 2, a.h / 2, a.w / 2};
  y[v * yld + yoff + ch] = x[vox_index(b, cs) * xld + xoff + ch];
}

__global__ void k_up_bwd(unet_shape cs, int c, const uint16_t* __restrict__ dy, int dld, int doff,
                         uint16_t* __restrict__ dx, int xld, int xoff) {
  const unet_shape f{cs.n, 2 * cs.d, 2 * cs.h, 2 * cs.w};
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncv = (long long)cs.n * cs.d * cs.h * cs.w;
  if (i >= ncv * c) return;
  const long long V = i / c;
  const int ch = (int)(i - V * c);
  const Vox a = vox_of(V, cs);
  float acc = 0.f;
  for (int q = 0; q < 8; ++q) {
    const Vox b{a.n, 2 * a.d + (q >> 2), 2 * a.h + ((q >> 1) & 1), 2 * a.w + (q & 1)};
    acc += bf2f(dy[vox_index(b, f) * dld + doff + ch]);
  }
  dx[V * xld + xoff + ch] = f2bf(acc);
}

// 1x1x1 head to one channel: y[v] = b + sum_c w[c] x[v][c] (FP32 out).
__global__ void k_head_fwd(long long nvox, int c, const uint16_t* __restrict__ x, int xld, int xoff,
                           const float* __restrict__ w, const float* __restrict__ b,
                           float* __restrict__ y) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  float acc = 0.f;
  for (int ch = 0; ch < c; ++ch) acc += w[ch] * bf2f(x[v * xld + xoff + ch]);
  y[v] = acc + b[0];
}

// dx[v][c] = w[c] dy[v]
__global__ void k_head_dgrad(long long nvox, int c, const float* __restrict__ w,
                             const float* __restrict__ dy, uint16_t* __restrict__ dx, int xld,
                             int xoff) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  dx[v * xld + xoff + ch] = f2bf(w[ch] * dy[v]);
}

// partials of dw[c] = sum_v dy[v] x[v][c] and db = sum_v dy[v]: wsp[chunk][c+1]
__global__ __launch_bounds__(256) void k_head_wgrad_partial(long long nvox, int c,
                                                            const uint16_t* __restrict__ x, int xld,
                                                            int xoff, const float* __restrict__ dy,
                                                            long long vchunk,
                                                            float* __restrict__ wsp) {
  const long long v0 = (long long)blockIdx.x * vchunk, v1 = min(nvox, v0 + vchunk);
  for (int ch = threadIdx.x; ch <= c; ch += blockDim.x) {
    float acc = 0.f;
    for (long long v = v0; v < v1; ++v)
      acc += dy[v] * (ch < c ? bf2f(x[v * xld + xoff + ch]) : 1.f);
    wsp[(long long)blockIdx.x * (c + 1) + ch] = acc;
  }
}

// ---- 8-channel forms (16-byte accesses) for channel counts that are
// multiples of 8: one thread per (voxel, 8-channel group); the arithmetic and
// its order per element are those of the one-channel kernels above.
__device__ __forceinline__ uint4 ld16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ void st16(uint16_t* p, const uint4& v) { *reinterpret_cast<uint4*>(p) = v; }
__device__ __forceinline__ void unpack8(const uint4& r, float (&f)[8]) {
  const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    f[2 * e] = __uint_as_float(u[e] << 16);
    f[2 * e + 1] = __uint_as_float(u[e] & 0xFFFF0000u);
  }
}
__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
  uint32_t u[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) u[e] = (uint32_t)f2bf(f[2 * e]) | ((uint32_t)f2bf(f[2 * e + 1]) << 16);
  return make_uint4(u[0], u[1], u[2], u[3]);
}

__global__ void k_relu_bwd8(long long nvox, int g8, const uint16_t* __restrict__ y, int yld,
                            int yoff, const uint16_t* __restrict__ dy, int dld, int doff,
                            uint16_t* __restrict__ out, int old, int ooff) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * g8) return;
  const long long v = i / g8;
  const int c = (int)(i - v * g8) * 8;
  float fy[8];
  unpack8(ld16(y + v * yld + yoff + c), fy);
  const uint4 d = ld16(dy + v * dld + doff + c);
  const uint32_t du[4] = {d.x, d.y, d.z, d.w};
  uint32_t o[4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    o[e] = (fy[2 * e] > 0.f ? (du[e] & 0xFFFFu) : 0u) | (fy[2 * e + 1] > 0.f ? (du[e] & 0xFFFF0000u) : 0u);
  st16(out + v * old + ooff + c, make_uint4(o[0], o[1], o[2], o[3]));
}

__global__ void k_pool_fwd8(unet_shape f, int g8, const uint16_t* __restrict__ x, int xld, int xoff,
                            uint16_t* __restrict__ y, int yld, int yoff) {
  unet_shape cs{f.n, f.d / 2, f.h / 2, f.w / 2};
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncv = (long long)cs.n * cs.d * cs.h * cs.w;
  if (i >= ncv * g8) return;
  const long long V = i / g8;
  const int c = (int)(i - V * g8) * 8;
  const Vox a = vox_of(V, cs);
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int q = 0; q < 8; ++q) {
    const Vox b{a.n, 2 * a.d + (q >> 2), 2 * a.h + ((q >> 1) & 1), 2 * a.w + (q & 1)};
    float fx[8];
    unpack8(ld16(x + vox_index(b, f) * xld + xoff + c), fx);
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] += fx[e];
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) acc[e] *= 0.125f;
  st16(y + V * yld + yoff + c, pack8(acc));
}

__global__ void k_pool_bwd8(unet_shape f, int g8, const uint16_t* __restrict__ dy, int dld,
                            int doff, uint16_t* __restrict__ dx, int xld, int xoff, int accumulate) {
  unet_shape cs{f.n, f.d / 2, f.h / 2, f.w / 2};
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nfv = (long long)f.n * f.d * f.h * f.w;
  if (i >= nfv * g8) return;
  const long long v = i / g8;
  const int c = (int)(i - v * g8) * 8;
  const Vox a = vox_of(v, f);
  const Vox b{a.n, a.d / 2, a.h / 2, a.w / 2};
  float g[8];
  unpack8(ld16(dy + vox_index(b, cs) * dld + doff + c), g);
#pragma unroll
  for (int e = 0; e < 8; ++e) g[e] *= 0.125f;
  if (accumulate) {
    float o[8];
    unpack8(ld16(dx + v * xld + xoff + c), o);
#pragma unroll
    for (int e = 0; e < 8; ++e) g[e] += o[e];
  }
  st16(dx + v * xld + xoff + c, pack8(g));
}

__global__ void k_up_fwd8(unet_shape cs, int g8, const uint16_t* __restrict__ x, int xld, int xoff,
                          uint16_t* __restrict__ y, int yld, int yoff) {
  const unet_shape f{cs.n, 2 * cs.d, 2 * cs.h, 2 * cs.w};
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nfv = (long long)f.n * f.d * f.h * f.w;
  if (i >= nfv * g8) return;
  const long long v = i / g8;
  const int c = (int)(i - v * g8) * 8;
  const Vox a = vox_of(v, f);
  const Vox b{a.n, a.d / 2, a.h / 2, a.w / 2};
  st16(y + v * yld + yoff + c, ld16(x + vox_index(b, cs) * xld + xoff + c));
}

__global__ void k_up_bwd8(unet_shape cs, int g8, const uint16_t* __restrict__ dy, int dld, int doff,
                          uint16_t* __restrict__ dx, int xld, int xoff) {
  const unet_shape f{cs.n, 2 * cs.d, 2 * cs.h, 2 * cs.w};
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncv = (long long)cs.n * cs.d * cs.h * cs.w;
  if (i >= ncv * g8) return;
  const long long V = i / g8;
  const int c = (int)(i - V * g8) * 8;
  const Vox a = vox_of(V, cs);
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int q = 0; q < 8; ++q) {
    const Vox b{a.n, 2 * a.d + (q >> 2), 2 * a.h + ((q >> 1) & 1), 2 * a.w + (q & 1)};
    float g[8];
    unpack8(ld16(dy + vox_index(b, f) * dld + doff + c), g);
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] += g[e];
  }
  st16(dx + V * xld + xoff + c, pack8(acc));
}

__global__ void k_head_fwd8(long long nvox, int g8, const uint16_t* __restrict__ x, int xld,
                            int xoff, const float* __restrict__ w, const float* __restrict__ b,
                            float* __restrict__ y) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  float acc = 0.f;
  for (int g = 0; g < g8; ++g) {
    float fx[8];
    unpack8(ld16(x + v * xld + xoff + 8 * g), fx);
#pragma unroll
    for (int e = 0; e < 8; ++e) acc += w[8 * g + e] * fx[e];
  }
  y[v] = acc + b[0];
}

__global__ void k_head_dgrad8(long long nvox, int g8, const float* __restrict__ w,
                              const float* __restrict__ dy, uint16_t* __restrict__ dx, int xld,
                              int xoff) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * g8) return;
  const long long v = i / g8;
  const int c = (int)(i - v * g8) * 8;
  const float d = dy[v];
  float o[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) o[e] = w[c + e] * d;
  st16(dx + v * xld + xoff + c, pack8(o));
}

// Head weight-gradient partials, 8-channel form: workgroup = voxel chunk,
// thread (j, g) sums voxels v0 + j, v0 + j + J, ... for channels 8g..8g+7
// (g = 0 also the bias column); the J voxel lanes are then added by a fixed
// pairwise tree in LDS.  wsp[chunk][c + 1] as k_head_wgrad_partial.
__global__ __launch_bounds__(256) void k_head_wgrad8(long long nvox, int g8,
                                                     const uint16_t* __restrict__ x, int xld,
                                                     int xoff, const float* __restrict__ dy,
                                                     long long vchunk, float* __restrict__ wsp) {
  __shared__ float red[256][9];
  const int tid = threadIdx.x, J = 256 / g8;
  const int g = tid % g8, j = tid / g8;
  const long long v0 = (long long)blockIdx.x * vchunk, v1 = min(nvox, v0 + vchunk);
  float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (j < J) {
    for (long long v = v0 + j; v < v1; v += J) {
      const float d = dy[v];
      float fx[8];
      unpack8(ld16(x + v * xld + xoff + 8 * g), fx);
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] += d * fx[e];
      acc[8] += d;
    }
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) red[tid][e] = acc[e];
  __syncthreads();
  for (int st = 1; st < J; st *= 2) {
    if (j < J && j % (2 * st) == 0 && j + st < J)
#pragma unroll
      for (int e = 0; e < 9; ++e) red[tid][e] += red[tid + st * g8][e];
    __syncthreads();
  }
  if (j == 0) {
    const int c = g8 * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) wsp[(long long)blockIdx.x * (c + 1) + 8 * g + e] = red[g][e];
    if (g == 0) wsp[(long long)blockIdx.x * (c + 1) + c] = red[0][8];
  }
}

// masked MSE: per-block partial sums of the squared error and mask count,
// and the gradient 2 (pred - target) mask / count (count passed in).
__global__ __launch_bounds__(256) void k_mse_partial(long long nvox, const float* __restrict__ p,
                                                     const float* __restrict__ t,
                                                     const uint8_t* __restrict__ m,
                                                     double* __restrict__ part) {
  __shared__ double s1[256], s2[256];
  double a = 0.0, c = 0.0;
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (long long)gridDim.x * 256)
    if (m[v]) {
      const double d = (double)p[v] - (double)t[v];
      a += d * d;
      c += 1.0;
    }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ __launch_bounds__(256) void k_mse_finish(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out) {
  __shared__ double s1[256], s2[256];
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += part[2 * i];
    c += part[2 * i + 1];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double cnt = fmax(s2[0], 1.0);
    out[0] = s1[0] / cnt;
    out[1] = cnt;
  }
}

__global__ void k_mse_grad(long long nvox, const float* __restrict__ p, const float* __restrict__ t,
                           const uint8_t* __restrict__ m, const double* __restrict__ stats,
                           float* __restrict__ g) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  const double cnt = stats[1];
  g[v] = m[v] ? (float)(2.0 * ((double)p[v] - (double)t[v]) / cnt) : 0.f;
}

__global__ void k_adam(long long n, float* __restrict__ master, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ g,
                       uint16_t* __restrict__ out, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float p = master[i] - lr * mh / (sqrtf(vh) + eps);
  master[i] = p;
  if (out) out[i] = f2bf(p);
}

__global__ void k_scale(long long n, const float* __restrict__ in, float a, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * in[i];
}

__global__ void k_scale_f64(long long n, const float* __restrict__ in, double a,
                            double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * (double)in[i];
}

__global__ void k_to_bf16(long long n, const float* __restrict__ in, uint16_t* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(in[i]);
}
__global__ void k_from_bf16(long long n, const uint16_t* __restrict__ in, float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = bf2f(in[i]);
}

struct Scales {
  float s[64];
};
__global__ void k_pack_input(long long nvs, int ns, const float* __restrict__ sigma,
                             const float* __restrict__ L, Scales sc, uint16_t* __restrict__ x) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvs * ns) return;
  const int k = (int)(i / nvs);
  const long long v = i - (long long)k * nvs;
  const float* Lk = L + (long long)k * 3 * nvs;
  uint16_t row[8];
  row[0] = f2bf(sigma[i] / sc.s[k]);
  row[1] = f2bf(Lk[v]);
  row[2] = f2bf(Lk[nvs + v]);
  row[3] = f2bf(Lk[2 * nvs + v]);
  row[4] = row[5] = row[6] = row[7] = 0;
  uint4 raw;
  __builtin_memcpy(&raw, row, 16);
  *reinterpret_cast<uint4*>(x + i * 8) = raw;
}

inline unsigned nblk(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }
inline long long nvox_of(const unet_shape& s) { return (long long)s.n * s.d * s.h * s.w; }

bool act_ok(const unet_act& a, int mult) {
  return a.p && a.ld > 0 && a.c > 0 && a.off >= 0 && a.off + a.c <= a.ld && a.ld % 8 == 0 &&
         a.off % 8 == 0 && a.c % mult == 0;
}
bool shape_ok(const unet_shape& s) { return s.n > 0 && s.d > 0 && s.h > 0 && s.w > 0; }

long long wgrad_chunk(long long nvox) {
  // about 512 chunks, each a multiple of 32 voxels, at least 1024 voxels
  long long c = (nvox + 511) / 512;
  c = std::max<long long>(1024, ((c + 31) / 32) * 32);
  return c;
}


// Launch plan of the forward convolution (and of the data gradient, which is
// a forward convolution).
//   CONV_TILE:   3x3x3 taps, 8, 16, 32 or 64 input channels, 16-64 output
//                channels, w a multiple of 64 and h of 4 (64 x 4 tiles) or
//                w = 32 and h a multiple of 8 (32 x 8 tiles): LDS tiles.
//   CONV_GATHER: everything else: 64 (or 16) voxels per wave, operands
//                gathered from global memory.
// Both split the output channels over workgroups while the grid would leave
// CUs without work (tiles: until every CU has as many workgroups as its LDS
// holds).  Measured on 32^3 grids: tiles with 32 -> 64 channels 188 -> 302
// TFLOP/s, 64 -> 64 220 -> 308; gathered 16^3 grids 18-21 -> 54-88, 32^3
// with 128 channels 105-126 -> 170-180.
enum { CONV_GATHER = 0, CONV_TILE = 1 };
struct ConvPlan {
  int kind, mb, nb, tw;
  long long grid;  // workgroups per output-channel group
};

ConvPlan conv_plan(unet_shape s, int cin, int cout, int taps) {
  ConvPlan p{};
  const long long nv = (long long)s.n * s.d * s.h * s.w;
  const int ob = cout / 16;
  const bool t64 = s.w % 64 == 0 && s.h % 4 == 0, t32 = s.w == 32 && s.h % 8 == 0;
  if (taps == 27 && (t64 || t32) && ob <= 4 &&
      (cin == 8 || cin == 16 || cin == 32 || cin == 64)) {
    p.kind = CONV_TILE;
    p.tw = t64 ? 64 : 32;
    const int th = 256 / p.tw;
    const long long tiles = nv / 256;
    const long long lds = 3LL * (th + 2) * (p.tw + 2) * cin * 2;
    const long long target = 256 * std::min<long long>(4, (160 * 1024) / lds);
    p.nb = ob;
    while (p.nb > 1 && tiles * (ob / p.nb) < target) p.nb /= 2;
    p.grid = tiles;
  } else {
    // the widest output block per wave that still gives every CU a
    // workgroup, with 64 voxels per wave, else 16
    p.kind = CONV_GATHER;
    auto wgs = [&](int m, int b) { return ((nv + 64 * m - 1) / (64 * m)) * (ob / b); };
    p.mb = 4;
    p.nb = ob;
    while (p.nb > 1 && wgs(4, p.nb) < 256) p.nb /= 2;
    if (wgs(4, p.nb) < 256) {
      p.mb = 1;
      p.nb = std::min(ob, 2);
      while (p.nb > 1 && wgs(1, p.nb) < 256) p.nb /= 2;
    }
    p.grid = (nv + 64 * p.mb - 1) / (64 * p.mb);
  }
  return p;
}

// Groups of 64 chunk rows summed first when there are more than 64 rows.
long long sum_groups(long long nchunk) { return nchunk > 64 ? (nchunk + 63) / 64 : 0; }

// Fixed-order sum of nchunk partial rows ws[c * rs + i] (i < rs): entries
// below nw go to dw, the rest to db.  Groups of 64 rows first (into the
// sum_groups(nchunk) rows after the partials) when there are more.
void enq_sum_rows(float* ws, long long nchunk, long long rs, long long nw, float* dw, float* db,
                  hipStream_t st) {
  const float* rows = ws;
  long long nrows = nchunk;
  const long long ng = sum_groups(nchunk);
  if (ng > 0) {
    float* tmp = ws + nchunk * rs;
    hipLaunchKernelGGL(k_sum_groups, dim3((unsigned)((rs + 63) / 64), (unsigned)ng), dim3(256), 0,
                       st, ws, rs, (int)nchunk, tmp);
    rows = tmp;
    nrows = ng;
  }
  hipLaunchKernelGGL(k_sum_split, dim3((unsigned)((rs + 255) / 256)), dim3(256), 0, st, rows, rs,
                     (int)nrows, nw, dw, db);
}

// Launch plan of the weight gradient.  Row kernel when the grid tiles into
// 4-row blocks of 32-voxel rows (w a multiple of 32) or row pairs (w = 16),
// with 8 or a multiple of 16 input channels and 3x3x3 taps; otherwise the
// voxel-chunk kernel.  Channel parts start at 32 x 32 and are halved while the
// grid would have fewer than 512 workgroups; d ranges of at least 4 planes
// then bring it to about 1024, while the partial rows stay within 8 Mi floats.
struct WgradPlan {
  bool rows;
  int ct, ot, ws, nws, nhb, nds, dper, ncp, nop;
  long long nchunk, ngroup, rs, vchunk;
};

WgradPlan wgrad_plan(unet_shape s, int cin, int cout, int taps) {
  WgradPlan p{};
  const long long nv = (long long)s.n * s.d * s.h * s.w;
  p.rs = (long long)cout * taps * cin + cout;
  const int ws = s.w % 32 == 0 ? 32 : (s.w == 16 ? 16 : 0);
  p.rows = taps == 27 && ws > 0 && s.h % 4 == 0 && (cin == 8 || cin % 16 == 0) && cout % 16 == 0;
  if (p.rows) {
    auto blocks = [](int ot, int ct) { return (ot / 16) * (std::max(ct, 16) / 16); };
    const int pmin = ws == 16 ? 2 : 1;  // a 4-row block of w = 16 holds only 2 units
    int ot = cout % 32 == 0 ? 32 : 16;
    int ct = cin == 8 ? 8 : (cin % 32 == 0 ? 32 : 16);
    const long long cols = (long long)s.n * (s.w / ws) * (s.h / 4);
    const int maxnds = std::max(1, s.d / 4);
    for (;;) {
      const long long base = cols * (cin / ct) * (cout / ot);
      if (base * maxnds >= 512) break;
      if (ot == 32 && ot >= ct && blocks(16, ct) >= pmin)
        ot = 16;
      else if (ct == 32 && blocks(ot, 16) >= pmin)
        ct = 16;
      else
        break;
    }
    p.rows = blocks(ot, ct) >= pmin;
    if (p.rows) {
      p.ct = ct;
      p.ot = ot;
      p.ws = ws;
      p.nws = s.w / ws;
      p.nhb = s.h / 4;
      p.ncp = cin / ct;
      p.nop = cout / ot;
      const long long base = cols * p.ncp * p.nop;
      const long long want = (1024 + base - 1) / base;
      int nds = (int)std::min<long long>(maxnds, std::max<long long>(1, want));
      // partial rows beyond 8 Mi floats cost more to sum than the split gains
      while (nds > 1 && cols * nds * p.rs > (8LL << 20)) nds = (nds + 1) / 2;
      p.dper = (s.d + nds - 1) / nds;
      p.nds = (s.d + p.dper - 1) / p.dper;
      p.nchunk = cols * p.nds;
    }
  }
  if (!p.rows) {
    p.vchunk = wgrad_chunk(nv);
    p.nchunk = (nv + p.vchunk - 1) / p.vchunk;
  }
  p.ngroup = sum_groups(p.nchunk);
  return p;
}

}  // namespace

extern "C" {

const char* unet_last_error(void) { return g_err.c_str(); }

unet_status unet_mfma_selfcheck(const void* a, const void* b, float* out, void* stream) {
  if (!a || !b || !out) return ufail(UNET_EINVAL, "NULL argument");
  hipLaunchKernelGGL(k_mfma_selfcheck, dim3(1), dim3(64), 0, (hipStream_t)stream,
                     (const uint16_t*)a, (const uint16_t*)b, out);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_conv_fwd(unet_shape s, unet_act x, const void* w, const float* bias, int32_t taps,
                          unet_act y, float* out_f32, int32_t relu, void* stream) {
  if (!shape_ok(s) || !w || (taps != 27 && taps != 1)) return ufail(UNET_EINVAL, "bad conv args");
  if (!act_ok(x, 8) || x.c > 256)
    return ufail(UNET_EINVAL, "bad input view (ld/off/c multiples of 8, c <= 256)");
  if (nvox_of(s) >= (1LL << 31)) return ufail(UNET_EINVAL, "too many voxels (limit 2^31)");
  if (y.c % 16 || y.c > 128 || y.c <= 0 || y.ld % 8 || y.off % 8 || y.off + y.c > y.ld ||
      (!out_f32 && !y.p))
    return ufail(UNET_EINVAL, "bad output view (c multiple of 16, <= 128)");
  const int ob = y.c / 16;
  if (ob != 1 && ob != 2 && ob != 4 && ob != 8)
    return ufail(UNET_EINVAL, "output channels must be 16, 32, 64 or 128");
  const ConvPlan p = conv_plan(s, x.c, y.c, taps);
  hipStream_t st = (hipStream_t)stream;
  const uint16_t* xp = (const uint16_t*)x.p;
  const uint16_t* wp = (const uint16_t*)w;
  uint16_t* yp = (uint16_t*)y.p;
  const dim3 grid((unsigned)p.grid, (unsigned)(ob / p.nb));
  auto nbs = [&](auto fn) {  // NB as a compile-time constant
    switch (p.nb) {
      case 1: fn(std::integral_constant<int, 1>{}); break;
      case 2: fn(std::integral_constant<int, 2>{}); break;
      case 4: fn(std::integral_constant<int, 4>{}); break;
      default: fn(std::integral_constant<int, 8>{}); break;
    }
  };
  if (p.kind == CONV_TILE) {
    auto go = [&](auto cinc) {
      constexpr int CIN = decltype(cinc)::value;
      nbs([&](auto nbc) {
        constexpr int NB = decltype(nbc)::value;
        if constexpr (NB <= 4) {
          if (p.tw == 64)
            hipLaunchKernelGGL((k_conv_fwd_tile<CIN, NB, 64>), grid, dim3(256), 0, st, s, xp,
                               x.ld, x.off, wp, bias, yp, y.ld, y.off, out_f32, relu);
          else
            hipLaunchKernelGGL((k_conv_fwd_tile<CIN, NB, 32>), grid, dim3(256), 0, st, s, xp,
                               x.ld, x.off, wp, bias, yp, y.ld, y.off, out_f32, relu);
        }
      });
    };
    if (x.c == 8)
      go(std::integral_constant<int, 8>{});
    else if (x.c == 16)
      go(std::integral_constant<int, 16>{});
    else if (x.c == 32)
      go(std::integral_constant<int, 32>{});
    else
      go(std::integral_constant<int, 64>{});
  } else {
    nbs([&](auto nbc) {
      constexpr int NB = decltype(nbc)::value;
      if (p.mb == 4)
        hipLaunchKernelGGL((k_conv_fwd<4, NB>), grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c,
                           wp, bias, taps, yp, y.ld, y.off, out_f32, relu);
      else if constexpr (NB <= 2)
        hipLaunchKernelGGL((k_conv_fwd<1, NB>), grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c,
                           wp, bias, taps, yp, y.ld, y.off, out_f32, relu);
    });
  }
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_conv_kernel(unet_shape s, int32_t cin, int32_t cout, int32_t taps,
                             int32_t* info) {
  if (!info || !shape_ok(s) || cin <= 0 || cin % 8 || cin > 256 || (taps != 27 && taps != 1) ||
      (cout != 16 && cout != 32 && cout != 64 && cout != 128))
    return ufail(UNET_EINVAL, "bad conv_kernel args");
  const ConvPlan p = conv_plan(s, cin, cout, taps);
  info[0] = p.kind;
  info[1] = p.kind == CONV_GATHER ? p.mb : p.tw;
  info[2] = p.nb;
  info[3] = cout / 16 / p.nb;
  return UNET_OK;
}

unet_status unet_conv_dgrad(unet_shape s, unet_act dy, const void* w, int32_t taps, unet_act dx,
                            void* wflip, void* stream) {
  if (!shape_ok(s) || !w || !wflip || (taps != 27 && taps != 1))
    return ufail(UNET_EINVAL, "bad dgrad args");
  if (!act_ok(dy, 16) || !act_ok(dx, 16)) return ufail(UNET_EINVAL, "bad dgrad views");
  const long long n = (long long)dy.c * dx.c * taps;
  hipLaunchKernelGGL(k_flip_weights, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream,
                     (const uint16_t*)w, (uint16_t*)wflip, dy.c, dx.c, taps);
  UHIP(hipGetLastError());
  return unet_conv_fwd(s, dy, wflip, nullptr, taps, dx, nullptr, 0, stream);
}

size_t unet_wgrad_workspace(unet_shape s, int32_t cin, int32_t cout, int32_t taps) {
  if (!shape_ok(s) || cin <= 0 || cout <= 0 || (taps != 27 && taps != 1)) return 0;
  const WgradPlan p = wgrad_plan(s, cin, cout, taps);
  return (size_t)((p.nchunk + p.ngroup) * p.rs) * sizeof(float);
}

unet_status unet_wgrad_kernel(unet_shape s, int32_t cin, int32_t cout, int32_t taps,
                              int32_t* info) {
  if (!info || !shape_ok(s) || cin <= 0 || cin % 8 || cout <= 0 || cout % 16 || cout > 128 ||
      (taps != 27 && taps != 1))
    return ufail(UNET_EINVAL, "bad wgrad_kernel args");
  const WgradPlan p = wgrad_plan(s, cin, cout, taps);
  info[0] = p.rows ? 1 : 0;
  info[1] = p.ct;
  info[2] = p.ot;
  info[3] = p.ws;
  info[4] = (int32_t)p.nchunk;
  info[5] = p.dper;
  return UNET_OK;
}

unet_status unet_conv_wgrad(unet_shape s, unet_act x, unet_act dy, int32_t taps, float* dw,
                            float* db, void* ws, void* stream) {
  if (!shape_ok(s) || !dw || !db || !ws || (taps != 27 && taps != 1))
    return ufail(UNET_EINVAL, "bad wgrad args");
  if (!act_ok(x, 8) || !act_ok(dy, 16) || dy.c > 128) return ufail(UNET_EINVAL, "bad wgrad views");
  hipStream_t st = (hipStream_t)stream;
  const WgradPlan p = wgrad_plan(s, x.c, dy.c, taps);
  const int K = taps * x.c;
  const long long nw = (long long)dy.c * K;
  float* wsp = (float*)ws;
  const uint16_t* xp = (const uint16_t*)x.p;
  const uint16_t* dp = (const uint16_t*)dy.p;
  if (p.rows) {
    WgradRowsArgs a{s, xp, x.ld, x.off, x.c, dp, dy.ld, dy.off, dy.c,
                    p.nws, p.nhb, p.nds, p.dper, p.ncp, p.rs, wsp};
    const dim3 grid((unsigned)p.nchunk, (unsigned)(p.ncp * p.nop));
    const int key = p.ct * 10000 + p.ot * 100 + p.ws;
    switch (key) {
#define WGROWS(CT, OT, WS)                                                             \
  case CT * 10000 + OT * 100 + WS:                                                     \
    hipLaunchKernelGGL((k_wgrad_rows<CT, OT, WS>), grid, dim3(256), 0, st, a);         \
    break;
      WGROWS(8, 16, 32)
      WGROWS(8, 32, 32)
      WGROWS(16, 16, 32)
      WGROWS(16, 32, 32)
      WGROWS(32, 16, 32)
      WGROWS(32, 32, 32)
      WGROWS(8, 32, 16)
      WGROWS(16, 32, 16)
      WGROWS(32, 16, 16)
      WGROWS(32, 32, 16)
#undef WGROWS
      default:
        return ufail(UNET_EINVAL, "wgrad: no row kernel for this channel tiling");
    }
  } else {
    const dim3 grid((K + 63) / 64, (unsigned)p.nchunk);
    switch (dy.c / 16) {
      case 1:
        hipLaunchKernelGGL(k_conv_wgrad<1>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, dp,
                           dy.ld, dy.off, taps, p.vchunk, p.rs, wsp);
        break;
      case 2:
        hipLaunchKernelGGL(k_conv_wgrad<2>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, dp,
                           dy.ld, dy.off, taps, p.vchunk, p.rs, wsp);
        break;
      case 4:
        hipLaunchKernelGGL(k_conv_wgrad<4>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, dp,
                           dy.ld, dy.off, taps, p.vchunk, p.rs, wsp);
        break;
      case 8:
        hipLaunchKernelGGL(k_conv_wgrad<8>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, dp,
                           dy.ld, dy.off, taps, p.vchunk, p.rs, wsp);
        break;
      default:
        return ufail(UNET_EINVAL, "output channels must be 16, 32, 64 or 128");
    }
    hipLaunchKernelGGL(k_bias_partial, dim3((unsigned)p.nchunk), dim3(128), 0, st, s, dp, dy.ld,
                       dy.off, dy.c, p.vchunk, p.rs, wsp + nw);
  }
  UHIP(hipGetLastError());
  enq_sum_rows(wsp, p.nchunk, p.rs, nw, dw, db, st);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_relu_bwd(unet_shape s, unet_act y, unet_act dy, unet_act out, void* stream) {
  if (!shape_ok(s) || !act_ok(y, 1) || !act_ok(dy, 1) || !act_ok(out, 1) || y.c != dy.c ||
      y.c != out.c)
    return ufail(UNET_EINVAL, "bad relu_bwd views");
  const long long n = nvox_of(s) * y.c;
  if (y.c % 8 == 0)
    hipLaunchKernelGGL(k_relu_bwd8, dim3(nblk(n / 8)), dim3(256), 0, (hipStream_t)stream,
                       nvox_of(s), y.c / 8, (const uint16_t*)y.p, y.ld, y.off,
                       (const uint16_t*)dy.p, dy.ld, dy.off, (uint16_t*)out.p, out.ld, out.off);
  else
    hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, nvox_of(s),
                       y.c, (const uint16_t*)y.p, y.ld, y.off, (const uint16_t*)dy.p, dy.ld,
                       dy.off, (uint16_t*)out.p, out.ld, out.off);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_pool_fwd(unet_shape f, unet_act x, unet_act y, void* stream) {
  if (!shape_ok(f) || f.d % 2 || f.h % 2 || f.w % 2 || !act_ok(x, 1) || !act_ok(y, 1) || x.c != y.c)
    return ufail(UNET_EINVAL, "bad pool args");
  const long long n = nvox_of(f) / 8 * x.c;
  if (x.c % 8 == 0)
    hipLaunchKernelGGL(k_pool_fwd8, dim3(nblk(n / 8)), dim3(256), 0, (hipStream_t)stream, f,
                       x.c / 8, (const uint16_t*)x.p, x.ld, x.off, (uint16_t*)y.p, y.ld, y.off);
  else
    hipLaunchKernelGGL(k_pool_fwd, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, f, x.c,
                       (const uint16_t*)x.p, x.ld, x.off, (uint16_t*)y.p, y.ld, y.off);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_pool_bwd(unet_shape f, unet_act dy, unet_act dx, int32_t accumulate, void* stream) {
  if (!shape_ok(f) || f.d % 2 || f.h % 2 || f.w % 2 || !act_ok(dy, 1) || !act_ok(dx, 1) ||
      dx.c != dy.c)
    return ufail(UNET_EINVAL, "bad pool_bwd args");
  const long long n = nvox_of(f) * dx.c;
  if (dx.c % 8 == 0)
    hipLaunchKernelGGL(k_pool_bwd8, dim3(nblk(n / 8)), dim3(256), 0, (hipStream_t)stream, f,
                       dx.c / 8, (const uint16_t*)dy.p, dy.ld, dy.off, (uint16_t*)dx.p, dx.ld,
                       dx.off, accumulate);
  else
    hipLaunchKernelGGL(k_pool_bwd, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, f, dx.c,
                       (const uint16_t*)dy.p, dy.ld, dy.off, (uint16_t*)dx.p, dx.ld, dx.off,
                       accumulate);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_up_fwd(unet_shape cs, unet_act x, unet_act y, void* stream) {
  if (!shape_ok(cs) || !act_ok(x, 1) || !act_ok(y, 1) || x.c != y.c)
    return ufail(UNET_EINVAL, "bad up args");
  const long long n = nvox_of(cs) * 8 * x.c;
  if (x.c % 8 == 0)
    hipLaunchKernelGGL(k_up_fwd8, dim3(nblk(n / 8)), dim3(256), 0, (hipStream_t)stream, cs,
                       x.c / 8, (const uint16_t*)x.p, x.ld, x.off, (uint16_t*)y.p, y.ld, y.off);
  else
    hipLaunchKernelGGL(k_up_fwd, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, cs, x.c,
                       (const uint16_t*)x.p, x.ld, x.off, (uint16_t*)y.p, y.ld, y.off);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_up_bwd(unet_shape cs, unet_act dy, unet_act dx, void* stream) {
  if (!shape_ok(cs) || !act_ok(dy, 1) || !act_ok(dx, 1) || dx.c != dy.c)
    return ufail(UNET_EINVAL, "bad up_bwd args");
  const long long n = nvox_of(cs) * dx.c;
  if (dx.c % 8 == 0)
    hipLaunchKernelGGL(k_up_bwd8, dim3(nblk(n / 8)), dim3(256), 0, (hipStream_t)stream, cs,
                       dx.c / 8, (const uint16_t*)dy.p, dy.ld, dy.off, (uint16_t*)dx.p, dx.ld,
                       dx.off);
  else
    hipLaunchKernelGGL(k_up_bwd, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, cs, dx.c,
                       (const uint16_t*)dy.p, dy.ld, dy.off, (uint16_t*)dx.p, dx.ld, dx.off);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_head_fwd(unet_shape s, unet_act x, const float* w, const float* b, float* y,
                          void* stream) {
  if (!shape_ok(s) || !act_ok(x, 1) || !w || !b || !y) return ufail(UNET_EINVAL, "bad head args");
  const long long nv = nvox_of(s);
  if (x.c % 8 == 0)
    hipLaunchKernelGGL(k_head_fwd8, dim3(nblk(nv)), dim3(256), 0, (hipStream_t)stream, nv,
                       x.c / 8, (const uint16_t*)x.p, x.ld, x.off, w, b, y);
  else
    hipLaunchKernelGGL(k_head_fwd, dim3(nblk(nv)), dim3(256), 0, (hipStream_t)stream, nv, x.c,
                       (const uint16_t*)x.p, x.ld, x.off, w, b, y);
  UHIP(hipGetLastError());
  return UNET_OK;
}

size_t unet_head_workspace(unet_shape s, int32_t cin) {
  if (!shape_ok(s) || cin <= 0) return 0;
  const long long nv = nvox_of(s);
  const long long ch = wgrad_chunk(nv);
  const long long nc = (nv + ch - 1) / ch;
  return (size_t)(nc + sum_groups(nc)) * (cin + 1) * sizeof(float);
}

unet_status unet_head_bwd(unet_shape s, unet_act x, const float* w, const float* dy, unet_act dx,
                          float* dw, float* db, void* ws, void* stream) {
  if (!shape_ok(s) || !act_ok(x, 1) || !w || !dy || !dw || !db || !ws)
    return ufail(UNET_EINVAL, "bad head_bwd args");
  hipStream_t st = (hipStream_t)stream;
  const long long nv = nvox_of(s);
  const bool v8 = x.c % 8 == 0 && x.c <= 256;
  if (dx.p) {
    if (!act_ok(dx, 1) || dx.c != x.c) return ufail(UNET_EINVAL, "bad head dx view");
    if (v8)
      hipLaunchKernelGGL(k_head_dgrad8, dim3(nblk(nv * x.c / 8)), dim3(256), 0, st, nv, x.c / 8,
                         w, dy, (uint16_t*)dx.p, dx.ld, dx.off);
    else
      hipLaunchKernelGGL(k_head_dgrad, dim3(nblk(nv * x.c)), dim3(256), 0, st, nv, x.c, w, dy,
                         (uint16_t*)dx.p, dx.ld, dx.off);
  }
  const long long ch = wgrad_chunk(nv);
  const int nc = (int)((nv + ch - 1) / ch);
  float* wsp = (float*)ws;
  if (v8)
    hipLaunchKernelGGL(k_head_wgrad8, dim3(nc), dim3(256), 0, st, nv, x.c / 8,
                       (const uint16_t*)x.p, x.ld, x.off, dy, ch, wsp);
  else
    hipLaunchKernelGGL(k_head_wgrad_partial, dim3(nc), dim3(64), 0, st, nv, x.c,
                       (const uint16_t*)x.p, x.ld, x.off, dy, ch, wsp);
  // wsp[chunk][c + 1] -> dw[c] (the last column is the bias gradient)
  enq_sum_rows(wsp, nc, x.c + 1, x.c, dw, db, st);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_mse(unet_shape s, const float* pred, const float* target, const uint8_t* mask,
                     float* dpred, double* stats_dev, double* loss, void* stream) {
  if (!shape_ok(s) || !pred || !target || !mask || !dpred || !stats_dev)
    return ufail(UNET_EINVAL, "bad mse args");
  hipStream_t st = (hipStream_t)stream;
  const long long nv = nvox_of(s);
  const int nb = 256;
  double* part = stats_dev + 2;  // caller provides 2 + 2 * 256 doubles
  hipLaunchKernelGGL(k_mse_partial, dim3(nb), dim3(256), 0, st, nv, pred, target, mask, part);
  hipLaunchKernelGGL(k_mse_finish, dim3(1), dim3(256), 0, st, part, nb, stats_dev);
  hipLaunchKernelGGL(k_mse_grad, dim3(nblk(nv)), dim3(256), 0, st, nv, pred, target, mask,
                     stats_dev, dpred);
  UHIP(hipGetLastError());
  if (loss) {
    UHIP(hipMemcpyAsync(loss, stats_dev, sizeof(double), hipMemcpyDeviceToHost, st));
    UHIP(hipStreamSynchronize(st));
  }
  return UNET_OK;
}

unet_status unet_adam(int64_t n, float* master, float* m, float* v, const float* g, void* bf16_out,
                      float lr, float beta1, float beta2, float eps, int32_t t, void* stream) {
  if (n <= 0 || !master || !m || !v || !g || t < 1) return ufail(UNET_EINVAL, "bad adam args");
  const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, (long long)n, master,
                     m, v, g, (uint16_t*)bf16_out, lr, beta1, beta2, eps, c1, c2);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_scale(int64_t n, const float* in, float a, float* out, void* stream) {
  if (n <= 0 || !in || !out) return ufail(UNET_EINVAL, "bad args");
  hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, (long long)n, in, a,
                     out);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_scale_f64(int64_t n, const float* in, double a, double* out, void* stream) {
  if (n <= 0 || !in || !out) return ufail(UNET_EINVAL, "bad args");
  hipLaunchKernelGGL(k_scale_f64, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, (long long)n,
                     in, a, out);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_to_bf16(int64_t n, const float* in, void* out, void* stream) {
  if (n <= 0 || !in || !out) return ufail(UNET_EINVAL, "bad args");
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, (long long)n, in,
                     (uint16_t*)out);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_from_bf16(int64_t n, const void* in, float* out, void* stream) {
  if (n <= 0 || !in || !out) return ufail(UNET_EINVAL, "bad args");
  hipLaunchKernelGGL(k_from_bf16, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, (long long)n,
                     (const uint16_t*)in, out);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_pack_input(unet_shape s, const float* sigma, const float* L, const float* scale,
                            void* x, void* stream) {
  if (!shape_ok(s) || !sigma || !L || !scale || !x || s.n > 64)
    return ufail(UNET_EINVAL, "bad pack args (at most 64 samples)");
  Scales sc;
  for (int k = 0; k < s.n; ++k) sc.s[k] = scale[k] > 0.f ? scale[k] : 1.f;
  const long long nvs = (long long)s.d * s.h * s.w;
  hipLaunchKernelGGL(k_pack_input, dim3(nblk(nvs * s.n)), dim3(256), 0, (hipStream_t)stream, nvs,
                     s.n, sigma, L, sc, (uint16_t*)x);
  UHIP(hipGetLastError());
  return UNET_OK;
}

}  // extern "C"
