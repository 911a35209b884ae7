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
// Implicit-GEMM convolution forward: each wave computes 64 voxels (4 blocks
// of 16) x NB*16 output channels; K steps of 32 = 4 lanes-groups x 8
// consecutive input channels of one tap.
// ---------------------------------------------------------------------------

template <int NB>
__global__ __launch_bounds__(256) void k_conv_fwd(unet_shape s, const uint16_t* __restrict__ x,
                                                  int xld, int xoff, int cin,
                                                  const uint16_t* __restrict__ w,
                                                  const float* __restrict__ bias, int taps,
                                                  uint16_t* __restrict__ y, int yld, int yoff,
                                                  float* __restrict__ yf, int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long nvox = (long long)s.n * s.d * s.h * s.w;
  const long long vbase = (long long)blockIdx.x * 256 + wave * 64;
  const int K = taps * cin;
  const int ksteps = (K + 31) / 32;
  // Each of the lane's four voxels: its index (the host keeps voxel counts
  // below 2^31) and a mask of the taps that land inside the grid (bit t for
  // tap t in (kd, kh, kw) order; zero padding elsewhere).  A tap's neighbour
  // is then the voxel index plus an offset that is the same for every voxel.
  int vi[4];
  uint32_t vm[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
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
  auto load = [&](int ks, bf16x8 (&a)[4], bf16x8 (&b)[NB]) {
    const int k = ks * 32 + kl;
    const bool kin = k < K;
    const int kk = kin ? k : K - 8;
    const int t = (int)(((uint32_t)kk * rcin) >> 22), ci = kk - t * cin;
    const int off = (taps == 1) ? 0 : (t / 9 - 1) * hw + ((t / 3) % 3 - 1) * s.w + (t % 3 - 1);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const bool use = kin && ((vm[mb] >> t) & 1u);
      const bf16x8 v = ld8(x + (long long)(use ? vi[mb] + off : vi[mb]) * xld + xoff + ci);
      a[mb] = use ? v : zero8();
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 v = ld8(w + (long long)(nb * 16 + (lane & 15)) * K + kk);
      b[nb] = kin ? v : zero8();
    }
  };
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 a0[4], b0[NB], a1[4], b1[NB];
  load(0, a0, b0);
  for (int ks = 0; ks < ksteps; ++ks) {
    load(ks + 1 < ksteps ? ks + 1 : ks, a1, b1);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[mb], b0[nb], acc[mb][nb], 0, 0, 0);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) a0[mb] = a1[mb];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b0[nb] = b1[nb];
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = nb * 16 + (lane & 15);
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
  f32x4 acc[4][NB];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ks = 0; ks < ksteps; ++ks) {
    const int k = ks * 32 + kl;
    const bool kin = k < K;
    const int kk = kin ? k : K - 8;
    const int t = kk / CIN, ci = kk % CIN;
    const int dd = t / 9, dh = (t / 3) % 3, dw = t % 3;
    bf16x8 a[4], bb[NB];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      // the wave's voxel mb * 16 + (lane & 15): row l / TW of its rows
      const int l = mb * 16 + (lane & 15), row = l / kTW, wl = l % kTW;
      const int slot = (dd * kSH + kRW * wave + row + dh) * kSW + wl + dw;
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(tile + slot * CIN + ci);
      a[mb] = kin ? v : zero8();
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 v = ld8(w + (long long)(nb * 16 + (lane & 15)) * K + kk);
      bb[nb] = kin ? v : zero8();
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], bb[nb], acc[mb][nb], 0, 0, 0);
  }
  const long long vbase = (((long long)n0 * s.d + d0) * s.h + h0 + kRW * wave) * s.w + w0;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = nb * 16 + (lane & 15);
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
                                                    float* __restrict__ ws) {
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
  // partial dW of this chunk: ws[chunk][o][k]
  float* out = ws + (long long)blockIdx.y * COUT * K;
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = ob * 16 + 4 * (lane >> 4) + r;
      const int k = k0 + wave * 16 + (lane & 15);
      if (k < K) out[(long long)o * K + k] = acc[ob][r];
    }
}

// Per-chunk channel sums of dy (bias gradient partials): wsb[chunk][o].
__global__ __launch_bounds__(256) void k_bias_partial(unet_shape s, const uint16_t* __restrict__ dy,
                                                      int dld, int doff, int cout, long long vchunk,
                                                      float* __restrict__ wsb) {
  const long long nvox = (long long)s.n * s.d * s.h * s.w;
  const long long v0 = (long long)blockIdx.x * vchunk, v1 = min(nvox, v0 + vchunk);
  for (int o = threadIdx.x; o < cout; o += blockDim.x) {
    float acc = 0.f;
    for (long long v = v0; v < v1; ++v) acc += bf2f(dy[v * dld + doff + o]);
    wsb[(long long)blockIdx.x * cout + o] = acc;
  }
}

// out[i] = sum over chunks of ws[chunk][i] in chunk order.
__global__ void k_sum_chunks(const float* __restrict__ ws, long long n, int nchunks,
                             float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int c = 0; c < nchunks; ++c) acc += ws[(long long)c * n + i];
  out[i] = acc;
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
  const long long nv = nvox_of(s);
  const dim3 grid(nblk(nv, 256));
  hipStream_t st = (hipStream_t)stream;
  const uint16_t* xp = (const uint16_t*)x.p;
  const uint16_t* wp = (const uint16_t*)w;
  uint16_t* yp = (uint16_t*)y.p;
  // LDS-tiled form for grids with w a multiple of 64 and h of 4, or w = 32
  // and h a multiple of 8; 8 to 64 input channels and 16 to 64 output channels
  const bool t64 = s.w % 64 == 0 && s.h % 4 == 0, t32 = s.w == 32 && s.h % 8 == 0;
  if (taps == 27 && (t64 || t32) && (x.c == 8 || x.c == 16 || x.c == 32 || x.c == 64) &&
      (y.c == 16 || y.c == 32 || y.c == 64)) {
    const dim3 tg((unsigned)(nv / 256));
    auto go = [&](auto cinc, auto nbc) {
      constexpr int CIN = decltype(cinc)::value, NB = decltype(nbc)::value;
      if (t64)
        hipLaunchKernelGGL((k_conv_fwd_tile<CIN, NB, 64>), tg, dim3(256), 0, st, s, xp, x.ld,
                           x.off, wp, bias, yp, y.ld, y.off, out_f32, relu);
      else
        hipLaunchKernelGGL((k_conv_fwd_tile<CIN, NB, 32>), tg, dim3(256), 0, st, s, xp, x.ld,
                           x.off, wp, bias, yp, y.ld, y.off, out_f32, relu);
    };
    auto by_out = [&](auto cinc) {
      if (y.c == 16)
        go(cinc, std::integral_constant<int, 1>{});
      else if (y.c == 32)
        go(cinc, std::integral_constant<int, 2>{});
      else
        go(cinc, std::integral_constant<int, 4>{});
    };
    if (x.c == 8)
      by_out(std::integral_constant<int, 8>{});
    else if (x.c == 16)
      by_out(std::integral_constant<int, 16>{});
    else if (x.c == 32)
      by_out(std::integral_constant<int, 32>{});
    else
      by_out(std::integral_constant<int, 64>{});
    UHIP(hipGetLastError());
    return UNET_OK;
  }
  switch (y.c / 16) {
    case 1:
      hipLaunchKernelGGL(k_conv_fwd<1>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, wp, bias,
                         taps, yp, y.ld, y.off, out_f32, relu);
      break;
    case 2:
      hipLaunchKernelGGL(k_conv_fwd<2>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, wp, bias,
                         taps, yp, y.ld, y.off, out_f32, relu);
      break;
    case 4:
      hipLaunchKernelGGL(k_conv_fwd<4>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, wp, bias,
                         taps, yp, y.ld, y.off, out_f32, relu);
      break;
    case 8:
      hipLaunchKernelGGL(k_conv_fwd<8>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, wp, bias,
                         taps, yp, y.ld, y.off, out_f32, relu);
      break;
    default:
      return ufail(UNET_EINVAL, "output channels must be 16, 32, 64 or 128");
  }
  UHIP(hipGetLastError());
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
  const long long nv = nvox_of(s);
  const long long ch = wgrad_chunk(nv);
  const long long nc = (nv + ch - 1) / ch;
  return (size_t)(nc * ((long long)cout * cin * taps + cout)) * sizeof(float);
}

unet_status unet_conv_wgrad(unet_shape s, unet_act x, unet_act dy, int32_t taps, float* dw,
                            float* db, void* ws, void* stream) {
  if (!shape_ok(s) || !dw || !db || !ws || (taps != 27 && taps != 1))
    return ufail(UNET_EINVAL, "bad wgrad args");
  if (!act_ok(x, 8) || !act_ok(dy, 16) || dy.c > 128) return ufail(UNET_EINVAL, "bad wgrad views");
  hipStream_t st = (hipStream_t)stream;
  const long long nv = nvox_of(s);
  const long long ch = wgrad_chunk(nv);
  const int nc = (int)((nv + ch - 1) / ch);
  const int K = taps * x.c;
  float* wsw = (float*)ws;
  float* wsb = wsw + (long long)nc * dy.c * K;
  const dim3 grid((K + 63) / 64, nc);
  const uint16_t* xp = (const uint16_t*)x.p;
  const uint16_t* dp = (const uint16_t*)dy.p;
  switch (dy.c / 16) {
    case 1:
      hipLaunchKernelGGL(k_conv_wgrad<1>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, dp,
                         dy.ld, dy.off, taps, ch, wsw);
      break;
    case 2:
      hipLaunchKernelGGL(k_conv_wgrad<2>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, dp,
                         dy.ld, dy.off, taps, ch, wsw);
      break;
    case 4:
      hipLaunchKernelGGL(k_conv_wgrad<4>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, dp,
                         dy.ld, dy.off, taps, ch, wsw);
      break;
    case 8:
      hipLaunchKernelGGL(k_conv_wgrad<8>, grid, dim3(256), 0, st, s, xp, x.ld, x.off, x.c, dp,
                         dy.ld, dy.off, taps, ch, wsw);
      break;
    default:
      return ufail(UNET_EINVAL, "output channels must be 16, 32, 64 or 128");
  }
  hipLaunchKernelGGL(k_bias_partial, dim3(nc), dim3(128), 0, st, s, dp, dy.ld, dy.off, dy.c, ch, wsb);
  const long long nw = (long long)dy.c * K;
  hipLaunchKernelGGL(k_sum_chunks, dim3(nblk(nw)), dim3(256), 0, st, wsw, nw, nc, dw);
  hipLaunchKernelGGL(k_sum_chunks, dim3(nblk(dy.c)), dim3(256), 0, st, wsb, (long long)dy.c, nc, db);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_relu_bwd(unet_shape s, unet_act y, unet_act dy, unet_act out, void* stream) {
  if (!shape_ok(s) || !act_ok(y, 1) || !act_ok(dy, 1) || !act_ok(out, 1) || y.c != dy.c ||
      y.c != out.c)
    return ufail(UNET_EINVAL, "bad relu_bwd views");
  const long long n = nvox_of(s) * y.c;
  hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, nvox_of(s), y.c,
                     (const uint16_t*)y.p, y.ld, y.off, (const uint16_t*)dy.p, dy.ld, dy.off,
                     (uint16_t*)out.p, out.ld, out.off);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_pool_fwd(unet_shape f, unet_act x, unet_act y, void* stream) {
  if (!shape_ok(f) || f.d % 2 || f.h % 2 || f.w % 2 || !act_ok(x, 1) || !act_ok(y, 1) || x.c != y.c)
    return ufail(UNET_EINVAL, "bad pool args");
  const long long n = nvox_of(f) / 8 * x.c;
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
  hipLaunchKernelGGL(k_up_fwd, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, cs, x.c,
                     (const uint16_t*)x.p, x.ld, x.off, (uint16_t*)y.p, y.ld, y.off);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_up_bwd(unet_shape cs, unet_act dy, unet_act dx, void* stream) {
  if (!shape_ok(cs) || !act_ok(dy, 1) || !act_ok(dx, 1) || dx.c != dy.c)
    return ufail(UNET_EINVAL, "bad up_bwd args");
  const long long n = nvox_of(cs) * dx.c;
  hipLaunchKernelGGL(k_up_bwd, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, cs, dx.c,
                     (const uint16_t*)dy.p, dy.ld, dy.off, (uint16_t*)dx.p, dx.ld, dx.off);
  UHIP(hipGetLastError());
  return UNET_OK;
}

unet_status unet_head_fwd(unet_shape s, unet_act x, const float* w, const float* b, float* y,
                          void* stream) {
  if (!shape_ok(s) || !act_ok(x, 1) || !w || !b || !y) return ufail(UNET_EINVAL, "bad head args");
  const long long nv = nvox_of(s);
  hipLaunchKernelGGL(k_head_fwd, dim3(nblk(nv)), dim3(256), 0, (hipStream_t)stream, nv, x.c,
                     (const uint16_t*)x.p, x.ld, x.off, w, b, y);
  UHIP(hipGetLastError());
  return UNET_OK;
}

size_t unet_head_workspace(unet_shape s, int32_t cin) {
  const long long nv = nvox_of(s);
  const long long ch = wgrad_chunk(nv);
  return (size_t)((nv + ch - 1) / ch) * (cin + 1) * sizeof(float);
}

unet_status unet_head_bwd(unet_shape s, unet_act x, const float* w, const float* dy, unet_act dx,
                          float* dw, float* db, void* ws, void* stream) {
  if (!shape_ok(s) || !act_ok(x, 1) || !w || !dy || !dw || !db || !ws)
    return ufail(UNET_EINVAL, "bad head_bwd args");
  hipStream_t st = (hipStream_t)stream;
  const long long nv = nvox_of(s);
  if (dx.p) {
    if (!act_ok(dx, 1) || dx.c != x.c) return ufail(UNET_EINVAL, "bad head dx view");
    hipLaunchKernelGGL(k_head_dgrad, dim3(nblk(nv * x.c)), dim3(256), 0, st, nv, x.c, w, dy,
                       (uint16_t*)dx.p, dx.ld, dx.off);
  }
  const long long ch = wgrad_chunk(nv);
  const int nc = (int)((nv + ch - 1) / ch);
  float* wsp = (float*)ws;
  hipLaunchKernelGGL(k_head_wgrad_partial, dim3(nc), dim3(64), 0, st, nv, x.c,
                     (const uint16_t*)x.p, x.ld, x.off, dy, ch, wsp);
  // wsp[chunk][c + 1] -> dw[c] (the last column is the bias gradient)
  hipLaunchKernelGGL(k_sum_chunks, dim3(nblk(x.c)), dim3(256), 0, st, wsp, (long long)(x.c + 1),
                     nc, dw);
  hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(256), 0, st, wsp + x.c, (long long)(x.c + 1), nc, db);
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
