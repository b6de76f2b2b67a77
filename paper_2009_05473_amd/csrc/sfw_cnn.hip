// The proposal network: four 3x3x3 convolutions with 32 channels (the first of stride 2, ReLU
// between) that read the certificate-scaled adjoint x = Phi^T r / lambda and predict, on the
// half-resolution grid, a centre heatmap logit and the sigma and d of the next atom (step 1 of
// Algorithms 1 and 2 takes the grid maximum instead; the network is a proposal that the
// certificate then accepts or rejects). Training and inference run on these kernels only.
//
// Layouts: activations bf16 channels-last [z][y][x][C] (C = 32; the gradient of the output
// layer has 16 channels, 3 used); the output layer f32 [z][y][x][4] (heatmap logit, sigma, d,
// unused). Master parameters f32 in the layout [co][ci][tz][ty][tx] then biases, layer after
// layer. For the matrix cores each layer keeps bf16 copies: forward [27][Co][Ci] (tap, output
// channel, input channel; the first layer [32][32] with the 27 taps as K, padded), backward
// [27][Ci][Co] with the taps flipped (the data gradient of a stride-1 layer is the
// convolution of the output gradient with the flipped, transposed kernel).
//
// Convolutions are implicit GEMMs on the matrix cores: a wave owns 64 consecutive output voxels
// along x (M, four tiles) and 16 or 32 output channels (N, one or two tiles); K runs over the
// taps and the input channels, 32 at a time on gfx950's 16x16x32 bf16 MFMA (16 where the input
// has 16 channels). Activations are staged in LDS per block, weights read through the caches.
// Weight gradients are float32 VALU sums over voxel chunks staged in LDS, then a fixed-order
// sum over chunks.
#include <hip/hip_runtime.h>

#include <limits>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "sfw.h"
#include "sfw_internal.h"
#include "sfw_ops.h"

namespace sfw {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kNetC = 32;       // hidden channels
constexpr int kNetOut = 3;      // heatmap logit, sigma, d
constexpr int kNetOutPad = 16;  // output-layer channels as the matrix cores see them
constexpr int kNetMaxAtoms = 96;

// parameter counts per layer (weights, then biases) in the master layout
constexpr int kW1 = kNetC * 1 * 27, kW2 = kNetC * kNetC * 27, kW4 = kNetOut * kNetC * 27;
constexpr int kOff1 = 0, kOff2 = kOff1 + kW1 + kNetC, kOff3 = kOff2 + kW2 + kNetC;
constexpr int kOff4 = kOff3 + kW2 + kNetC, kNetParams = kOff4 + kW4 + kNetOut;

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// four bf16 (two packed words, lower half first) as float32
__device__ __forceinline__ float4 bf4(uint32_t lo, uint32_t hi) {
  return make_float4(__uint_as_float(lo << 16), __uint_as_float(lo & 0xffff0000u),
                     __uint_as_float(hi << 16), __uint_as_float(hi & 0xffff0000u));
}

// ---------------------------------------------------------------- convolutions

// One MFMA step of K = 16 (v_mfma_f32_16x16x16bf16_1k, 4 bf16 per lane) or K = 32 (gfx950's
// v_mfma_f32_16x16x32_bf16, 8 per lane). Lane l supplies row l % 16 of A and column l % 16 of
// B with the K slice (l / 16) * K / 4 ..; both share the 16x16 f32 output layout (lane l holds
// rows 4 (l / 16) .. + 3 of column l % 16).
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v4f mma(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mma(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8b, a),
                                                  __builtin_bit_cast(v8b, b), c, 0, 0, 0);
}
template <int CIN> struct FragOf { typedef v8s T; static constexpr int K = 32; };
template <> struct FragOf<16> { typedef v4s T; static constexpr int K = 16; };

// Stride-1 convolution of a channels-last bf16 input with CIN channels into NT * 16 output
// channels, on the grid (Z, Y, X). w: [27][NT*16][CIN] bf16. EPI 0: + bias, ReLU, bf16 out
// [v][NT*16]; EPI 1: + bias, f32 out [v][4] (channels < cout); EPI 2: times (mask[v][c] > 0)
// (the ReLU of the layer below), bf16 out [v][NT*16]. A block covers 64 x 4 output voxels of
// one z plane (wave w: row y0 + w, four 16-voxel M-tiles that share every weight fragment).
// It first stages its input tile, 66 x 6 x 3 voxels with zeros outside the grid, in LDS (all
// of a thread's loads issued before its first store; channel chunks swizzled against bank
// conflicts); then every wave runs the 27 taps, activations from LDS and
// weights (a few tens of KB, shared by every block) from the caches, each tap's weight
// fragments loaded two taps ahead so that the cache latency hides behind the MFMAs.
constexpr int kConvTX = 64, kConvTY = 4, kConvMT = kConvTX / 16;
// LDS position of a voxel's fragment-sized channel chunk g (of four): rows are not padded, the
// chunk index is XORed with bits 2..3 of the voxel index, so any 16 consecutive voxels' chunk
// g fall in 16 distinct 16-byte bank groups (and two 76 KB tiles fit per CU).
__device__ __forceinline__ int swz(int g, int vox) { return g ^ ((vox >> 2) & 3); }
template <int CIN, int NT, int EPI>
__global__ __launch_bounds__(256) void k_net_conv(const uint16_t* __restrict__ in, int Z, int Y,
                                                  int X, const uint16_t* __restrict__ w,
                                                  const float* __restrict__ bias, int cout,
                                                  void* __restrict__ out,
                                                  const uint16_t* __restrict__ mask) {
  using Frag = typename FragOf<CIN>::T;
  constexpr int KC = FragOf<CIN>::K, FL = KC / 4;  // K per MFMA; bf16 per lane and fragment
  constexpr int CO = NT * 16, CP = CIN, KT = CIN / KC, GR = CIN / FL;
  static_assert(KT == 1 && GR == 4, "one K step of four fragment-sized chunks per voxel");
  constexpr int TX = kConvTX + 2, TY = kConvTY + 2, NTILE = 3 * TY * TX;
  __shared__ __align__(16) uint16_t tile[NTILE * CP];
  const int nbx = (X + kConvTX - 1) / kConvTX, nby = (Y + kConvTY - 1) / kConvTY;
  const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, z = blockIdx.x / (nbx * nby);
  const int x0 = bx * kConvTX, y0 = by * kConvTY;
  {  // stage: element (voxel, fragment-sized channel group) of the tile
    constexpr int NE = NTILE * GR, PER = (NE + 255) / 256;
    Frag buf[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 256 * i;
      buf[i] = Frag{};
      const int cg = e % GR, vox = e / GR;
      const int lx = vox % TX, ly = (vox / TX) % TY, lz = vox / (TX * TY);
      const int xx = x0 + lx - 1, yy = y0 + ly - 1, zz = z + lz - 1;
      if (e < NE && xx >= 0 && xx < X && yy >= 0 && yy < Y && zz >= 0 && zz < Z)
        buf[i] = *reinterpret_cast<const Frag*>(in + (((size_t)zz * Y + yy) * X + xx) * CIN +
                                                FL * cg);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < NE) {
        const int vox = e / GR;
        *reinterpret_cast<Frag*>(tile + vox * CP + FL * swz(e % GR, vox)) = buf[i];
      }
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 15, q = lane >> 4;
  const int y = y0 + wave;
  v4f acc[kConvMT][NT];
#pragma unroll
  for (int h = 0; h < kConvMT; ++h)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[h][nt] = v4f{0.f, 0.f, 0.f, 0.f};
  // lane (m, q) supplies row m of A (voxel) and column m of B (output channel) with the input
  // channels kt KC + FL q .. kt KC + FL q + FL - 1
  const uint16_t* wl = w + m * CIN + FL * q;
  const int vl = wave * TX + m;  // the lane's voxel in the tile at tap 0, M-tile 0
  constexpr int D = 2;  // prefetch distance in taps
  Frag bq[D + 1][KT][NT];
#pragma unroll
  for (int s = 0; s < 27 + D; ++s) {
    if (s < 27) {
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          bq[s % (D + 1)][kt][nt] =
              *reinterpret_cast<const Frag*>(wl + (s * CO + nt * 16) * CIN + kt * KC);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this tap's MFMAs
    if (s >= D) {
      const int t = s - D;
      const int offv = ((t / 9) * TY + (t / 3) % 3) * TX + t % 3;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        Frag a[kConvMT];
#pragma unroll
        for (int h = 0; h < kConvMT; ++h) {
          const int vox = vl + offv + 16 * h;
          a[h] = *reinterpret_cast<const Frag*>(tile + vox * CP + FL * swz(q, vox));
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
          for (int h = 0; h < kConvMT; ++h)
            acc[h][nt] = mma(a[h], bq[t % (D + 1)][kt][nt], acc[h][nt]);
      }
    }
  }
  if (y >= Y) return;
  // lane holds D[4 q + i][m] of M-tile h: voxel x0 + 16 h + 4 q + i, channel nt * 16 + m
#pragma unroll
  for (int h = 0; h < kConvMT; ++h)
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int c = nt * 16 + m;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int x = x0 + 16 * h + 4 * q + i;
      if (x >= X) continue;
      const size_t v = ((size_t)z * Y + y) * X + x;
      float val = acc[h][nt][i];
      if (EPI == 0) {
        val = fmaxf(val + bias[c], 0.f);
        reinterpret_cast<uint16_t*>(out)[v * CO + c] = f2bf(val);
      } else if (EPI == 1) {
        if (c < cout) reinterpret_cast<float*>(out)[v * 4 + c] = val + bias[c];
      } else {
        if (!(bf2f(mask[v * CO + c]) > 0.f)) val = 0.f;
        reinterpret_cast<uint16_t*>(out)[v * CO + c] = f2bf(val);
      }
    }
  }
}

// The first layer: x (f32, full resolution (Zi, Yi, Xi), times scale) to 32 channels on the
// half-resolution grid (Z, Y, X), stride 2, + bias, ReLU, bf16 out [v][32]. K = the 27 taps
// padded to 32; w: [32 co][32 k] bf16.
__global__ __launch_bounds__(256) void k_net_conv1(const float* __restrict__ xin, int Zi, int Yi,
                                                   int Xi, float scale, int Z, int Y, int X,
                                                   const uint16_t* __restrict__ w,
                                                   const float* __restrict__ bias,
                                                   uint16_t* __restrict__ out) {
  __shared__ uint16_t ws[32 * 32];
  for (int e = threadIdx.x; e < 32 * 32 / 4; e += 256)
    reinterpret_cast<uint2*>(ws)[e] = reinterpret_cast<const uint2*>(w)[e];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 15, q = lane >> 4;
  const int nxs = (X + 15) / 16;
  const long long seg = (long long)blockIdx.x * 4 + wave;
  const int xs = (int)(seg % nxs);
  const long long r = seg / nxs;
  const int y = (int)(r % Y), z = (int)(r / Y);
  if (z >= Z) return;
  const int x0 = xs * 16;
  v4f acc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
  for (int kc = 0; kc < 2; ++kc) {
    v4s a;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = kc * 16 + 4 * q + j;
      float v = 0.f;
      if (t < 27) {
        const int zz = 2 * z + t / 9 - 1, yy = 2 * y + (t / 3) % 3 - 1, xx = 2 * (x0 + m) + t % 3 - 1;
        if (zz >= 0 && zz < Zi && yy >= 0 && yy < Yi && xx >= 0 && xx < Xi && x0 + m < X)
          v = xin[((size_t)zz * Yi + yy) * Xi + xx] * scale;
      }
      a[j] = (short)f2bf(v);
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const v4s b = *reinterpret_cast<const v4s*>(ws + (nt * 16 + m) * 32 + kc * 16 + 4 * q);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int c = nt * 16 + m;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int x = x0 + 4 * q + i;
      if (x >= X) continue;
      const size_t v = ((size_t)z * Y + y) * X + x;
      out[v * 32 + c] = f2bf(fmaxf(acc[nt][i] + bias[c], 0.f));
    }
  }
}

// ---------------------------------------------------------------- weight gradients

// part[g][t][co][ci] = sum over voxels v of group g of dy[v][co] * x[v + t - 1][ci] (stride 1,
// zero outside; x bf16 [v][CIN], dy bf16 [v][COP]; block (t, g), voxel indices fit in int,
// checked by the launcher), on the matrix cores: for tap t the 16 x 16 tiles of the [COP][CIN]
// product dY^T X_t, with K running over the group's voxels 32 at a time
// (v_mfma_f32_16x16x32_bf16, bf16 products exact in float32, float32 accumulation). Voxels are
// staged 64 at a time in LDS, transposed so that a lane's 8 consecutive voxels of one channel
// are one 16-byte read: sdy[co][j] = dy[v0 + j][co], sx[ci][j] = x[v0 + j + t - 1][ci] (zero
// outside). The T = COP CIN / 256 tiles go to the 4 waves, 4 / T waves per tile splitting the
// K steps; their accumulators meet in LDS and are added in wave order. The centre tap's
// blocks also leave the bias partial bpart[g][co] (float32 sums over the staged voxels).
template <int CIN, int COP>
__global__ __launch_bounds__(256) void k_net_wgrad_mfma(const uint16_t* __restrict__ x,
                                                        const uint16_t* __restrict__ dy, int Z,
                                                        int Y, int X, int vpg,
                                                        float* __restrict__ part,
                                                        float* __restrict__ bpart) {
  constexpr int TI = CIN / 16, T = (COP / 16) * TI, KS = 4 / T;
  static_assert(CIN % 16 == 0 && COP % 16 == 0 && (T == 1 || T == 2 || T == 4),
                "whole 16 x 16 tiles, shared evenly by four waves");
  constexpr int JP = 64 + 8;  // row pitch (bf16) of the transposed tiles
  __shared__ __align__(16) uint16_t sdy[COP][JP];
  __shared__ __align__(16) uint16_t sx[CIN][JP];
  __shared__ float red[4][64][4];
  const int t = blockIdx.x, g = blockIdx.y;
  const int dz = t / 9 - 1, dyy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  const int V = Z * Y * X;
  const int v0 = g * vpg, v1 = min(V, v0 + vpg);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tile = wave % T, ks = wave / T;
  const int co0 = (tile / TI) * 16, ci0 = (tile % TI) * 16;
  const int m = lane & 15, q = lane >> 4;
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int vb = v0; vb < v1; vb += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * COP / 8; e += 256) {
      const int j = e / (COP / 8), c8 = (e % (COP / 8)) * 8, v = vb + j;
      uint4 raw = make_uint4(0u, 0u, 0u, 0u);
      if (v < v1) raw = *reinterpret_cast<const uint4*>(dy + (size_t)v * COP + c8);
      const uint32_t w4[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        sdy[c8 + 2 * i][j] = (uint16_t)(w4[i] & 0xffffu);
        sdy[c8 + 2 * i + 1][j] = (uint16_t)(w4[i] >> 16);
      }
    }
    for (int e = tid; e < 64 * CIN / 8; e += 256) {
      const int j = e / (CIN / 8), c8 = (e % (CIN / 8)) * 8, v = vb + j;
      uint4 raw = make_uint4(0u, 0u, 0u, 0u);
      if (v < v1) {
        const int xx = v % X + dx, r = v / X;
        const int yy = r % Y + dyy, zz = r / Y + dz;
        if (xx >= 0 && xx < X && yy >= 0 && yy < Y && zz >= 0 && zz < Z)
          raw = *reinterpret_cast<const uint4*>(x + (((size_t)zz * Y + yy) * X + xx) * CIN + c8);
      }
      const uint32_t w4[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        sx[c8 + 2 * i][j] = (uint16_t)(w4[i] & 0xffffu);
        sx[c8 + 2 * i + 1][j] = (uint16_t)(w4[i] >> 16);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {  // K steps of 32 voxels
      if (s % KS != ks) continue;
      const int j0 = 32 * s + 8 * q;
      const v8s a = *reinterpret_cast<const v8s*>(&sdy[co0 + m][j0]);
      const v8s b = *reinterpret_cast<const v8s*>(&sx[ci0 + m][j0]);
      acc = mma(a, b, acc);
    }
    if (t == 13 && tid < COP)
      for (int j = 0; j < 64; ++j) bsum += bf2f(sdy[tid][j]);
  }
  // lane (m, q) holds the tile's rows co0 + 4 q + i, column ci0 + m
#pragma unroll
  for (int i = 0; i < 4; ++i) red[wave][lane][i] = acc[i];
  __syncthreads();
  if (ks == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float sum = red[wave][lane][i];
      for (int k = 1; k < KS; ++k) sum += red[wave + k * T][lane][i];
      part[(((size_t)g * 27 + t) * COP + co0 + 4 * q + i) * CIN + ci0 + m] = sum;
    }
  }
  if (t == 13 && tid < COP) bpart[(size_t)g * COP + tid] = bsum;
}

// The first layer's weight gradient: part[g][t][co] = sum over voxels v of group g of
// dy[v][co] * scale x[2 v + t - 1] (full-resolution input, zero outside). Block (t, g): 32 co
// x 8 voxel lanes. The centre tap's blocks also leave bpart[g][co] = sum of dy[v][co]. Voxel
// indices fit in int (checked by the launcher).
__global__ __launch_bounds__(256) void k_net_wgrad1(const float* __restrict__ xin, int Zi, int Yi,
                                                    int Xi, float scale,
                                                    const uint16_t* __restrict__ dy, int Z, int Y,
                                                    int X, int vpg, float* __restrict__ part,
                                                    float* __restrict__ bpart) {
  __shared__ float red[8][32];
  __shared__ float bred[8][32];
  const int t = blockIdx.x, g = blockIdx.y;
  const int dz = t / 9 - 1, dyy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  const int V = Z * Y * X;
  const int v0 = g * vpg, v1 = min(V, v0 + vpg);
  const int co = threadIdx.x & 31, lv = threadIdx.x >> 5;
  float acc = 0.f, bsum = 0.f;
  // the voxel's coordinates, divided out once and then stepped by 8 voxels
  int x = (v0 + lv) % X, y = ((v0 + lv) / X) % Y, z = (v0 + lv) / (X * Y);
#pragma unroll 4
  for (int v = v0 + lv; v < v1; v += 8) {
    const int xx = 2 * x + dx, yy = 2 * y + dyy, zz = 2 * z + dz;
    const float d = bf2f(dy[(size_t)v * 32 + co]);
    bsum += d;
    if (xx >= 0 && xx < Xi && yy >= 0 && yy < Yi && zz >= 0 && zz < Zi)
      acc = fmaf(d, xin[((size_t)zz * Yi + yy) * Xi + xx] * scale, acc);
    for (x += 8; x >= X; x -= X)
      if (++y == Y) {
        y = 0;
        ++z;
      }
  }
  red[lv][co] = acc;
  bred[lv][co] = bsum;
  __syncthreads();
  if (lv == 0) {
    float s = 0.f, b = 0.f;
    for (int i = 0; i < 8; ++i) {
      s += red[i][co];
      b += bred[i][co];
    }
    part[((size_t)g * 27 + t) * 32 + co] = s;
    if (t == 13) bpart[(size_t)g * 32 + co] = b;
  }
}

// Sums the weight-gradient partials over the ng groups (in group order) into the master
// layout grad[co][ci][t] (co < cout, ci < cin), and the bias gradient sum_v dy[v][co] (cop
// channels per voxel) into bgrad[co]: one thread per output.
__global__ __launch_bounds__(256) void k_net_wgrad_sum(const float* __restrict__ part, int ng,
                                                       int cop, int cinp, int cout, int cin,
                                                       float* __restrict__ grad) {
  const int e = blockIdx.x * 256 + threadIdx.x;  // (co, ci, t) in the master layout
  if (e >= cout * cin * 27) return;
  const int t = e % 27, ci = (e / 27) % cin, co = e / (27 * cin);
  float s = 0.f;
#pragma unroll 8
  for (int g = 0; g < ng; ++g) s += part[(((size_t)g * 27 + t) * cop + co) * cinp + ci];
  grad[e] = s;
}

// bgrad[co] = sum over the ng groups (in order) of bpart[g][co], co < cout.
__global__ __launch_bounds__(64) void k_net_bgrad(const float* __restrict__ bpart, int ng, int cop,
                                                  int cout, float* __restrict__ bgrad) {
  const int co = threadIdx.x;
  if (co >= cout) return;
  float s = 0.f;
#pragma unroll 8
  for (int g = 0; g < ng; ++g) s += bpart[(size_t)g * cop + co];
  bgrad[co] = s;
}

// ---------------------------------------------------------------- loss, packing, update

struct NetAtoms {
  float a[kNetMaxAtoms][6];
};

// Targets of the atoms still to be found (w, mx, my, mz, sigma, d; full-resolution centres)
// on the half-resolution grid and the squared-error loss: the gradient of the output layer
// (bf16 [v][16], channels 0..2) and per-block float64 partials of the loss.
__global__ __launch_bounds__(256) void k_net_loss(const float* __restrict__ out, int Z, int Y,
                                                  int X, NetAtoms atoms, int k,
                                                  uint16_t* __restrict__ dout,
                                                  double* __restrict__ lpart) {
  __shared__ double red[256];
  const long long V = (long long)Z * Y * X;
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (v < V) {
    const int x = (int)(v % X);
    const long long rr = v / X;
    const int y = (int)(rr % Y), z = (int)(rr / Y);
    float T = 0.f, best = INFINITY, S = 0.f, D = 0.f;
    for (int j = 0; j < k; ++j) {
      const float ex = x - 0.5f * atoms.a[j][1], ey = y - 0.5f * atoms.a[j][2],
                  ez = z - 0.5f * atoms.a[j][3];
      const float d2 = ex * ex + ey * ey + ez * ez;
      T = fmaxf(T, expf(-0.5f * d2));
      if (d2 < best) {
        best = d2;
        S = atoms.a[j][4];
        D = atoms.a[j][5];
      }
    }
    const float M = best <= 1.f ? 1.f : 0.f;
    const float r0 = out[v * 4] - T, r1 = M * (out[v * 4 + 1] - S), r2 = M * (out[v * 4 + 2] - D);
    l = (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2;
    const float s = 2.f / (float)V;
    uint16_t* g = dout + v * kNetOutPad;
    g[0] = f2bf(s * r0);
    g[1] = f2bf(s * r1);
    g[2] = f2bf(s * r2);
    for (int c = 3; c < kNetOutPad; ++c) g[c] = 0;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_net_loss_sum(const double* __restrict__ lpart, int n,
                                                      long long V, double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += lpart[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (double)V;
}

// bf16 matrix-core copies of one layer's weights from the master f32 [co][ci][27]: forward
// wf[t][cop][cip] and, for a stride-1 layer, backward wb[t'][cip][cop] = w[co][ci][26 - t'];
// padded entries are zero. One thread per (t, a, b) of the larger layout.
__global__ __launch_bounds__(256) void k_net_pack(const float* __restrict__ wm, int cout, int cin,
                                                  int cop, int cip, uint16_t* __restrict__ wf,
                                                  uint16_t* __restrict__ wb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= 27 * cop * cip) return;
  const int t = e / (cop * cip), co = (e / cip) % cop, ci = e % cip;
  const float v = (co < cout && ci < cin) ? wm[((size_t)co * cin + ci) * 27 + t] : 0.f;
  wf[e] = f2bf(v);
  if (wb) wb[((size_t)(26 - t) * cip + ci) * cop + co] = f2bf(v);
}

// The first layer's forward copy: wf[co][k] = w[co][0][k] for k < 27, 0 for 27 <= k < 32.
__global__ __launch_bounds__(256) void k_net_pack1(const float* __restrict__ wm,
                                                   uint16_t* __restrict__ wf) {
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int co = e / 32, k = e % 32;
    wf[e] = f2bf(k < 27 ? wm[co * 27 + k] : 0.f);
  }
}

// Adam on the master parameters (float32), step count folded into the bias corrections
// c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ __launch_bounds__(256) void k_net_adam(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m1, float* __restrict__ m2,
                                                  int n, float lr, float b1, float b2, float c1,
                                                  float c2, float eps) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi, b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a * c1) / (sqrtf(b * c2) + eps);
}

// Maximum of the heatmap logit over the half-resolution grid, ties to the lowest voxel: block
// partials (value, voxel), then one block folds them and writes the proposal (value, voxel,
// sigma, d) to res[0..3] (host memory is fine) and signals.
__global__ __launch_bounds__(256) void k_net_argmax(const float* __restrict__ out, long long V,
                                                    float* __restrict__ pv,
                                                    long long* __restrict__ pi) {
  __shared__ float rv[256];
  __shared__ long long ri[256];
  float bv = -INFINITY;
  long long bi = V;
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < V; v += (long long)gridDim.x * 256) {
    const float h = out[v * 4];
    if (h > bv) {
      bv = h;
      bi = v;
    }
  }
  rv[threadIdx.x] = bv;
  ri[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const float ov = rv[threadIdx.x + o];
      const long long oi = ri[threadIdx.x + o];
      if (ov > rv[threadIdx.x] || (ov == rv[threadIdx.x] && oi < ri[threadIdx.x])) {
        rv[threadIdx.x] = ov;
        ri[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = rv[0];
    pi[blockIdx.x] = ri[0];
  }
}

// The heatmap is fitted to unit Gaussian blobs, so log h is quadratic near a centre: the peak
// of the parabola through the maximum and its two neighbours along each axis (h clamped to
// 1e-3, offset clamped to half a voxel) refines the centre below the grid step. res[4..6] =
// the offsets along x, y, z (half-resolution voxels).
__device__ __forceinline__ double peak_offset(float hm, float h0, float hp) {
  const double a = log(fmax((double)hm, 1e-3)), b = log(fmax((double)h0, 1e-3)),
               c = log(fmax((double)hp, 1e-3));
  const double den = a - 2.0 * b + c;
  if (!(den < 0.0)) return 0.0;
  return fmin(0.5, fmax(-0.5, 0.5 * (a - c) / den));
}

__global__ __launch_bounds__(64) void k_net_argmax_final(const float* __restrict__ pv,
                                                         const long long* __restrict__ pi, int n,
                                                         const float* __restrict__ out, int Z,
                                                         int Y, int X, double* __restrict__ res,
                                                         SigArgs sig) {
  const int lane = threadIdx.x;
  float bv = -INFINITY;
  long long bi = 0x7fffffffffffffffLL;
  for (int i = lane; i < n; i += 64)
    if (pv[i] > bv || (pv[i] == bv && pi[i] < bi)) {
      bv = pv[i];
      bi = pi[i];
    }
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(bv, o, 64);
    const long long oi = __shfl_xor(bi, o, 64);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    res[0] = bv;
    res[1] = (double)bi;
    const bool ok = bi >= 0 && bi != 0x7fffffffffffffffLL && bv > -INFINITY;
    res[2] = ok ? out[bi * 4 + 1] : 0.0;
    res[3] = ok ? out[bi * 4 + 2] : 0.0;
    res[4] = res[5] = res[6] = 0.0;
    res[7] = ok ? 1.0 : 0.0;  // no finite heatmap value (a diverged network): no proposal
    if (ok) {
      const int x = (int)(bi % X), y = (int)((bi / X) % Y), z = (int)(bi / ((long long)X * Y));
      const float h0 = out[bi * 4];
      const long long sx = 1, sy = X, sz = (long long)X * Y;
      if (x > 0 && x + 1 < X) res[4] = peak_offset(out[(bi - sx) * 4], h0, out[(bi + sx) * 4]);
      if (y > 0 && y + 1 < Y) res[5] = peak_offset(out[(bi - sy) * 4], h0, out[(bi + sy) * 4]);
      if (z > 0 && z + 1 < Z) res[6] = peak_offset(out[(bi - sz) * 4], h0, out[(bi + sz) * 4]);
    }
  }
  if (lane < 64) __threadfence_system();
  if (lane == 0 && sig.flag) *reinterpret_cast<volatile int*>(sig.flag) = sig.seq;
}

}  // namespace
}  // namespace sfw

// ---------------------------------------------------------------- the network object

struct sfw_net {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t vcap = 0;   // full-resolution voxels
  size_t vhcap = 0;  // half-resolution voxels
  float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
  uint16_t *wf1 = nullptr, *wf2 = nullptr, *wf3 = nullptr, *wf4 = nullptr;
  uint16_t *wb2 = nullptr, *wb3 = nullptr, *wb4 = nullptr;
  uint16_t *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *dout = nullptr;
  uint16_t *g1 = nullptr, *g2 = nullptr, *g3 = nullptr;
  float* out = nullptr;
  float* part = nullptr;
  float* bpart = nullptr;  // [64 groups][32] bias partials
  size_t part_cap = 0;  // floats
  double *lpart = nullptr, *loss = nullptr;
  float* apv = nullptr;
  long long* api = nullptr;
  double* hres = nullptr;  // pinned [8]
  int* sig_flag = nullptr;  // coherent pinned
  int sig_seq = 0;
  int step = 0;
};

namespace sfw {
namespace {

constexpr int kNetArgBlocks = 256;

struct NetDims {
  int Zi, Yi, Xi, Z, Y, X;
  long long V() const { return (long long)Z * Y * X; }
};

NetDims net_dims(const sfw_dims& vol) {
  NetDims d;
  d.Zi = vol.nz;
  d.Yi = vol.ny;
  d.Xi = vol.nx;
  d.Z = (vol.nz + 1) / 2;
  d.Y = (vol.ny + 1) / 2;
  d.X = (vol.nx + 1) / 2;
  return d;
}

unsigned conv_blocks(const NetDims& d) {  // k_net_conv1: four 16-voxel segments per block
  const long long seg = (long long)((d.X + 15) / 16) * d.Y * d.Z;
  return (unsigned)((seg + 3) / 4);
}

unsigned tile_blocks(const NetDims& d) {  // k_net_conv: 64 x 4 voxels of one plane per block
  return (unsigned)((long long)((d.X + kConvTX - 1) / kConvTX) * ((d.Y + kConvTY - 1) / kConvTY) *
                    d.Z);
}

int net_check(const sfw_net* net, const float* x, const sfw_dims& vol) {
  if (!net) return fail(SFW_EINVAL, "net is NULL");
  if (!x) return fail(SFW_EINVAL, "x is NULL");
  int rc = check_dims(vol, "vol");
  if (rc) return rc;
  if ((size_t)vol.nx * vol.ny * vol.nz > net->vcap)
    return fail(SFW_EINVAL, "vol exceeds the network's vol_max");
  if (net_dims(vol).V() > (long long)net->vhcap) return fail(SFW_EINVAL, "vol exceeds vol_max");
  return SFW_OK;
}

hipError_t net_pack(sfw_net* n) {
  hipLaunchKernelGGL(k_net_pack1, dim3(1), dim3(256), 0, n->stream, n->params + kOff1, n->wf1);
  const int e32 = 27 * 32 * 32;
  hipLaunchKernelGGL(k_net_pack, dim3((e32 + 255) / 256), dim3(256), 0, n->stream,
                     n->params + kOff2, 32, 32, 32, 32, n->wf2, n->wb2);
  hipLaunchKernelGGL(k_net_pack, dim3((e32 + 255) / 256), dim3(256), 0, n->stream,
                     n->params + kOff3, 32, 32, 32, 32, n->wf3, n->wb3);
  const int e4 = 27 * kNetOutPad * 32;
  hipLaunchKernelGGL(k_net_pack, dim3((e4 + 255) / 256), dim3(256), 0, n->stream,
                     n->params + kOff4, kNetOut, 32, kNetOutPad, 32, n->wf4, n->wb4);
  return hipGetLastError();
}

int net_forward(sfw_net* n, const float* x, const NetDims& d, float scale) {
  const unsigned nb = conv_blocks(d), tb = tile_blocks(d);
  hipLaunchKernelGGL(k_net_conv1, dim3(nb), dim3(256), 0, n->stream, x, d.Zi, d.Yi, d.Xi, scale,
                     d.Z, d.Y, d.X, n->wf1, n->params + kOff1 + kW1, n->a1);
  hipLaunchKernelGGL((k_net_conv<32, 2, 0>), dim3(tb), dim3(256), 0, n->stream, n->a1, d.Z, d.Y,
                     d.X, n->wf2, n->params + kOff2 + kW2, 32, (void*)n->a2, nullptr);
  hipLaunchKernelGGL((k_net_conv<32, 2, 0>), dim3(tb), dim3(256), 0, n->stream, n->a2, d.Z, d.Y,
                     d.X, n->wf3, n->params + kOff3 + kW2, 32, (void*)n->a3, nullptr);
  hipLaunchKernelGGL((k_net_conv<32, 1, 1>), dim3(tb), dim3(256), 0, n->stream, n->a3, d.Z, d.Y,
                     d.X, n->wf4, n->params + kOff4 + kW4, kNetOut, (void*)n->out, nullptr);
  SFW_HIP(hipGetLastError());
  return SFW_OK;
}

// weight and bias gradients of one layer into grads (master layout)
template <int CIN, int COP>
int net_wgrad(sfw_net* n, const uint16_t* xin, const uint16_t* dy, const NetDims& d, int cout,
              float* gw, float* gb) {
  const long long V = d.V();
  const int ng = (int)std::max<long long>(1, std::min<long long>(64, (V + 1023) / 1024));
  const int vpg = (int)((V + ng - 1) / ng);
  if ((size_t)ng * 27 * COP * CIN > n->part_cap) return fail(SFW_EINVAL, "gradient partials too small");
  if (V > INT_MAX - 64) return fail(SFW_EINVAL, "half-resolution volume too large");
  hipLaunchKernelGGL((k_net_wgrad_mfma<CIN, COP>), dim3(27, ng), dim3(256), 0, n->stream, xin, dy,
                     d.Z, d.Y, d.X, vpg, n->part, n->bpart);
  const int e = cout * CIN * 27;
  hipLaunchKernelGGL(k_net_wgrad_sum, dim3((e + 255) / 256), dim3(256), 0, n->stream, n->part, ng,
                     COP, CIN, cout, CIN, gw);
  hipLaunchKernelGGL(k_net_bgrad, dim3(1), dim3(64), 0, n->stream, n->bpart, ng, COP, cout, gb);
  SFW_HIP(hipGetLastError());
  return SFW_OK;
}

// forward, loss against the atoms still to be found, backward: grads and n->loss
int net_backprop(sfw_net* n, const float* x, const NetDims& d, float scale, const float* atoms,
                 int k) {
  int rc = net_forward(n, x, d, scale);
  if (rc) return rc;
  NetAtoms na;
  std::memset(&na, 0, sizeof(na));
  std::memcpy(na.a, atoms, sizeof(float) * 6 * (size_t)k);
  const long long V = d.V();
  const unsigned lb = (unsigned)((V + 255) / 256);
  hipLaunchKernelGGL(k_net_loss, dim3(lb), dim3(256), 0, n->stream, n->out, d.Z, d.Y, d.X, na, k,
                     n->dout, n->lpart);
  hipLaunchKernelGGL(k_net_loss_sum, dim3(1), dim3(256), 0, n->stream, n->lpart, (int)lb, V,
                     n->loss);
  SFW_HIP(hipGetLastError());
  const unsigned tb = tile_blocks(d);
  // layer 4
  rc = net_wgrad<32, kNetOutPad>(n, n->a3, n->dout, d, kNetOut, n->grads + kOff4,
                                  n->grads + kOff4 + kW4);
  if (rc) return rc;
  hipLaunchKernelGGL((k_net_conv<kNetOutPad, 2, 2>), dim3(tb), dim3(256), 0, n->stream, n->dout,
                     d.Z, d.Y, d.X, n->wb4, nullptr, 32, (void*)n->g3, n->a3);
  // layer 3
  rc = net_wgrad<32, 32>(n, n->a2, n->g3, d, 32, n->grads + kOff3, n->grads + kOff3 + kW2);
  if (rc) return rc;
  hipLaunchKernelGGL((k_net_conv<32, 2, 2>), dim3(tb), dim3(256), 0, n->stream, n->g3, d.Z, d.Y,
                     d.X, n->wb3, nullptr, 32, (void*)n->g2, n->a2);
  // layer 2
  rc = net_wgrad<32, 32>(n, n->a1, n->g2, d, 32, n->grads + kOff2, n->grads + kOff2 + kW2);
  if (rc) return rc;
  hipLaunchKernelGGL((k_net_conv<32, 2, 2>), dim3(tb), dim3(256), 0, n->stream, n->g2, d.Z, d.Y,
                     d.X, n->wb2, nullptr, 32, (void*)n->g1, n->a1);
  // layer 1 (stride 2 from the full-resolution input)
  if (V > INT_MAX - 64) return fail(SFW_EINVAL, "half-resolution volume too large");
  const int ng = (int)std::max<long long>(1, std::min<long long>(64, (V + 1023) / 1024));
  const int vpg = (int)((V + ng - 1) / ng);
  hipLaunchKernelGGL(k_net_wgrad1, dim3(27, ng), dim3(256), 0, n->stream, x, d.Zi, d.Yi, d.Xi,
                     scale, n->g1, d.Z, d.Y, d.X, vpg, n->part, n->bpart);
  hipLaunchKernelGGL(k_net_wgrad_sum, dim3((32 * 27 + 255) / 256), dim3(256), 0, n->stream,
                     n->part, ng, 32, 1, 32, 1, n->grads + kOff1);
  hipLaunchKernelGGL(k_net_bgrad, dim3(1), dim3(64), 0, n->stream, n->bpart, ng, 32, 32,
                     n->grads + kOff1 + kW1);
  SFW_HIP(hipGetLastError());
  return SFW_OK;
}

}  // namespace

// the solver's proposal: seed theta = (m, sigma, d) from the heatmap maximum (host [5]),
// *score = the heatmap logit there; x is the adjoint volume, scaled by `scale`
int net_propose(sfw_net* n, const float* x, const sfw_dims& vol, float scale, double theta[5],
                double* score) {
  const NetDims d = net_dims(vol);
  int rc = net_forward(n, x, d, scale);
  if (rc) return rc;
  const long long V = d.V();
  const int nb = (int)std::max<long long>(1, std::min<long long>(kNetArgBlocks, (V + 255) / 256));
  hipLaunchKernelGGL(k_net_argmax, dim3(nb), dim3(256), 0, n->stream, n->out, V, n->apv, n->api);
  if (++n->sig_seq <= 0) n->sig_seq = 1;
  const SigArgs sig{n->sig_flag, nullptr, n->sig_seq};
  hipLaunchKernelGGL(k_net_argmax_final, dim3(1), dim3(64), 0, n->stream, n->apv, n->api, nb,
                     n->out, d.Z, d.Y, d.X, n->hres, sig);
  SFW_HIP(hipGetLastError());
  for (unsigned long spins = 1;; ++spins) {
    if (__atomic_load_n(n->sig_flag, __ATOMIC_ACQUIRE) == sig.seq) break;
    if ((spins & 0x3fff) == 0) {
      const hipError_t e = hipStreamQuery(n->stream);
      if (e == hipSuccess) {
        if (__atomic_load_n(n->sig_flag, __ATOMIC_ACQUIRE) == sig.seq) break;
        return fail(SFW_EHIP, "the stream finished without the proposal's completion signal");
      }
      if (e != hipErrorNotReady) return hip_fail(e, "waiting for the proposal");
    }
    __builtin_ia32_pause();
  }
  if (n->hres[7] == 0.0) {  // no finite heatmap value: report that there is no proposal
    for (int c = 0; c < 5; ++c) theta[c] = std::numeric_limits<double>::quiet_NaN();
    *score = -std::numeric_limits<double>::infinity();
    return SFW_OK;
  }
  const long long v = (long long)n->hres[1];
  const int ox = (int)(v % d.X), oy = (int)((v / d.X) % d.Y), oz = (int)(v / ((long long)d.X * d.Y));
  theta[0] = 2.0 * (ox + n->hres[4]);
  theta[1] = 2.0 * (oy + n->hres[5]);
  theta[2] = 2.0 * (oz + n->hres[6]);
  theta[3] = n->hres[2];
  theta[4] = n->hres[3];
  *score = n->hres[0];
  return SFW_OK;
}

}  // namespace sfw

hipStream_t net_stream(const sfw_net* n) { return n->stream; }

using namespace sfw;

extern "C" {

int sfw_net_num_params(void) { return kNetParams; }

void sfw_net_destroy(sfw_net* n) {
  if (!n) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(n->device);
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  void* dev[] = {n->params, n->grads, n->m1, n->m2, n->wf1, n->wf2, n->wf3, n->wf4, n->wb2,
                 n->wb3, n->wb4, n->a1, n->a2, n->a3, n->dout, n->g1, n->g2, n->g3, n->out,
                 n->part, n->bpart, n->lpart, n->loss, n->apv, n->api};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (n->hres) (void)hipHostFree(n->hres);
  if (n->sig_flag) (void)hipHostFree(n->sig_flag);
  (void)hipSetDevice(cur);
  delete n;
}

int sfw_net_create(sfw_net** out, sfw_dims vol_max, hipStream_t stream) {
  if (!out) return fail(SFW_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_dims(vol_max, "vol_max");
  if (rc) return rc;
  sfw_net* n = new (std::nothrow) sfw_net();
  if (!n) return fail(SFW_ENOMEM, "host allocation failed");
  (void)hipGetDevice(&n->device);
  n->stream = stream;
  n->vcap = (size_t)vol_max.nx * vol_max.ny * vol_max.nz;
  n->vhcap = (size_t)((vol_max.nx + 1) / 2) * ((vol_max.ny + 1) / 2) * ((vol_max.nz + 1) / 2);
  const size_t vh = n->vhcap;
  const long long ngmax = 64;
  n->part_cap = (size_t)ngmax * 27 * 32 * 32;
#define NET_ALLOC(ptr, bytes)                                                        \
  if (hipMalloc(reinterpret_cast<void**>(&(ptr)), (bytes)) != hipSuccess) {          \
    (void)hipGetLastError();                                                         \
    sfw_net_destroy(n);                                                              \
    return fail(SFW_ENOMEM, "device allocation of the network failed");             \
  }
  NET_ALLOC(n->params, kNetParams * sizeof(float));
  NET_ALLOC(n->grads, kNetParams * sizeof(float));
  NET_ALLOC(n->m1, kNetParams * sizeof(float));
  NET_ALLOC(n->m2, kNetParams * sizeof(float));
  NET_ALLOC(n->wf1, 32 * 32 * 2);
  NET_ALLOC(n->wf2, 27 * 32 * 32 * 2);
  NET_ALLOC(n->wf3, 27 * 32 * 32 * 2);
  NET_ALLOC(n->wf4, 27 * kNetOutPad * 32 * 2);
  NET_ALLOC(n->wb2, 27 * 32 * 32 * 2);
  NET_ALLOC(n->wb3, 27 * 32 * 32 * 2);
  NET_ALLOC(n->wb4, 27 * kNetOutPad * 32 * 2);
  NET_ALLOC(n->a1, vh * 32 * 2);
  NET_ALLOC(n->a2, vh * 32 * 2);
  NET_ALLOC(n->a3, vh * 32 * 2);
  NET_ALLOC(n->g1, vh * 32 * 2);
  NET_ALLOC(n->g2, vh * 32 * 2);
  NET_ALLOC(n->g3, vh * 32 * 2);
  NET_ALLOC(n->dout, vh * kNetOutPad * 2);
  NET_ALLOC(n->out, vh * 4 * sizeof(float));
  NET_ALLOC(n->part, n->part_cap * sizeof(float));
  NET_ALLOC(n->bpart, 64 * 32 * sizeof(float));
  NET_ALLOC(n->lpart, ((vh + 255) / 256) * sizeof(double));
  NET_ALLOC(n->loss, sizeof(double));
  NET_ALLOC(n->apv, kNetArgBlocks * sizeof(float));
  NET_ALLOC(n->api, kNetArgBlocks * sizeof(long long));
#undef NET_ALLOC
  if (hipHostMalloc(reinterpret_cast<void**>(&n->hres), 8 * sizeof(double), 0) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&n->sig_flag), 64, hipHostMallocCoherent) !=
          hipSuccess) {
    (void)hipGetLastError();
    sfw_net_destroy(n);
    return fail(SFW_ENOMEM, "pinned host allocation of the network failed");
  }
  *n->sig_flag = 0;
  if (hipMemset(n->params, 0, kNetParams * sizeof(float)) != hipSuccess ||
      hipMemset(n->m1, 0, kNetParams * sizeof(float)) != hipSuccess ||
      hipMemset(n->m2, 0, kNetParams * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    sfw_net_destroy(n);
    return fail(SFW_EHIP, "clearing the network failed");
  }
  if (net_pack(n) != hipSuccess || hipStreamSynchronize(n->stream) != hipSuccess) {
    (void)hipGetLastError();
    sfw_net_destroy(n);
    return fail(SFW_EHIP, "packing the network weights failed");
  }
  *out = n;
  return SFW_OK;
}

int sfw_net_set_params(sfw_net* n, const float* params, int count) {
  if (!n || !params) return fail(SFW_EINVAL, "net or params is NULL");
  if (count != kNetParams) return fail(SFW_EINVAL, "params must hold sfw_net_num_params() values");
  SFW_HIP(hipMemcpyAsync(n->params, params, sizeof(float) * kNetParams, hipMemcpyHostToDevice,
                         n->stream));
  SFW_HIP(hipMemsetAsync(n->m1, 0, sizeof(float) * kNetParams, n->stream));
  SFW_HIP(hipMemsetAsync(n->m2, 0, sizeof(float) * kNetParams, n->stream));
  n->step = 0;
  SFW_HIP(net_pack(n));
  SFW_HIP(hipStreamSynchronize(n->stream));
  return SFW_OK;
}

int sfw_net_get_params(sfw_net* n, float* params, int count) {
  if (!n || !params) return fail(SFW_EINVAL, "net or params is NULL");
  if (count != kNetParams) return fail(SFW_EINVAL, "params must hold sfw_net_num_params() values");
  SFW_HIP(hipMemcpyAsync(params, n->params, sizeof(float) * kNetParams, hipMemcpyDeviceToHost,
                         n->stream));
  SFW_HIP(hipStreamSynchronize(n->stream));
  return SFW_OK;
}

int sfw_net_forward(sfw_net* n, const float* x, sfw_dims vol, float scale, float* out) {
  int rc = net_check(n, x, vol);
  if (rc) return rc;
  if (!out) return fail(SFW_EINVAL, "out is NULL");
  const NetDims d = net_dims(vol);
  rc = net_forward(n, x, d, scale);
  if (rc) return rc;
  SFW_HIP(hipMemcpyAsync(out, n->out, sizeof(float) * 4 * (size_t)d.V(), hipMemcpyDeviceToDevice,
                         n->stream));
  return SFW_OK;
}

int sfw_net_gradients(sfw_net* n, const float* x, sfw_dims vol, float scale, const float* atoms,
                      int k, double* loss, float* grads) {
  int rc = net_check(n, x, vol);
  if (rc) return rc;
  if (k < 0 || k > kNetMaxAtoms || (k > 0 && !atoms))
    return fail(SFW_EINVAL, "atoms: 0 <= k <= 96 host rows (w, mx, my, mz, sigma, d)");
  rc = net_backprop(n, x, net_dims(vol), scale, atoms, k);
  if (rc) return rc;
  if (loss)
    SFW_HIP(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
  if (grads)
    SFW_HIP(hipMemcpyAsync(grads, n->grads, sizeof(float) * kNetParams, hipMemcpyDeviceToHost,
                           n->stream));
  SFW_HIP(hipStreamSynchronize(n->stream));
  return SFW_OK;
}

int sfw_net_train_step(sfw_net* n, const float* x, sfw_dims vol, float scale, const float* atoms,
                       int k, float lr, double* loss) {
  int rc = net_check(n, x, vol);
  if (rc) return rc;
  if (k < 0 || k > kNetMaxAtoms || (k > 0 && !atoms))
    return fail(SFW_EINVAL, "atoms: 0 <= k <= 96 host rows (w, mx, my, mz, sigma, d)");
  if (!(lr > 0.f)) return fail(SFW_EINVAL, "lr must be > 0");
  rc = net_backprop(n, x, net_dims(vol), scale, atoms, k);
  if (rc) return rc;
  n->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f / (1.f - std::pow(b1, (float)n->step));
  const float c2 = 1.f / (1.f - std::pow(b2, (float)n->step));
  hipLaunchKernelGGL(k_net_adam, dim3((kNetParams + 255) / 256), dim3(256), 0, n->stream,
                     n->params, n->grads, n->m1, n->m2, kNetParams, lr, b1, b2, c1, c2, 1e-8f);
  SFW_HIP(hipGetLastError());
  SFW_HIP(net_pack(n));
  if (loss) {
    SFW_HIP(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    SFW_HIP(hipStreamSynchronize(n->stream));
  }
  return SFW_OK;
}

int sfw_net_propose(sfw_net* n, const float* x, sfw_dims vol, float scale, double* theta,
                    double* score) {
  int rc = net_check(n, x, vol);
  if (rc) return rc;
  if (!theta || !score) return fail(SFW_EINVAL, "theta or score is NULL");
  return net_propose(n, x, vol, scale, theta, score);
}

}  // extern "C"
