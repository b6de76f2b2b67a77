// gfx950 kernels of the BSFW / SFW hot path (render, PSF convolution, residual, adjoint,
// gradient reduction, grid certificate and its maximum, LASSO dot products).
//
// The paper computes the convolutions in the Fourier domain and parallelises C and grad C
// across atoms (section 2). The Fourier-domain blur and certificate are in sfw_blur.hip and
// sfw_fft*.hip; this file holds the data-parallel kernels beside them: voxel columns for the
// atom sums, LDS-staged input tiles with register blocking along z for the direct
// convolutions (the blur's second and third paths), and wavefront DPP reductions for the
// per-atom gradient sums.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>

#include <cfloat>
#include <cmath>

#include "sfw_internal.h"

#include <algorithm>

namespace sfw {

namespace {

constexpr double kLog2Log2e = 0.52876637294489772;  // log2(log2(e))
constexpr double kLn2 = 0.69314718055994531;

__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// DPP row/broadcast controls (GFX9 encoding).
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int CTRL, int ROWMASK, bool BOUND>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                               ROWMASK, 0xf, BOUND));
}

// Sum of v over the 64 lanes of the wavefront, returned as a wave-uniform value.
// Requires all 64 lanes active.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<kRowShr1, 0xf, true>(v);
  v += dpp_f<kRowShr2, 0xf, true>(v);
  v += dpp_f<kRowShr4, 0xf, true>(v);
  v += dpp_f<kRowShr8, 0xf, true>(v);
  v += dpp_f<kRowBcast15, 0xa, false>(v);
  v += dpp_f<kRowBcast31, 0xc, false>(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ double shfl_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ bool arg_better(float v, long long i, float bv, long long bi) {
  return v > bv || (v == bv && i < bi);
}

// ------------------------------------------------------------------ preparation

// One launch for everything an evaluation needs before the render: grid.y = 0 computes the
// atom constants, grid.y = 1 / 2 the forward / adjoint PSF operands (matrix-core A operands
// when mfma != 0, else the [ky][kx][kzp] copies).
__global__ void k_prep(const sfw_atom* __restrict__ atoms, int n, int unit_weight,
                       AtomK* __restrict__ ak, const float* __restrict__ H, int px, int py,
                       int pz, int mfma, int steps, int kzp, int want_fwd, int want_adj,
                       float* __restrict__ out_fwd, float* __restrict__ out_adj) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int which = blockIdx.y;
  if (which == 0) {
    if (i >= n) return;
    const sfw_atom a = atoms[i];
    AtomK k;
    k.w = unit_weight ? 1.0f : a.w;
    k.mx = a.mx;
    k.my = a.my;
    k.mz = a.mz;
    k.hd = 0.5f * a.d;
    k.hdm1 = k.hd - 1.0f;
    k.c = (float)(-(double)a.d * log2((double)a.sigma) - 1.0 + kLog2Log2e);
    k.rcut2 = atom_rcut2((double)a.sigma, (double)a.d);
    ak[i] = k;
    return;
  }
  const int flip = which == 2;
  if ((flip && !want_adj) || (!flip && !want_fwd)) return;
  float* out = flip ? out_adj : out_fwd;
  if (mfma) {
    if (i >= steps * 64) return;
    const int lane = i & 63, s = i >> 6;
    const int kz = lane & 15;
    const int k = 4 * s + (lane >> 4);
    float v = 0.f;
    if (kz < pz && k < px * py) {
      const int ky = k / px, kx = k - ky * px;
      const int sz = flip ? pz - 1 - kz : kz;
      const int sy = flip ? py - 1 - ky : ky;
      const int sx = flip ? px - 1 - kx : kx;
      v = H[((size_t)sz * py + sy) * px + sx];
    }
    out[i] = v;
  } else {
    if (i >= px * py * kzp) return;
    const int kz = i % kzp;
    const int kx = (i / kzp) % px;
    const int ky = i / (kzp * px);
    float v = 0.f;
    if (kz < pz) {
      const int sz = flip ? pz - 1 - kz : kz;
      const int sy = flip ? py - 1 - ky : ky;
      const int sx = flip ? px - 1 - kx : kx;
      v = H[((size_t)sz * py + sy) * px + sx];
    }
    out[i] = v;
  }
}

// Completion signal (SigArgs), called by every thread of every block of a signalling kernel
// after its last write of results for the host. Only the block's first wave may write such
// results: its writes are made visible at system scope (one fence, which writes back the L2,
// per block) before the block is counted, and the block that completes the count resets the
// ticket and stores the sequence number into the host flag (a vector store).
__device__ __forceinline__ void signal_host(const SigArgs& s, unsigned nblocks) {
  if (!s.flag) return;
  if (threadIdx.x < 64) __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned done = nblocks > 1 ? atomicAdd(s.ticket, 1u) + 1u : 1u;
    if (done == nblocks) {
      if (nblocks > 1) *s.ticket = 0u;  // every block has been counted
      __threadfence_system();
      *reinterpret_cast<volatile int*>(s.flag) = s.seq;
    }
  }
}

// Order-independent 64-bit fingerprint of a float array: sum over i of bits(v[i]) * (2 i + 1)
// (mod 2^64). Used to recognise inputs already seen by cached LASSO columns. Blocks [0, by)
// take y and blocks [by, gridDim.x) take H; each leaves one partial, in part[b] (y) or
// part[kFpParts + b] (H). Threads read four consecutive values at a time where the array is
// 16-byte aligned.
__device__ __forceinline__ unsigned long long fp_term(float v, size_t i) {
  return (unsigned long long)__float_as_uint(v) * (2ull * i + 1ull);
}
__global__ __launch_bounds__(256) void k_fingerprints(const float* __restrict__ y, size_t ny,
                                                      int by, const float* __restrict__ H,
                                                      size_t nh,
                                                      unsigned long long* __restrict__ part) {
  __shared__ unsigned long long red[4];
  const bool is_y = (int)blockIdx.x < by;
  const int b = is_y ? (int)blockIdx.x : (int)blockIdx.x - by;
  const float* v = is_y ? y : H;
  const size_t len = is_y ? ny : nh;
  const size_t stride = (size_t)(is_y ? by : (int)gridDim.x - by) * 256;
  const size_t t0 = (size_t)b * 256 + threadIdx.x;
  unsigned long long h = 0ull;
  size_t done = 0;
  if ((reinterpret_cast<uintptr_t>(v) & 15) == 0) {
    const float4* v4 = reinterpret_cast<const float4*>(v);
    const size_t n4 = len / 4;
#pragma unroll 4
    for (size_t i = t0; i < n4; i += stride) {
      const float4 q = v4[i];
      const size_t e = 4 * i;
      h += fp_term(q.x, e) + fp_term(q.y, e + 1) + fp_term(q.z, e + 2) + fp_term(q.w, e + 3);
    }
    done = 4 * n4;
  }
  for (size_t i = done + t0; i < len; i += stride) h += fp_term(v[i], i);
  for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = h;
  __syncthreads();
  if (threadIdx.x == 0) part[(is_y ? 0 : kFpParts) + b] = red[0] + red[1] + red[2] + red[3];
}

// One wave: out[0] = fingerprint of y (the sum of its by partials), out[1] = that of H, and a
// copy of the n atoms (6 floats each) in atoms_out; out and atoms_out may be pinned host memory
// (signalled).
__global__ __launch_bounds__(64) void k_fingerprints_final(
    const unsigned long long* __restrict__ part, int by, int bh,
    const float* __restrict__ atoms, int n, unsigned long long* __restrict__ out,
    float* __restrict__ atoms_out, SigArgs sig) {
  const int lane = threadIdx.x;
  unsigned long long a = 0ull, c = 0ull;
  for (int i = lane; i < by; i += 64) a += part[i];
  for (int i = lane; i < bh; i += 64) c += part[kFpParts + i];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  if (lane == 0) {
    out[0] = a;
    out[1] = c;
  }
  for (int i = lane; i < 6 * n; i += 64) atoms_out[i] = atoms[i];
  signal_host(sig, 1);
}

// Stores up to kAtomArgs atom constants carried in the kernel arguments.
struct AtomArgs {
  AtomK a[kAtomArgs];
};
__global__ void k_store_atoms(AtomArgs args, int n, AtomK* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = args.a[i];
}

// Stores up to kDoubleArgs float64 values carried in the kernel arguments.
struct DoubleArgs {
  double v[kDoubleArgs];
};
__global__ void k_store_doubles(DoubleArgs args, int n, double* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = args.v[i];
}

// Voxel tiles of the render and gradient kernels: a block of 256 threads owns a 16 x 16 patch
// of (y, x) columns (thread t: x = 16 bx + t % 16, y = 16 by + t / 16), so a wave owns a
// 16 x 4 patch; tiles are numbered bx + tiles_x * by.
constexpr int kTile = 16;
struct TileXY {
  int x, y;     // this thread's column
  bool in;      // inside the plane
  int x0, y0w;  // wave patch origin (wave-uniform)
  int y0b;      // block tile's first row
};
__device__ __forceinline__ TileXY tile_xy(int tile, int nx, int ny, int rx0 = 0, int ry0 = 0,
                                          int rtx = -1) {
  const int tiles_x = rtx > 0 ? rtx : (nx + kTile - 1) / kTile;
  const int by = ry0 + tile / tiles_x, bx = rx0 + tile % tiles_x;
  TileXY t;
  t.x0 = bx * kTile;
  t.x = t.x0 + (int)(threadIdx.x & (kTile - 1));
  t.y = by * kTile + (int)(threadIdx.x / kTile);
  t.y0w = __builtin_amdgcn_readfirstlane(by * kTile + (int)((threadIdx.x & ~63u) / kTile));
  t.y0b = by * kTile;
  t.in = t.x < nx && t.y < ny;
  return t;
}

// Bounding box of the voxels of the calling wave (its 16 x 4 patch over planes zlo..zhi,
// clipped to the volume). misses(k) tells that atom k is exactly zero on all of them: its cut
// ball does not reach the box. Wave-uniform.
struct WaveBox {
  float xlo, xhi, ylo, yhi, zlo, zhi;
  __device__ bool misses(const AtomK& k) const {
    const float dx = fmaxf(0.f, fmaxf(xlo - k.mx, k.mx - xhi));
    const float dy = fmaxf(0.f, fmaxf(ylo - k.my, k.my - yhi));
    const float dz = fmaxf(0.f, fmaxf(zlo - k.mz, k.mz - zhi));
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz)) > k.rcut2;
  }
};
__device__ __forceinline__ WaveBox wave_box(const TileXY& t, int nx, int ny, int zlo, int zhi) {
  WaveBox b;
  b.xlo = (float)t.x0;
  b.xhi = (float)min(t.x0 + kTile - 1, nx - 1);
  b.ylo = (float)min(t.y0w, ny - 1);
  b.yhi = (float)min(t.y0w + 64 / kTile - 1, ny - 1);
  b.zlo = (float)zlo;
  b.zhi = (float)max(zhi, zlo);
  return b;
}

// Atom lists of one wave: lane l loads the constants of atom a0 + l (a < a1, at most 64 atoms,
// one coalesced load) and tests it against the wave's box; the returned ballot marks the atoms
// whose cut ball meets the box, the only ones with a nonzero term there. The wave then walks
// the set bits in increasing atom order and takes each atom's constants from its lane
// (lane_atom: eight readlanes into scalar registers), with no memory access per atom.
__device__ __forceinline__ unsigned long long wave_hits(const AtomK* __restrict__ ak, int a0,
                                                        int a1, const WaveBox& wb, AtomK& mine) {
  const int a = a0 + (int)(threadIdx.x & 63);
  bool hit = false;
  if (a < a1) {
    mine = ak[a];
    hit = !wb.misses(mine);
  } else {
    mine = AtomK{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  }
  return __ballot(hit);
}
__device__ __forceinline__ float lane_f(float v, int i) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), i));
}
__device__ __forceinline__ AtomK lane_atom(const AtomK& m, int i) {
  return AtomK{lane_f(m.w, i),  lane_f(m.mx, i), lane_f(m.my, i),   lane_f(m.mz, i),
               lane_f(m.hd, i), lane_f(m.c, i),  lane_f(m.hdm1, i), lane_f(m.rcut2, i)};
}

// ------------------------------------------------------------------ render

// f(s) = sum_n w_n exp(-u_n(s)) for every voxel; thread = one (y, x) column of a 16 x 16 tile
// (blockIdx.x), VPT planes (blockIdx.y). Each wave evaluates only the atoms whose cut
// ball meets its voxels (wave_hits); the others add exact zeros there. Atoms are summed in
// increasing index order.
template <int VPT>
__global__ __launch_bounds__(256) void k_render(const AtomK* __restrict__ ak, int n, int nx,
                                                int ny, int nz, float* __restrict__ f) {
  const TileXY t = tile_xy(blockIdx.x, nx, ny);
  const int nxy = nx * ny;
  const int x = min(t.x, nx - 1), y = min(t.y, ny - 1);
  const int z0 = blockIdx.y * VPT;
  const float fx = (float)x, fy = (float)y, fz0 = (float)z0;
  const WaveBox wb = wave_box(t, nx, ny, z0, min(z0 + VPT, nz) - 1);
  float acc[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) acc[j] = 0.f;
  for (int a0 = 0; a0 < n; a0 += 64) {
    AtomK mine;
    unsigned long long m = wave_hits(ak, a0, min(n, a0 + 64), wb, mine);
    while (m) {
      const int i = __builtin_ctzll(m);
      m &= m - 1;
      const AtomK k = lane_atom(mine, i);
      const float dx = fx - k.mx;
      const float dy = fy - k.my;
      const float dxy2 = fmaf(dx, dx, fmaf(dy, dy, kTinyR2));
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const float dz = (fz0 + (float)j) - k.mz;  // z - m_z of this voxel, whatever VPT is
        const float r2 = fmaf(dz, dz, dxy2);
        const float l = fast_log2(r2);
        const float up = fast_exp2(fmaf(k.hd, l, k.c));  // u * log2(e)
        const float g = fast_exp2(-up);
        acc[j] = fmaf(k.w, g, acc[j]);
      }
    }
  }
  if (!t.in) return;
  float* col = f + (size_t)z0 * nxy + (size_t)y * nx + x;
#pragma unroll
  for (int j = 0; j < VPT; ++j)
    if (z0 + j < nz) col[(size_t)j * nxy] = acc[j];
}

// ------------------------------------------------------------------ direct convolution

// z stride of the staged tile: >= RZ + KZ - 1, a multiple of 4 floats (128-bit reads) and an
// odd multiple of 4 so the 16 lanes of a 128-bit LDS read phase hit distinct banks.
constexpr int conv_lzp(int rz, int kz) {
  int l = (rz + kz - 1 + 3) / 4 * 4;
  return (l / 4) % 2 == 1 ? l : l + 4;
}

// out[z][y][x] = sum_{kz,ky,kx} W[ky][kx][kz] in[z + cz - kz][y + cy - ky][x + cx - kx],
// in = 0 outside the volume. Block = TX x TY threads over an output tile TX x TY x RZ; each
// thread keeps RZ outputs along z in registers. Taps are visited in passes of KZ (z) by kyc
// (y) by px (x); each pass stages the input sub-tile it needs in LDS as [ly][lx][lz] with a
// compile-time z stride, then for every (ky, kx) a thread reads one contiguous input column
// of RZ + KZ - 1 values and does RZ * KZ FMAs with wave-uniform (scalar) weights.
template <int TX, int TY, int RZ, int KZ, int EPI>
__global__ __launch_bounds__(TX* TY) void k_conv(
    const float* __restrict__ in, const float* __restrict__ wt, int px, int py, int pz, int kzp,
    int kyc, int nx, int ny, int nz, float* __restrict__ out, const float* __restrict__ yobs,
    double* __restrict__ dpart, float scale, long long idx_base, ArgPart* __restrict__ apart) {
  extern __shared__ float lds[];
  constexpr int NT = TX * TY;
  constexpr int LZ = RZ + KZ - 1;
  constexpr int LZP = conv_lzp(RZ, KZ);
  const int tid = threadIdx.x;
  const int tx = tid % TX;
  const int ty = tid / TX;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * RZ;
  const int cx = (px - 1) / 2, cy = (py - 1) / 2, cz = (pz - 1) / 2;
  const int LX = TX + px - 1;
  const size_t nxy = (size_t)nx * ny;

  float acc[RZ];
#pragma unroll
  for (int j = 0; j < RZ; ++j) acc[j] = 0.f;

  for (int kz0 = 0; kz0 < kzp; kz0 += KZ) {
    for (int ky0 = 0; ky0 < py; ky0 += kyc) {
      const int kyn = min(kyc, py - ky0);
      const int LY = TY + kyn - 1;
      const int ix0 = x0 + cx - px + 1;
      const int iy0 = y0 + cy - ky0 - kyn + 1;
      const int iz0 = z0 + cz - kz0 - KZ + 1;
      __syncthreads();
      // stage in[iz0 .. iz0+LZ) x [iy0 .. iy0+LY) x [ix0 .. ix0+LX) (zero outside) as
      // lds[(ly * LX + lx) * LZP + lz]
      const int nrows = LY * LZ;
      for (int row = tid / 64; row < nrows; row += NT / 64) {
        const int lz = row / LY;
        const int ly = row - lz * LY;
        const int gz = iz0 + lz, gy = iy0 + ly;
        const bool rin = gz >= 0 && gz < nz && gy >= 0 && gy < ny;
        const float* src = rin ? in + (size_t)gz * nxy + (size_t)gy * nx : in;
        float* dst = lds + (size_t)ly * LX * LZP + lz;
        for (int lx = tid & 63; lx < LX; lx += 64) {
          const int gx = ix0 + lx;
          dst[lx * LZP] = (rin && gx >= 0 && gx < nx) ? src[gx] : 0.f;
        }
      }
      __syncthreads();
      // blocked summation: each pass accumulates into fresh partials added to acc at the end
      float part[RZ];
#pragma unroll
      for (int j = 0; j < RZ; ++j) part[j] = 0.f;
      for (int kk = 0; kk < kyn; ++kk) {
        const int ky = ky0 + kk;
        const int ly = ty + kyn - 1 - kk;
        const float* wrow = wt + (size_t)ky * px * kzp + kz0;
        const float* lcol = lds + ((size_t)ly * LX + tx + px - 1) * LZP;
        for (int kx = 0; kx < px; ++kx) {
          float w[KZ];
#pragma unroll
          for (int t = 0; t < KZ; ++t) w[t] = wrow[(size_t)kx * kzp + t];
          const float4* c4 = reinterpret_cast<const float4*>(lcol - (size_t)kx * LZP);
          float v[LZP];
#pragma unroll
          for (int t = 0; t < LZP / 4; ++t) {
            const float4 q4 = c4[t];
            v[4 * t + 0] = q4.x;
            v[4 * t + 1] = q4.y;
            v[4 * t + 2] = q4.z;
            v[4 * t + 3] = q4.w;
          }
#pragma unroll
          for (int t = 0; t < KZ; ++t)
#pragma unroll
            for (int j = 0; j < RZ; ++j) part[j] = fmaf(w[t], v[j + KZ - 1 - t], part[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < RZ; ++j) acc[j] += part[j];
    }
  }

  const int x = x0 + tx, y = y0 + ty;
  const bool xy_in = x < nx && y < ny;
  if (EPI == kEpiPlain) {
    if (xy_in) {
#pragma unroll
      for (int j = 0; j < RZ; ++j)
        if (z0 + j < nz) out[(size_t)(z0 + j) * nxy + (size_t)y * nx + x] = acc[j];
    }
  } else if (EPI == kEpiResidual) {
    double ss = 0.0;
    if (xy_in) {
      float ssf = 0.f;
#pragma unroll
      for (int j = 0; j < RZ; ++j) {
        if (z0 + j < nz) {
          const size_t v = (size_t)(z0 + j) * nxy + (size_t)y * nx + x;
          const float rv = yobs[v] - acc[j];
          out[v] = rv;
          ssf = fmaf(rv, rv, ssf);
        }
      }
      ss = (double)ssf;
    }
    __shared__ double red[NT / 64];
    ss = shfl_sum_d(ss);
    if ((tid & 63) == 0) red[tid / 64] = ss;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int i = 0; i < NT / 64; ++i) t += red[i];
      dpart[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
    }
  } else {  // kEpiArgmax
    float bv = -INFINITY;
    long long bi = 0x7fffffffffffffffLL;
    if (xy_in) {
#pragma unroll
      for (int j = 0; j < RZ; ++j) {
        if (z0 + j < nz) {
          const size_t v = (size_t)(z0 + j) * nxy + (size_t)y * nx + x;
          const float e = acc[j] * scale;
          if (out) out[v] = e;
          const long long gi = idx_base + (long long)v;
          if (arg_better(e, gi, bv, bi)) {
            bv = e;
            bi = gi;
          }
        }
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const float ov = __shfl_xor(bv, o, 64);
      const long long oi = __shfl_xor(bi, o, 64);
      if (arg_better(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
      }
    }
    __shared__ float rv[NT / 64];
    __shared__ long long ri[NT / 64];
    if ((tid & 63) == 0) {
      rv[tid / 64] = bv;
      ri[tid / 64] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      for (int i = 1; i < NT / 64; ++i)
        if (arg_better(rv[i], ri[i], bv, bi)) {
          bv = rv[i];
          bi = ri[i];
        }
      ArgPart ap;
      ap.val = bv;
      ap.pad = 0;
      ap.idx = bi;
      apart[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = ap;
    }
  }
}

// ------------------------------------------------------------------ convolution on MFMA

typedef float floatx4 __attribute__((ext_vector_type(4)));

// out[z][y][x] = sum_{kz,ky,kx} W[kz][ky][kx] in[z + cz - kz][y + cy - ky][x + cx - kx] on the
// matrix cores (pz <= 16, px * py <= 4 * STEPS; amat holds STEPS steps, zero past the taps).
// A block owns 16 consecutive x of 4 rows y and streams the input planes zi = 0 .. nz-1.
// For each plane the in-plane taps form the K dimension of a chain of
// v_mfma_f32_16x16x4_f32 with A = W[kz][tap] (registers), B[tap][n] =
// in[zi][y + cy - ky][x0 + n + cx - kx] and accumulator rows indexed by kz: row j holds a
// partial sum of output plane zi - cz + j.
//
// Two accumulators take the even (E) and the odd (O) input planes, so every wave runs two
// independent MFMA chains per iteration of two planes. After its plane, an accumulator's rows
// 0 and 1 hold its final share of two output planes; they are read out and the rows roll up by
// two (one 16-lane shuffle per two rows). Output plane 2t - cz is E's row 0 of iteration t plus
// O's row 1 of iteration t - 1; plane 2t - cz + 1 is E's row 1 plus O's row 0 of iteration t.
// Each row is served by two waves (8 waves per block, two per SIMD) that split the taps; the
// second hands its shares to the first through LDS. The block stages each plane's
// (16 + px - 1) x (4 + py - 1) input patch (zero outside the volume) in a ring of 8 LDS
// buffers: planes 2t + 4 and 2t + 5 are stored at iteration t from registers loaded one
// iteration earlier, with one barrier per iteration.
// Accumulator layout (16x16x4 f32): lane l holds rows 4 (l / 16) + 0..3 of column l % 16.
//
// Output region: tiles (tx0 + blockIdx.x, ty0 + blockIdx.y) and output planes
// [zlo + blockIdx.z * zchunk, min(zhi, that + zchunk)); a block streams the input planes from
// cz below its first output plane (rounded down to an even plane, never below 0). The whole
// volume is tx0 = ty0 = 0, zlo = 0, zhi = zchunk = nz.
template <int STEPS, int EPI>
__global__ __launch_bounds__(512) void k_conv_mfma(
    const float* __restrict__ in, const float* __restrict__ amat, int px, int py, int pz,
    int nx, int ny, int nz, int tx0, int ty0, int zlo, int zhi, int zchunk,
    float* __restrict__ out, const float* __restrict__ yobs, double* __restrict__ dpart) {
  constexpr int NBUF = 8;
  constexpr int PLANE = kMfmaPatchMax;
  constexpr int SH = (STEPS + 1) / 2;  // taps of the first half (the second gets the rest)
  __shared__ float patch[NBUF][PLANE];
  __shared__ float xch[2][4][4][16];  // [t & 1][row][E0, E1, O0, O1][x]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int rowi = wave & 3, half = wave >> 2;
  const int n = lane & 15, g = lane >> 4;
  const int x0 = (tx0 + (int)blockIdx.x) * 16, y0 = (ty0 + (int)blockIdx.y) * 4;
  const int y = y0 + rowi, x = x0 + n;
  const int cx = (px - 1) / 2, cy = (py - 1) / 2, cz = (pz - 1) / 2;
  const size_t nxy = (size_t)nx * ny;
  const int PW = 16 + px - 1, PH = 4 + py - 1, PN = PW * PH;
  const int oc0 = zlo + (int)blockIdx.z * zchunk, oc1 = min(zhi, oc0 + zchunk);
  // first input plane streamed: even, so every output plane sees the same even / odd split and
  // summation order as in a whole-volume launch (bit-identical results)
  const int zb = max(0, oc0 - cz) & ~1;

  // staging: thread owns patch element tid (in-plane offset, -1 = zero)
  const bool lown = tid < PN;
  int goff = -1;
  if (lown) {
    const int row = tid / PW, col = tid - (tid / PW) * PW;
    const int iy = y0 + cy - (py - 1) + row, ix = x0 + cx - (px - 1) + col;
    if (iy >= 0 && iy < ny && ix >= 0 && ix < nx) goff = iy * nx + ix;
  }
  auto fetch = [&](int l) -> float {  // input plane zb + l
    const int plane = zb + l;
    const bool ok = plane < nz && goff >= 0;
    const float t = in[(size_t)min(plane, nz - 1) * nxy + max(goff, 0)];
    return ok ? t : 0.f;
  };
  // this wave's taps: steps [s0, s0 + SH) of the plan (past STEPS: zero weights)
  const int s0 = half * SH;
  float a[SH];
  int boff[SH];
#pragma unroll
  for (int s = 0; s < SH; ++s) {
    const int st = s0 + s;
    a[s] = st < STEPS ? amat[st * 64 + lane] : 0.f;
    const int k = 4 * st + g;
    int o = 0;
    if (st < STEPS && k < px * py) {
      const int ky = k / px, kx = k - ky * px;
      o = (rowi + py - 1 - ky) * PW + n + px - 1 - kx;
    }
    boff[s] = o;
  }
  // prologue: planes 0-3 in LDS, planes 4 and 5 in registers
  if (lown) {
#pragma unroll
    for (int p = 0; p < 4; ++p) patch[p][tid] = fetch(p);
  }
  float sa = fetch(4), sb = fetch(5);
  const bool out_lane = half == 0 && g == 0 && x < nx && y < ny;
  const size_t col = (size_t)min(y, ny - 1) * nx + min(x, nx - 1);
  // observed y at this iteration's two output planes (residual epilogue), one iteration ahead
  auto yat = [&](int o) -> float { return yobs[(size_t)min(max(o, 0), nz - 1) * nxy + col]; };
  float y1 = 0.f, y2 = 0.f;
  if (EPI == kEpiResidual) {
    y1 = yat(zb - cz);
    y2 = yat(zb + 1 - cz);
  }
  __syncthreads();

  floatx4 accE = {0.f, 0.f, 0.f, 0.f}, accO = {0.f, 0.f, 0.f, 0.f};
  float ssf = 0.f, ob_prev = 0.f;
  // iteration t completes output planes zb - cz + 2t and the next; the last one reaches oc1 - 1
  const int T = oc1 > oc0 ? (oc1 - 1 - (zb - cz)) / 2 + 1 : 0;
  auto roll2 = [&](floatx4& acc) {
    const float u0 = __shfl_down(acc[0], 16, 64);
    const float u1 = __shfl_down(acc[1], 16, 64);
    acc[0] = acc[2];
    acc[1] = acc[3];
    acc[2] = g < 3 ? u0 : 0.f;
    acc[3] = g < 3 ? u1 : 0.f;
  };
  // one iteration: planes 2t (E) and 2t + 1 (O); FULL: both planes inside the volume
  auto iteration = [&](int t, auto full) {
    constexpr bool FULL = decltype(full)::value;
    const int ze = 2 * t, zo = 2 * t + 1;  // local input planes (absolute: zb + local)
    const float na = fetch(ze + 6), nb = fetch(ze + 7);
    const float* bufE = patch[ze & (NBUF - 1)];
    const float* bufO = patch[zo & (NBUF - 1)];
    if (FULL) {
      float bE[SH], bO[SH];
#pragma unroll
      for (int s = 0; s < SH; ++s) {
        bE[s] = bufE[boff[s]];
        bO[s] = bufO[boff[s]];
      }
#pragma unroll
      for (int s = 0; s < SH; ++s) {
        accE = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bE[s], accE, 0, 0, 0);
        accO = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bO[s], accO, 0, 0, 0);
      }
    } else if (zb + ze < nz) {
      float bE[SH];
#pragma unroll
      for (int s = 0; s < SH; ++s) bE[s] = bufE[boff[s]];
#pragma unroll
      for (int s = 0; s < SH; ++s)
        accE = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bE[s], accE, 0, 0, 0);
    }
    const float e0 = accE[0], e1 = accE[1], o0 = accO[0], o1 = accO[1];
    roll2(accE);
    roll2(accO);
    if (half == 1 && g == 0) {
      float(*xc)[16] = xch[t & 1][rowi];
      xc[0][n] = e0;
      xc[1][n] = e1;
      xc[2][n] = o0;
      xc[3][n] = o1;
    }
    if (lown) {
      patch[(ze + 4) & (NBUF - 1)][tid] = sa;
      patch[(ze + 5) & (NBUF - 1)][tid] = sb;
    }
    sa = na;
    sb = nb;
    __syncthreads();
    if (half == 0) {
      // output planes 2t - cz and 2t - cz + 1
      const float(*xc)[16] = xch[t & 1][rowi];
      const float E0 = e0 + xc[0][n], E1 = e1 + xc[1][n];
      const float O0 = o0 + xc[2][n], O1 = o1 + xc[3][n];
      const float v1 = E0 + ob_prev, v2 = E1 + O0;
      ob_prev = O1;
      const int p1 = zb - cz + 2 * t, p2 = p1 + 1;
      float yn1 = 0.f, yn2 = 0.f;
      if (EPI == kEpiResidual) {
        yn1 = yat(p1 + 2);
        yn2 = yat(p2 + 2);
      }
      if (out_lane) {
        if (p1 >= oc0 && p1 < oc1) {
          const size_t v = (size_t)p1 * nxy + col;
          if (EPI != kEpiResidual) {
            out[v] = v1;
          } else {
            const float rv = y1 - v1;
            out[v] = rv;
            ssf = fmaf(rv, rv, ssf);
          }
        }
        if (p2 >= oc0 && p2 < oc1) {
          const size_t v = (size_t)p2 * nxy + col;
          if (EPI != kEpiResidual) {
            out[v] = v2;
          } else {
            const float rv = y2 - v2;
            out[v] = rv;
            ssf = fmaf(rv, rv, ssf);
          }
        }
      }
      if (EPI == kEpiResidual) {
        y1 = yn1;
        y2 = yn2;
      }
    }
  };
  const int TF = min(T, max(0, (nz - zb) / 2));  // iterations with both planes in the volume
  int t = 0;
  for (; t < TF; ++t) iteration(t, std::true_type{});
  for (; t < T; ++t) iteration(t, std::false_type{});
  if (EPI == kEpiResidual && half == 0) {
    double ss = shfl_sum_d((double)ssf);
    if (lane == 0)
      dpart[(((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 4 + rowi] =
          ss;
  }
}

// ------------------------------------------------------------------ gradient sums at points

// The per-atom sums of eta and its gradient at a few points (at most kAtomArgs unit-weight
// atoms, by value in `args`) in one launch: block = 256 (y, x) columns x VPT z of the region
// (ntile_xy tiles of 16 x 16 columns from tile (rx0, ry0), rtx per row, z tiles from rz0).
// Each wave evaluates only the atoms whose cut ball meets its 16 x 4 x VPT voxels (the other
// terms are exact zeros) and the tile partial gpart[tile][atom][0..5] = (S_g, S_u, S_l, S_mx,
// S_my, S_mz) is the four wave sums added in wave order; the last block to finish (ticket
// counter) sums the tile partials over tiles in a fixed order, in float64, into
// sums_out[6 a + c]. Nothing is left for the host but one synchronisation; sums_out may be
// pinned host memory: the kernel's writes to it are visible once the stream has been
// synchronised.
template <int VPT>
__global__ __launch_bounds__(kGradThreads) void k_grad_points(AtomArgs args, int n,
                                                              const float* __restrict__ q, int nx,
                                                              int ny, int nz, int ntile_xy,
                                                              int rx0, int ry0, int rtx, int rz0,
                                                              float* __restrict__ gpart,
                                                              int* __restrict__ ticket,
                                                              double* __restrict__ sums_out,
                                                              SigArgs sig) {
  constexpr int NW = kGradThreads / 64;
  static_assert(kAtomArgs <= 64, "one atom list per wave");
  __shared__ float red[NW][kAtomArgs][6];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int tile = blockIdx.x;
  const int txy = tile % ntile_xy;
  const int tz = rz0 + tile / ntile_xy;
  const int nxy = nx * ny;
  const TileXY t = tile_xy(txy, nx, ny, rx0, ry0, rtx);
  const bool pin = t.in;
  const int x = min(t.x, nx - 1), y = min(t.y, ny - 1);
  const int p = y * nx + x;
  const int z0 = tz * VPT;
  float qv[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j)
    qv[j] = (pin && z0 + j < nz) ? q[(size_t)(z0 + j) * nxy + p] : 0.f;
  const float fx = (float)x, fy = (float)y, fz0 = (float)z0;
  const int wave = tid / 64;
  const WaveBox wb = wave_box(t, nx, ny, z0, min(z0 + VPT, nz) - 1);
  for (int i = 0; i < n; ++i) {
    const AtomK k = args.a[i];
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f;
    if (!wb.misses(k)) {
      const float dx = fx - k.mx;
      const float dy = fy - k.my;
      const float dxy2 = fmaf(dx, dx, fmaf(dy, dy, kTinyR2));
      float sg = 0.f, su = 0.f, sl = 0.f, sc = 0.f, scz = 0.f;
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const float dz = (fz0 + (float)j) - k.mz;
        const float r2 = fmaf(dz, dz, dxy2);
        const float l = fast_log2(r2);
        const float vp = fast_exp2(fmaf(k.hdm1, l, k.c));  // u log2(e) / r^2
        const float up = vp * r2;                           // u log2(e)
        const float g = fast_exp2(-up);
        const float qg = qv[j] * g;
        sg += qg;
        const float qgu = qg * up;
        su += qgu;
        sl = fmaf(qgu, l, sl);
        const float c2 = qg * vp;
        sc += c2;
        scz = fmaf(c2, dz, scz);
      }
      s0 = wave_sum(sg);
      s1 = wave_sum(su);
      s2 = wave_sum(sl);
      s3 = wave_sum(sc * dx);
      s4 = wave_sum(sc * dy);
      s5 = wave_sum(scz);
    }
    if (lane == 0) {
      float* rr = red[wave][i];
      rr[0] = s0;
      rr[1] = s1;
      rr[2] = s2;
      rr[3] = s3;
      rr[4] = s4;
      rr[5] = s5;
    }
  }
  __syncthreads();
  for (int e = tid; e < n * 6; e += kGradThreads) {
    const int aa = e / 6, c = e - aa * 6;
    float v = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += red[w][aa][c];
    gpart[(size_t)tile * n * 6 + e] = v;
  }
  __shared__ int is_last;
  __shared__ double part[kGradThreads];
  static_assert(kAtomArgs * 6 <= 64, "the sums must be written by the first wave");
  // only the first wave wrote partials, so only it releases them (a device-scope release
  // writes back the L2; four per block cost more than the sums)
  if (tid < 64) __threadfence();
  __syncthreads();
  if (tid == 0) is_last = atomicAdd(ticket, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (is_last) {
    __threadfence();
    // the whole block sums the tiles: slice sl of (atom, component) pr takes the tiles
    // tt = sl (mod nsl), then one thread per pr adds its slices in order (fixed order)
    const int pairs = n * 6, ntiles = gridDim.x;
    const int nsl = kGradThreads / pairs;
    if (tid < pairs * nsl) {
      const int pr = tid % pairs, sl = tid / pairs;
      double acc = 0.0;
#pragma unroll 4
      for (int tt = sl; tt < ntiles; tt += nsl) acc += (double)gpart[(size_t)tt * pairs + pr];
      part[sl * pairs + pr] = acc;
    }
    __syncthreads();
    if (tid < pairs) {
      double S = 0.0;
      for (int sl = 0; sl < nsl; ++sl) S += part[sl * pairs + tid];
      sums_out[tid] = S;
    }
    if (tid == 0) *ticket = 0;  // ready for the next launch
    signal_host(sig, 1);
  }
}

// ------------------------------------------------------------------ gradient sums per item

// The gradient sums of a (C, grad C) evaluation with the work spread evenly over the blocks:
// an item is one atom on one 16 x 16 x 16 volume tile that meets the bounding box of the atom's
// cut ball, grown by a voxel; block b takes items b, b + gridDim.x, ... (every item costs
// about the same, where per-tile atom lists would leave the blocks over dense regions with
// many atoms each). Items go atom by atom (the atom's tiles with x fastest), so atom a owns
// items [start[a], start[a + 1]); every block computes these offsets itself (the atom
// constants are all it needs), keeping the atoms and their tile ranges in LDS (up to
// kItemsLdsAtoms atoms; beyond, they are read again per item), and block 0 stores the offsets
// in item_start for launch_grad_finalize. Item i writes gpart[6 i + c] = (S_g, S_u, S_l, S_mx,
// S_my, S_mz) of its atom over its tile: the four wave sums added in wave order (a wave whose
// 16 x 4 x 16 box the cut ball misses adds exact zeros and skips them). No partial depends on
// gridDim.x.
struct ItemBox {
  int tx, ty, tz;  // first tile per axis
  int cx, cy, cz;  // tiles per axis (0 when the cut ball misses the volume)
};
constexpr int kItemsLdsAtoms = 1024;
__device__ __forceinline__ void item_axis(float m, float R, int n, int& t0, int& cnt) {
  const float lo = fmaxf(0.f, floorf(m - R) - 1.f);
  const float hi = fminf((float)(n - 1), ceilf(m + R) + 1.f);
  if (lo <= hi) {
    t0 = (int)lo / kTile;
    cnt = (int)hi / kTile - t0 + 1;
  } else {
    t0 = 0;
    cnt = 0;
  }
}
__device__ __forceinline__ ItemBox item_box(const AtomK& k, int nx, int ny, int nz) {
  const float R = sqrtf(k.rcut2);
  ItemBox b;
  item_axis(k.mx, R, nx, b.tx, b.cx);
  item_axis(k.my, R, ny, b.ty, b.cy);
  item_axis(k.mz, R, nz, b.tz, b.cz);
  return b;
}

__global__ __launch_bounds__(kGradThreads) void k_grad_items(const AtomK* __restrict__ ak, int n,
                                                             const float* __restrict__ q, int nx,
                                                             int ny, int nz,
                                                             float* __restrict__ gpart,
                                                             int* __restrict__ item_start) {
  constexpr int VPT = kTile, NW = kGradThreads / 64;
  // dynamic LDS: item offsets [n + 1], then (cache) atoms [n] and their tile ranges [n]
  extern __shared__ __align__(16) unsigned char items_lds[];
  const bool cache = n <= kItemsLdsAtoms;
  int* starts = reinterpret_cast<int*>(items_lds);
  AtomK* atoms = reinterpret_cast<AtomK*>(items_lds + ((size_t)(n + 1) * sizeof(int) + 15) / 16 * 16);
  ItemBox* boxes = reinterpret_cast<ItemBox*>(atoms + n);
  __shared__ float red[NW][6];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < 64) {  // item offsets: a scan of the per-atom tile counts, 64 atoms at a time
    int carry = 0;
    for (int a0 = 0; a0 < n; a0 += 64) {
      const int a = a0 + lane;
      int c = 0;
      if (a < n) {
        const AtomK k = ak[a];
        const ItemBox b = item_box(k, nx, ny, nz);
        if (cache) {
          atoms[a] = k;
          boxes[a] = b;
        }
        c = b.cx * b.cy * b.cz;
      }
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(c, o, 64);
        if (lane >= o) c += v;
      }
      if (a < n) starts[a + 1] = carry + c;
      carry += __shfl(c, 63, 64);
    }
    if (lane == 0) starts[0] = 0;
  }
  __syncthreads();
  const int total = starts[n];
  if (blockIdx.x == 0)
    for (int a = tid; a <= n; a += kGradThreads) item_start[a] = starts[a];
  const int nxy = nx * ny;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    // its atom: the last a with starts[a] <= item (starts[n] = total > item)
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (starts[mid] <= item) lo = mid;
      else hi = mid;
    }
    const AtomK k = cache ? atoms[lo] : ak[lo];
    const ItemBox b = cache ? boxes[lo] : item_box(k, nx, ny, nz);
    int local = item - starts[lo];
    const int ix = local % b.cx;
    local /= b.cx;
    const int iy = local % b.cy, iz = local / b.cy;
    const int x0 = (b.tx + ix) * kTile, y0 = (b.ty + iy) * kTile, z0 = (b.tz + iz) * VPT;
    const int xx = x0 + (tid & (kTile - 1)), yy = y0 + tid / kTile;
    const bool pin = xx < nx && yy < ny;
    const int x = min(xx, nx - 1), y = min(yy, ny - 1);
    const int y0w = y0 + wave * (64 / kTile);
    const WaveBox wb{(float)x0,
                     (float)min(x0 + kTile - 1, nx - 1),
                     (float)min(y0w, ny - 1),
                     (float)min(y0w + 64 / kTile - 1, ny - 1),
                     (float)z0,
                     (float)max(min(z0 + VPT, nz) - 1, z0)};
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f, s5 = 0.f;
    if (!wb.misses(k)) {
      float qv[VPT];
#pragma unroll
      for (int j = 0; j < VPT; ++j)
        qv[j] = (pin && z0 + j < nz) ? q[(size_t)(z0 + j) * nxy + (size_t)y * nx + x] : 0.f;
      const float fx = (float)x, fy = (float)y, fz0 = (float)z0;
      const float dx = fx - k.mx;
      const float dy = fy - k.my;
      const float dxy2 = fmaf(dx, dx, fmaf(dy, dy, kTinyR2));
      float sg = 0.f, su = 0.f, sl = 0.f, sc = 0.f, scz = 0.f;
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        const float dz = (fz0 + (float)j) - k.mz;
        const float r2 = fmaf(dz, dz, dxy2);
        const float l = fast_log2(r2);
        const float vp = fast_exp2(fmaf(k.hdm1, l, k.c));  // u log2(e) / r^2
        const float up = vp * r2;                           // u log2(e)
        const float g = fast_exp2(-up);
        const float qg = qv[j] * g;
        sg += qg;
        const float qgu = qg * up;
        su += qgu;
        sl = fmaf(qgu, l, sl);
        const float c2 = qg * vp;
        sc += c2;
        scz = fmaf(c2, dz, scz);
      }
      s0 = wave_sum(sg);
      s1 = wave_sum(su);
      s2 = wave_sum(sl);
      s3 = wave_sum(sc * dx);
      s4 = wave_sum(sc * dy);
      s5 = wave_sum(scz);
    }
    if (lane == 0) {
      red[wave][0] = s0;
      red[wave][1] = s1;
      red[wave][2] = s2;
      red[wave][3] = s3;
      red[wave][4] = s4;
      red[wave][5] = s5;
    }
    __syncthreads();
    if (tid < 6) {
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) v += red[w][tid];
      gpart[(size_t)item * 6 + tid] = v;
    }
    __syncthreads();  // red is rewritten by the next item
  }
}

// Block per atom (blockIdx.x < n) plus one block for the loss (blockIdx.x == n).
// Partials in tile layout (gpart[(t n + a) 6 + c], t < ntiles) or, with item_start, in item
// layout (atom a's partials at gpart[6 i + c], item_start[a] <= i < item_start[a + 1]).
__global__ __launch_bounds__(256) void k_grad_finalize(
    const float* __restrict__ gpart, int ntiles, const int* __restrict__ item_start, int n,
    const double* __restrict__ loss_part, int nloss, const sfw_atom* __restrict__ atoms,
    float lambda, double* __restrict__ sums, sfw_atom* __restrict__ grad_out,
    double* __restrict__ loss_out, int vjp, SigArgs sig) {
  __shared__ double red[6][4];
  const int tid = threadIdx.x;
  const int a = blockIdx.x;
  if (a < n) {
    double s[6] = {0, 0, 0, 0, 0, 0};
    if (item_start) {
      const int i1 = item_start[a + 1];
      for (int i = item_start[a] + tid; i < i1; i += 256) {
        const float* g = gpart + (size_t)i * 6;
#pragma unroll
        for (int c = 0; c < 6; ++c) s[c] += (double)g[c];
      }
    } else {
      for (int t = tid; t < ntiles; t += 256) {
        const float* g = gpart + ((size_t)t * n + a) * 6;
#pragma unroll
        for (int c = 0; c < 6; ++c) s[c] += (double)g[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double v = shfl_sum_d(s[c]);
      if ((tid & 63) == 0) red[c][tid / 64] = v;
    }
    __syncthreads();
    if (tid == 0) {
      double S[6];
      for (int c = 0; c < 6; ++c) S[c] = red[c][0] + red[c][1] + red[c][2] + red[c][3];
      for (int c = 0; c < 6; ++c) sums[(size_t)a * 6 + c] = S[c];
      if (grad_out) {
        const sfw_atom at = atoms[a];
        const double w = at.w, d = at.d, sg = at.sigma;
        // dC/dtheta = lambda [theta = w] - sum_s q df/dtheta; the vector-Jacobian product of
        // the forward model is sum_s q df/dtheta itself (lambda = 0, opposite sign)
        const double sgn = vjp ? -1.0 : 1.0;
        const double lam = vjp ? 0.0 : (double)lambda;
        sfw_atom g;
        g.w = (float)(sgn * (lam - S[0]));
        const double fm = -sgn * w * d * kLn2;
        g.mx = (float)(fm * S[3]);
        g.my = (float)(fm * S[4]);
        g.mz = (float)(fm * S[5]);
        g.sigma = (float)(-sgn * w * (d / sg) * kLn2 * S[1]);
        g.d = (float)(sgn * w * (0.5 * kLn2 * kLn2 * S[2] - log(sg) * kLn2 * S[1]));
        grad_out[a] = g;
      }
    }
  } else {
    double s = 0.0;
    if (loss_part)
      for (int t = tid; t < nloss; t += 256) s += loss_part[t];
    s = shfl_sum_d(s);
    if ((tid & 63) == 0) red[0][tid / 64] = s;
    __syncthreads();
    if (tid == 0) {
      const double ss = red[0][0] + red[0][1] + red[0][2] + red[0][3];
      double wsum = 0.0;
      if (atoms)
        for (int i = 0; i < n; ++i) wsum += (double)atoms[i].w;
      const double loss = 0.5 * ss + (double)lambda * wsum;
      sums[(size_t)n * 6] = loss;
      sums[(size_t)n * 6 + 1] = 0.5 * ss;
      if (loss_out) *loss_out = loss;
    }
  }
  signal_host(sig, gridDim.x);
}

// ------------------------------------------------------------------ certificate maximum

__global__ __launch_bounds__(1024) void k_argmax_final(const ArgPart* __restrict__ apart,
                                                       int nparts, int nx, int ny, int nz, int nd,
                                                       sfw_argmax* __restrict__ best,
                                                       sfw_argmax* __restrict__ best_host,
                                                       SigArgs sig) {
  const int tid = threadIdx.x;
  float bv = -INFINITY;
  long long bi = 0x7fffffffffffffffLL;
  // eight partials in flight per thread: the 128 x 128 x 64 certificate's 6,144 in one round
  // (ties go to the lower index, so the order of the comparisons changes no result)
  for (int i0 = tid; i0 < nparts; i0 += 8 * 1024) {
    ArgPart ap[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * 1024;
      if (i < nparts) {
        ap[u] = apart[i];
      } else {
        ap[u].val = -INFINITY;
        ap[u].idx = 0x7fffffffffffffffLL;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (arg_better(ap[u].val, ap[u].idx, bv, bi)) {
        bv = ap[u].val;
        bi = ap[u].idx;
      }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(bv, o, 64);
    const long long oi = __shfl_xor(bi, o, 64);
    if (arg_better(ov, oi, bv, bi)) {
      bv = ov;
      bi = oi;
    }
  }
  __shared__ float rv[16];
  __shared__ long long ri[16];
  if ((tid & 63) == 0) {
    rv[tid / 64] = bv;
    ri[tid / 64] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 1; i < 16; ++i)
      if (arg_better(rv[i], ri[i], bv, bi)) {
        bv = rv[i];
        bi = ri[i];
      }
    sfw_argmax b;
    b.eta = bv;
    const long long V = (long long)nx * ny * nz;
    long long v = bi % V;
    const long long slice = bi / V;
    b.i_sigma = (int)(slice / nd);
    b.i_d = (int)(slice % nd);
    b.z = (int)(v / ((long long)nx * ny));
    v -= (long long)b.z * nx * ny;
    b.y = (int)(v / nx);
    b.x = (int)(v - (long long)b.y * nx);
    *best = b;
    if (best_host) *best_host = b;  // pinned host memory
  }
  signal_host(sig, 1);
}

// ------------------------------------------------------------------ LASSO dot products

// A LASSO column is valid on its box {x0, x1, y0, y1, z0, z1} (half-open, from slot_box) and
// stands for zero elsewhere: the slot may hold stale values there.
struct Box6 {
  int x0, x1, y0, y1, z0, z1;
};
__device__ __forceinline__ Box6 slot_box_of(const int* __restrict__ slot_box, int slot) {
  const int* b = slot_box + 6 * slot;
  return Box6{b[0], b[1], b[2], b[3], b[4], b[5]};
}
__device__ __forceinline__ bool in_box(const Box6& b, int x, int y, int z) {
  return x >= b.x0 && x < b.x1 && y >= b.y0 && y < b.y1 && z >= b.z0 && z < b.z1;
}
constexpr Box6 kBoxAll{0, 0x7fffffff, 0, 0x7fffffff, 0, 0x7fffffff};

// slot of column c: the first kSlotArgs come in the kernel arguments, the rest from device
// memory (only read when the support is longer)
__device__ __forceinline__ int slot_of(const SlotArgs& sa, const int* slots, int c) {
  return c < kSlotArgs ? sa.s[c] : slots[c];
}

// dpart[block][c] = partial sum over the block's voxels of a * cols[c] (c < k), a * y (c = k),
// in flat voxel order over the whole volume: a is valid on abox and column c on its own box
// (slot_box), and a product counts only where both are valid. Float32 products, float64
// accumulation, fixed-order block reduction. Used where the Gram-row box kernel does not
// apply (a column without a box, or rows that are not a multiple of four floats).
constexpr int kDotsHold = 4;
constexpr int kDotsCols = 4;

__device__ __forceinline__ double dot4(const float4& a, const float4& b) {
  return (double)(a.x * b.x) + (double)(a.y * b.y) + (double)(a.z * b.z) + (double)(a.w * b.w);
}

__global__ __launch_bounds__(256) void k_dots(const float* __restrict__ a, Box6 abox,
                                              const float* __restrict__ cols,
                                              SlotArgs sa, const int* __restrict__ slots,
                                              const int* __restrict__ slot_box, int k,
                                              size_t colstride, const float* __restrict__ y,
                                              int nx, int ny, size_t nvox,
                                              double* __restrict__ dpart) {
  __shared__ double red[kDotsCols][4];
  const int tid = threadIdx.x;
  const size_t stride = (size_t)gridDim.x * 256;
  for (int c0 = 0; c0 <= k; c0 += kDotsCols) {
    const int nc = min(kDotsCols, k + 1 - c0);
    const float* b[kDotsCols];
    Box6 bb[kDotsCols];
#pragma unroll
    for (int u = 0; u < kDotsCols; ++u) {
      const int c = min(c0 + u, k);
      const int sl = c < k ? slot_of(sa, slots, c) : 0;
      b[u] = c < k ? cols + (size_t)sl * colstride : y;
      bb[u] = c < k ? slot_box_of(slot_box, sl) : kBoxAll;
    }
    double s[kDotsCols] = {0.0, 0.0, 0.0, 0.0};
    for (size_t v = (size_t)blockIdx.x * 256 + tid; v < nvox; v += stride) {
      const size_t row = v / (size_t)nx;
      const int x = (int)(v - row * (size_t)nx);
      const int yy = (int)(row % (size_t)ny), zz = (int)(row / (size_t)ny);
      if (!in_box(abox, x, yy, zz)) continue;
      const float av = a[v];
#pragma unroll
      for (int u = 0; u < kDotsCols; ++u)
        if (in_box(bb[u], x, yy, zz)) s[u] += (double)(av * b[u][v]);
    }
#pragma unroll
    for (int u = 0; u < kDotsCols; ++u) {
      const double t = shfl_sum_d(s[u]);
      if ((tid & 63) == 0) red[u][tid / 64] = t;
    }
    __syncthreads();
    if (tid < nc)
      dpart[(size_t)blockIdx.x * (k + 1) + c0 + tid] =
          red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
    __syncthreads();
  }
}

// Gram rows of up to kDotsRows columns in one launch (blockIdx.z = row r): for row r, column
// a_r over its box (a_r is valid there and stands for zero elsewhere), partials
// dpart[part0_r + blockIdx.x][c] = sum over the box of a_r * col_c (c < k: cached column
// slot(c), counted only inside its own box; c = k: y) for the columns of chunk blockIdx.y (cpb
// per chunk), blockIdx.x < nbx_r. The box is rows (y, z) of bw4 float4 starting at x0 (x0, nx,
// the column stride and every column box's x bounds multiples of 4, so a float4 lies wholly
// inside or outside a box); a thread keeps its kDotsHold float4 of a_r in registers across
// the columns. A row's partials do not depend on the other rows of the launch.
struct DotsRow {
  const float* a;
  int x0, bw4, y0, bh, z0, nrows;  // box: nrows = bh * depth rows of bw4 float4
  int nbx, part0;                  // blocks of the row, its first partial
};
struct DotsRows {
  DotsRow r[kDotsRows];
};
__global__ __launch_bounds__(256) void k_dots_box(DotsRows rows, const float* __restrict__ cols,
                                                  SlotArgs sa, const int* __restrict__ slots,
                                                  const int* __restrict__ slot_box,
                                                  int k, size_t colstride,
                                                  const float* __restrict__ y,
                                                  int nx, int ny, int cpb,
                                                  double* __restrict__ dpart) {
  const DotsRow R = rows.r[blockIdx.z];
  if ((int)blockIdx.x >= R.nbx) return;  // the whole block: the row needs fewer blocks
  __shared__ double red[kDotsCols][4];
  const int tid = threadIdx.x;
  const int E = R.nrows * R.bw4;
  const int stride = R.nbx * 256;
  const int e0 = blockIdx.x * 256 + tid;
  const float* a = R.a;
  float4 ah[kDotsHold];
  size_t vh[kDotsHold];
  int xh[kDotsHold], yh[kDotsHold], zh[kDotsHold];
#pragma unroll
  for (int h = 0; h < kDotsHold; ++h) {
    const int e = e0 + h * stride;
    const bool ok = e < E;
    const int row = ok ? e / R.bw4 : 0;
    const int q = ok ? e - row * R.bw4 : 0;
    const int yy = R.y0 + row % R.bh, zz = R.z0 + row / R.bh;
    xh[h] = R.x0 + 4 * q;
    yh[h] = yy;
    zh[h] = zz;
    vh[h] = ((size_t)zz * ny + yy) * nx + R.x0 + 4 * q;
    ah[h] = ok ? *reinterpret_cast<const float4*>(a + vh[h]) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  const int cb = blockIdx.y * cpb, ce = min(k + 1, cb + cpb);
  for (int c0 = cb; c0 < ce; c0 += kDotsCols) {
    const int nc = min(kDotsCols, ce - c0);
    const float* b[kDotsCols];
    Box6 bb[kDotsCols];
#pragma unroll
    for (int u = 0; u < kDotsCols; ++u) {
      const int c = min(c0 + u, ce - 1);
      const int sl = c < k ? slot_of(sa, slots, c) : 0;
      b[u] = c < k ? cols + (size_t)sl * colstride : y;
      bb[u] = c < k ? slot_box_of(slot_box, sl) : kBoxAll;
    }
    double s[kDotsCols] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < kDotsHold; ++h) {
      if (e0 + h * stride < E) {
        float4 bv[kDotsCols];
#pragma unroll
        for (int u = 0; u < kDotsCols; ++u)
          bv[u] = in_box(bb[u], xh[h], yh[h], zh[h])
                      ? *reinterpret_cast<const float4*>(b[u] + vh[h])
                      : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < kDotsCols; ++u) s[u] += dot4(ah[h], bv[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kDotsCols; ++u) {
      const double t = shfl_sum_d(s[u]);
      if ((tid & 63) == 0) red[u][tid / 64] = t;
    }
    __syncthreads();
    if (tid < nc)
      dpart[(size_t)(R.part0 + blockIdx.x) * (k + 1) + c0 + tid] =
          red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
    __syncthreads();
  }
}

// Row r = blockIdx.x of a k_dots_box launch: out[r out_stride + c] = the sum of its nbx_r
// partials of column c, in float64, in partial order; the first wave stores (host memory is
// fine: see signal_host).
__global__ __launch_bounds__(256) void k_dots_rows_final(DotsRows rows, int k1,
                                                         const double* __restrict__ dpart,
                                                         double* __restrict__ out,
                                                         size_t out_stride, SigArgs sig) {
  __shared__ double res[256];
  const DotsRow R = rows.r[blockIdx.x];
  const int tid = threadIdx.x;
  double* o = out + blockIdx.x * out_stride;
  for (int c0 = 0; c0 < k1; c0 += 256) {
    const int cn = min(256, k1 - c0);
    if (tid < cn) {
      double s = 0.0;
#pragma unroll 8
      for (int b = 0; b < R.nbx; ++b) s += dpart[(size_t)(R.part0 + b) * k1 + c0 + tid];
      res[tid] = s;
    }
    __syncthreads();
    if (tid < 64)
      for (int cc = tid; cc < cn; cc += 64) o[c0 + cc] = res[cc];
    __syncthreads();
  }
  signal_host(sig, gridDim.x);
}

// out[c] for c < k1: the sum over the nblocks partials dpart[b][c], in float64, in partial
// order. One block, a thread per column (coalesced across columns, several partials in
// flight); the first wave stores the sums (host memory is fine: see signal_host).
__global__ __launch_bounds__(256) void k_dots_final(const double* __restrict__ dpart, int nblocks,
                                                    int k1, double* __restrict__ out,
                                                    SigArgs sig) {
  __shared__ double res[256];
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < k1; c0 += 256) {
    const int cn = min(256, k1 - c0);
    if (tid < cn) {
      double s = 0.0;
#pragma unroll 8
      for (int b = 0; b < nblocks; ++b) s += dpart[(size_t)b * k1 + c0 + tid];
      res[tid] = s;
    }
    __syncthreads();
    if (tid < 64)
      for (int cc = tid; cc < cn; cc += 64) out[c0 + cc] = res[cc];
    __syncthreads();
  }
  signal_host(sig, 1);
}

__global__ __launch_bounds__(256) void k_any_nonfinite(const float* __restrict__ v, size_t n,
                                                       int* __restrict__ flag) {
  const size_t stride = (size_t)gridDim.x * 256;
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const float x = v[i];
    bad |= !(x - x == 0.f);  // false for NaN and +-Inf
  }
  if (bad) atomicOr(flag, 1);
}

}  // namespace

// ------------------------------------------------------------------ launchers

ConvPlan plan_conv(sfw_dims vol, int px, int py, int pz) {
  ConvPlan p;
  p.px = px;
  p.py = py;
  p.pz = pz;
  const int LX = kConvTX + px - 1;
  // z taps per pass: the smallest of 4 / 8 / 16 covering pz, reduced while even a single
  // y tap per pass would not fit the LDS budget
  p.kz = pz <= 4 ? 4 : (pz <= 8 ? 8 : 16);
  while (p.kz > 4 && (size_t)LX * kConvTY * conv_tile_lzp(p.kz) * 4 > (size_t)kConvMaxLds)
    p.kz /= 2;
  p.kzp = (pz + p.kz - 1) / p.kz * p.kz;
  const int LZ = conv_tile_lzp(p.kz);
  int kyc = py;
  while (kyc > 1 && (size_t)LX * (kConvTY + kyc - 1) * LZ * 4 > (size_t)kConvMaxLds) --kyc;
  p.kyc = kyc;
  p.lds_bytes = (size_t)LX * (kConvTY + kyc - 1) * LZ * 4;
  p.grid = dim3((vol.nx + kConvTX - 1) / kConvTX, (vol.ny + kConvTY - 1) / kConvTY,
                (vol.nz + kConvRZ - 1) / kConvRZ);
  p.nblocks = (int)(p.grid.x * p.grid.y * p.grid.z);
  return p;
}

GradPlan plan_grad_box(sfw_dims vol, const int box[6]) {
  GradPlan p;
  // tiles 32 planes deep: shallower ones add blocks (each with its release fence and its
  // partials for the last block to sum) faster than they shorten the per-thread chain, and
  // 64 planes leave too few blocks for one point's box
  p.vpt = vol.nz >= 32 ? 32 : 16;
  p.rx0 = box[0] / kTile;
  p.rtx = std::max(1, (box[1] + kTile - 1) / kTile - p.rx0);
  p.ry0 = box[2] / kTile;
  const int rty = std::max(1, (box[3] + kTile - 1) / kTile - p.ry0);
  p.ntile_xy = p.rtx * rty;
  p.rz0 = box[4] / p.vpt;
  p.ntile_z = std::max(1, (box[5] + p.vpt - 1) / p.vpt - p.rz0);
  p.ntiles = p.ntile_xy * p.ntile_z;
  return p;
}

hipError_t launch_prep(const sfw_atom* atoms, int n, bool unit_weight, AtomK* ak, const float* H,
                       sfw_dims psf, bool mfma, int kzp, bool fwd, bool adj, float* out_fwd,
                       float* out_adj, hipStream_t st) {
  const int steps = mfma ? mfma_steps(psf.nx, psf.ny) : 0;
  const int npsf = (H && (fwd || adj)) ? (mfma ? steps * 64 : psf.nx * psf.ny * kzp) : 0;
  const int count = std::max(n, npsf);
  if (count <= 0) return hipSuccess;
  dim3 grid((count + 255) / 256, npsf > 0 ? 3 : 1);
  hipLaunchKernelGGL(k_prep, grid, dim3(256), 0, st, atoms, n, unit_weight ? 1 : 0, ak, H, psf.nx,
                     psf.ny, psf.nz, mfma ? 1 : 0, steps, kzp, (fwd && npsf) ? 1 : 0,
                     (adj && npsf) ? 1 : 0, out_fwd, out_adj);
  return hipGetLastError();
}

hipError_t launch_store_atoms(const AtomK* host, int n, AtomK* dst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kAtomArgs) return hipErrorInvalidValue;
  AtomArgs args;
  std::memset(&args, 0, sizeof(args));
  std::memcpy(args.a, host, sizeof(AtomK) * n);
  hipLaunchKernelGGL(k_store_atoms, dim3(1), dim3(64), 0, st, args, n, dst);
  return hipGetLastError();
}

__global__ void k_store_box(Box6 b, int* __restrict__ dst) {
  if (threadIdx.x == 0) {
    dst[0] = b.x0;
    dst[1] = b.x1;
    dst[2] = b.y0;
    dst[3] = b.y1;
    dst[4] = b.z0;
    dst[5] = b.z1;
  }
}

hipError_t launch_store_box(const int box[6], int* dst, hipStream_t st) {
  const Box6 b{box[0], box[1], box[2], box[3], box[4], box[5]};
  hipLaunchKernelGGL(k_store_box, dim3(1), dim3(64), 0, st, b, dst);
  return hipGetLastError();
}

hipError_t launch_store_doubles(const double* host, int n, double* dst, hipStream_t st) {
  for (int i0 = 0; i0 < n; i0 += kDoubleArgs) {
    const int m = std::min(kDoubleArgs, n - i0);
    DoubleArgs args;
    std::memset(&args, 0, sizeof(args));
    std::memcpy(args.v, host + i0, sizeof(double) * m);
    hipLaunchKernelGGL(k_store_doubles, dim3(1), dim3(kDoubleArgs), 0, st, args, m, dst + i0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static int fp_blocks(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)std::max<size_t>(1, std::min<size_t>(b, kFpParts));
}

hipError_t launch_fingerprints(const float* y, size_t ny, const float* H, size_t nh,
                               const sfw_atom* atoms, int n, unsigned long long* part,
                               unsigned long long* out, float* atoms_out, const SigArgs& sig,
                               hipStream_t st) {
  const int by = fp_blocks(ny), bh = fp_blocks(nh);
  hipLaunchKernelGGL(k_fingerprints, dim3((unsigned)(by + bh)), dim3(256), 0, st, y, ny, by, H,
                     nh, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fingerprints_final, dim3(1), dim3(64), 0, st, part, by, bh,
                     reinterpret_cast<const float*>(atoms), atoms ? n : 0, out, atoms_out, sig);
  return hipGetLastError();
}

hipError_t launch_render(const AtomK* ak, int n, sfw_dims vol, float* f, hipStream_t st, int vpt,
                         const KernelEvents& ev) {
  const int tiles = ((vol.nx + kTile - 1) / kTile) * ((vol.ny + kTile - 1) / kTile);
  dim3 grid(tiles, (vol.nz + vpt - 1) / vpt);
  switch (vpt) {
    case 4:
      SFW_LAUNCH(ev, k_render<4>, grid, dim3(256), 0, st, ak, n, vol.nx, vol.ny, vol.nz, f);
      break;
    case 8:
      SFW_LAUNCH(ev, k_render<8>, grid, dim3(256), 0, st, ak, n, vol.nx, vol.ny, vol.nz, f);
      break;
    case 16:
      SFW_LAUNCH(ev, k_render<16>, grid, dim3(256), 0, st, ak, n, vol.nx, vol.ny, vol.nz, f);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KZ, int EPI>
static hipError_t conv_t(const ConvPlan& p, const float* in, const float* wt, sfw_dims vol,
                         float* out, const float* yobs, double* dpart, float scale,
                         long long idx_base, ArgPart* apart, hipStream_t st) {
  hipLaunchKernelGGL((k_conv<kConvTX, kConvTY, kConvRZ, KZ, EPI>), p.grid,
                     dim3(kConvTX * kConvTY), p.lds_bytes, st, in, wt, p.px, p.py, p.pz, p.kzp,
                     p.kyc, vol.nx, vol.ny, vol.nz, out, yobs, dpart, scale, idx_base, apart);
  return hipGetLastError();
}

template <int EPI>
static hipError_t conv_kz(const ConvPlan& p, const float* in, const float* wt, sfw_dims vol,
                          float* out, const float* yobs, double* dpart, float scale,
                          long long idx_base, ArgPart* apart, hipStream_t st) {
  switch (p.kz) {
    case 4:
      return conv_t<4, EPI>(p, in, wt, vol, out, yobs, dpart, scale, idx_base, apart, st);
    case 8:
      return conv_t<8, EPI>(p, in, wt, vol, out, yobs, dpart, scale, idx_base, apart, st);
    default:
      return conv_t<16, EPI>(p, in, wt, vol, out, yobs, dpart, scale, idx_base, apart, st);
  }
}

hipError_t launch_conv(const ConvPlan& p, const float* in, const float* wt, sfw_dims vol, int epi,
                       float* out, const float* yobs, double* dpart, float scale,
                       long long idx_base, ArgPart* apart, hipStream_t st) {
  switch (epi) {
    case kEpiPlain:
      return conv_kz<kEpiPlain>(p, in, wt, vol, out, yobs, dpart, scale, idx_base, apart, st);
    case kEpiResidual:
      return conv_kz<kEpiResidual>(p, in, wt, vol, out, yobs, dpart, scale, idx_base, apart, st);
    default:
      return conv_kz<kEpiArgmax>(p, in, wt, vol, out, yobs, dpart, scale, idx_base, apart, st);
  }
}

bool mfma_conv_ok(int px, int py, int pz) {
  return pz <= 16 && px * py <= 4 * 32 && (16 + px - 1) * (4 + py - 1) <= kMfmaPatchMax;
}

// MFMA steps (4 taps each) actually run: the smallest instantiated count covering px * py.
int mfma_steps(int px, int py) {
  const int need = (px * py + 3) / 4;
  const int counts[] = {1, 3, 7, 13, 21, 32};
  for (int c : counts)
    if (need <= c) return c;
  return 32;
}

int mfma_conv_blocks(sfw_dims vol) { return ((vol.nx + 15) / 16) * ((vol.ny + 3) / 4); }

template <int STEPS, int EPI>
static hipError_t mfma_t(const float* in, const float* amat, sfw_dims psf, sfw_dims vol,
                         const ConvRegion& rg, float* out, const float* yobs, double* dpart,
                         hipStream_t st) {
  const int chunks = (rg.z1 - rg.z0 + rg.zchunk - 1) / rg.zchunk;
  dim3 grid(rg.tx1 - rg.tx0, rg.ty1 - rg.ty0, chunks);
  hipLaunchKernelGGL((k_conv_mfma<STEPS, EPI>), grid, dim3(512), 0, st, in, amat, psf.nx, psf.ny,
                     psf.nz, vol.nx, vol.ny, vol.nz, rg.tx0, rg.ty0, rg.z0, rg.z1, rg.zchunk, out,
                     yobs, dpart);
  return hipGetLastError();
}

template <int EPI>
static hipError_t mfma_e(const float* in, const float* amat, sfw_dims psf, sfw_dims vol,
                         const ConvRegion& rg, float* out, const float* yobs, double* dpart,
                         hipStream_t st) {
  switch (mfma_steps(psf.nx, psf.ny)) {
    case 1: return mfma_t<1, EPI>(in, amat, psf, vol, rg, out, yobs, dpart, st);
    case 3: return mfma_t<3, EPI>(in, amat, psf, vol, rg, out, yobs, dpart, st);
    case 7: return mfma_t<7, EPI>(in, amat, psf, vol, rg, out, yobs, dpart, st);
    case 13: return mfma_t<13, EPI>(in, amat, psf, vol, rg, out, yobs, dpart, st);
    case 21: return mfma_t<21, EPI>(in, amat, psf, vol, rg, out, yobs, dpart, st);
    default: return mfma_t<32, EPI>(in, amat, psf, vol, rg, out, yobs, dpart, st);
  }
}

ConvRegion conv_region_full(sfw_dims vol) {
  ConvRegion rg;
  rg.tx0 = 0;
  rg.tx1 = (vol.nx + 15) / 16;
  rg.ty0 = 0;
  rg.ty1 = (vol.ny + 3) / 4;
  rg.z0 = 0;
  rg.z1 = vol.nz;
  rg.zchunk = std::max(vol.nz, 1);
  return rg;
}

hipError_t launch_conv_mfma(const float* in, const float* amat, sfw_dims psf, sfw_dims vol,
                            int epi, float* out, const float* yobs, double* dpart,
                            hipStream_t st) {
  const ConvRegion rg = conv_region_full(vol);
  if (epi == kEpiResidual)
    return mfma_e<kEpiResidual>(in, amat, psf, vol, rg, out, yobs, dpart, st);
  return mfma_e<kEpiPlain>(in, amat, psf, vol, rg, out, yobs, dpart, st);
}

// ------------------------------------------------------------------ LASSO column over a box

// The LASSO column a = H * (w g) of one atom (unit weight in the LASSO) on the box
// [bx0, bx1) x [by0, by1) x [bz0, bz1) only, without a rendered volume: each block computes
// the atom on its input tile (its kBoxTX x kBoxTY x kBoxZ outputs grown by the PSF
// half-widths, zero outside the volume) straight into LDS with the render's arithmetic, and
// convolves. Every wave covers the block's kBoxTX x kBoxTY output columns, one per lane, for
// the tap rows ky = wave, wave + nwaves, ... (nwaves = min(P_y, kBoxMaxWaves) waves per
// block, so that a small box still gives the chip enough waves). For each tap (ky, kx) a lane
// keeps the kBoxZ + PZ - 1 tile values of its column in registers and applies the PZ taps
// along z, the same for the whole wave, to its kBoxZ outputs. The PSF is staged in LDS beside
// the tile, transposed so that a tap column's P_z values are a few float4 broadcasts (with
// scalar loads of H instead, the waves of the one or two blocks a CU runs waited on a cold
// scalar cache at every tap column); where it does not fit, H is read by scalar loads. The
// tile is filled by (x, y) columns, so each thread takes its column's offsets once. The partial
// sums of the waves meet in LDS and are added in wave order.
constexpr int kBoxTX = 16, kBoxTY = 4, kBoxZ = 4, kBoxMaxWaves = 16;
static_assert(kBoxTX * kBoxTY == 64, "one output column per lane");

// Up to kBoxColumns columns (one PSF) per launch: column c takes the blocks [first, first +
// gx gy gz) of the flat grid, its block b as (b % gx, b / gx % gy, b / (gx gy)).
struct BoxColumn {
  const AtomK* atom;
  float* out;
  int* box_out;
  int bx0, by0, bz0, bx1, by1, bz1;
  int gx, gy, first;
};
struct BoxColumns {
  BoxColumn c[kBoxColumns];
};

template <int PZ, bool HLDS>
__global__ __launch_bounds__(64 * kBoxMaxWaves) void k_column_box(
    BoxColumns cols, int ncols, const float* __restrict__ H, int pxs, int pys, int nx, int ny,
    int nz) {
  int ci = 0;
  while (ci + 1 < ncols && (int)blockIdx.x >= cols.c[ci + 1].first) ++ci;
  const BoxColumn& C = cols.c[ci];
  const AtomK* __restrict__ atom = C.atom;
  float* __restrict__ out = C.out;
  int* __restrict__ box_out = C.box_out;
  const int bx0 = C.bx0, by0 = C.by0, bz0 = C.bz0, bx1 = C.bx1, by1 = C.by1, bz1 = C.bz1;
  const int b = (int)blockIdx.x - C.first;
  const int bxi = b % C.gx, byi = (b / C.gx) % C.gy, bzi = b / (C.gx * C.gy);
  if (box_out && b == 0 && threadIdx.x == 0) {
    box_out[0] = bx0;  // the box this column is valid on (read by the Gram-row kernels)
    box_out[1] = bx1;
    box_out[2] = by0;
    box_out[3] = by1;
    box_out[4] = bz0;
    box_out[5] = bz1;
  }
  // tile [yy][xx][w] with the z window w innermost (WZP floats per column, 16-byte aligned),
  // read as float4; with HLDS, the PSF follows it as [ky][kx][kz] (PZP floats per tap column)
  constexpr int WZ = kBoxZ + PZ - 1, WZP = (WZ + 3) & ~3, PZP = (PZ + 3) & ~3;
  extern __shared__ float4 lds4[];
  float* tile = reinterpret_cast<float*>(lds4);
  const int LX = kBoxTX + pxs - 1, LY = kBoxTY + pys - 1;
  const int X0 = bx0 + bxi * kBoxTX, Y0 = by0 + byi * kBoxTY;
  const int Z0 = bz0 + bzi * kBoxZ;
  const int cx = (pxs - 1) / 2, cy = (pys - 1) / 2, cz = (PZ - 1) / 2;
  const int t = threadIdx.x;
  const int nwaves = (int)(blockDim.x >> 6);
  const int NT = (int)blockDim.x;
  const int ncol = LX * LY;
  const int tile_floats = max(WZP * ncol, nwaves * kBoxZ * 64);
  float* htile = tile + ((tile_floats + 3) & ~3);
  if (HLDS) {  // the PSF, read once per block with consecutive threads on consecutive taps
    const int plane = pxs * pys, ntap = plane * PZ;
    for (int e = t; e < ntap; e += NT) {
      const int kz = e / plane, r = e - kz * plane;
      htile[r * PZP + kz] = H[e];
    }
  }
  const AtomK k = *atom;
  // the tile by (x, y) columns: G = NT / ncol thread groups (at least one) split the z window
  {
    const int G = max(1, NT / ncol), chunk = (WZ + G - 1) / G;
    for (int c0 = t; c0 < ncol * G; c0 += NT) {
      const int g = c0 / ncol, c = c0 - g * ncol;
      const int xx = c % LX, yy = c / LX;
      const int x = X0 - cx + xx, y = Y0 - cy + yy;
      const bool inxy = x >= 0 && x < nx && y >= 0 && y < ny;
      const float dx = (float)x - k.mx, dy = (float)y - k.my;
      const float dxy2 = fmaf(dx, dx, fmaf(dy, dy, kTinyR2));
      float* col = tile + c * WZP;
      const int za = g * chunk, zb = min(WZ, za + chunk);
      for (int zz = za; zz < zb; ++zz) {
        const int z = Z0 - cz + zz;
        float gv = 0.f;
        if (inxy && z >= 0 && z < nz) {
          const float dz = (float)z - k.mz;
          const float r2 = fmaf(dz, dz, dxy2);
          const float up = fast_exp2(fmaf(k.hd, fast_log2(r2), k.c));  // u * log2(e)
          gv = k.w * fast_exp2(-up);
        }
        col[zz] = gv;
      }
    }
  }
  __syncthreads();
  const int lane = t & 63;
  const int xl = lane % kBoxTX, yl = lane / kBoxTX;
  const int part = __builtin_amdgcn_readfirstlane(t >> 6);
  const int hstride = pys * pxs;  // H is [kz][ky][kx]
  float acc[kBoxZ];
#pragma unroll
  for (int o = 0; o < kBoxZ; ++o) acc[o] = 0.f;
  for (int ky = part; ky < pys; ky += nwaves) {
    const int yy = yl + pys - 1 - ky;
#pragma unroll 3
    for (int kx = 0; kx < pxs; ++kx) {
      const int xx = xl + pxs - 1 - kx;
      const float4* tv = reinterpret_cast<const float4*>(tile + (yy * LX + xx) * WZP);
      float v[WZP], h[PZP];
#pragma unroll
      for (int q = 0; q < WZP / 4; ++q) {
        const float4 f = tv[q];
        v[4 * q] = f.x;
        v[4 * q + 1] = f.y;
        v[4 * q + 2] = f.z;
        v[4 * q + 3] = f.w;
      }
      if (HLDS) {
        const float4* hv = reinterpret_cast<const float4*>(htile + (ky * pxs + kx) * PZP);
#pragma unroll
        for (int q = 0; q < PZP / 4; ++q) {
          const float4 f = hv[q];
          h[4 * q] = f.x;
          h[4 * q + 1] = f.y;
          h[4 * q + 2] = f.z;
          h[4 * q + 3] = f.w;
        }
      } else {
        const float* hp = H + ky * pxs + kx;
#pragma unroll
        for (int kz = 0; kz < PZ; ++kz) h[kz] = hp[kz * hstride];
      }
#pragma unroll
      for (int kz = 0; kz < PZ; ++kz) {
#pragma unroll
        for (int o = 0; o < kBoxZ; ++o) acc[o] = fmaf(h[kz], v[o + PZ - 1 - kz], acc[o]);
      }
    }
  }
  // partial sums of the waves, through the (no longer needed) tile: [part][o][lane]
  __syncthreads();
#pragma unroll
  for (int o = 0; o < kBoxZ; ++o) tile[(part * kBoxZ + o) * 64 + lane] = acc[o];
  __syncthreads();
  if (part == 0) {
    const int ox = X0 + xl, oy = Y0 + yl;
    if (ox < bx1 && oy < by1) {
#pragma unroll
      for (int o = 0; o < kBoxZ; ++o) {
        float sum = 0.f;
        for (int q = 0; q < nwaves; ++q) sum += tile[(q * kBoxZ + o) * 64 + lane];
        const int oz = Z0 + o;
        if (oz < bz1) out[((size_t)oz * ny + oy) * nx + ox] = sum;
      }
    }
  }
}

static int column_box_waves(sfw_dims psf) { return std::min(psf.ny, kBoxMaxWaves); }

static size_t column_box_lds(sfw_dims psf) {
  const size_t wzp = (size_t)((kBoxZ + psf.nz - 1 + 3) & ~3);
  const size_t tile = std::max(wzp * (kBoxTY + psf.ny - 1) * (kBoxTX + psf.nx - 1),
                               (size_t)column_box_waves(psf) * kBoxZ * 64);
  return tile * sizeof(float);
}

// LDS with the PSF staged beside the tile ([ky][kx][kz], P_z padded to 4)
static size_t column_box_lds_h(sfw_dims psf) {
  const size_t tile = (column_box_lds(psf) / sizeof(float) + 3) & ~(size_t)3;
  const size_t h = (size_t)psf.nx * psf.ny * ((psf.nz + 3) & ~3);
  return (tile + h) * sizeof(float);
}

bool column_box_ok(sfw_dims psf) {
  // tile rows of at most one wave of x, P_z a supported template, the LDS of one CU
  return kBoxTX + psf.nx - 1 <= 64 && psf.nz <= 33 &&
         column_box_lds(psf) <= (size_t)kColumnBoxMaxLds;
}

hipError_t launch_column_boxes(const ColumnBoxJob* jobs, int n, const float* H, sfw_dims psf,
                               sfw_dims vol, hipStream_t st, const KernelEvents& ev) {
  if (!column_box_ok(psf) || n < 0 || n > kBoxColumns) return hipErrorInvalidValue;
  BoxColumns bc;
  std::memset(&bc, 0, sizeof(bc));
  int nc = 0, blocks = 0;
  for (int i = 0; i < n; ++i) {
    const int* box = jobs[i].box;
    const int bw = box[1] - box[0], bh = box[3] - box[2], bd = box[5] - box[4];
    if (bw <= 0 || bh <= 0 || bd <= 0) continue;  // nothing to compute
    const int gx = (bw + kBoxTX - 1) / kBoxTX, gy = (bh + kBoxTY - 1) / kBoxTY;
    const int gz = (bd + kBoxZ - 1) / kBoxZ;
    bc.c[nc++] = BoxColumn{jobs[i].atom, jobs[i].out, jobs[i].box_out, box[0], box[2], box[4],
                           box[1], box[3], box[5], gx, gy, blocks};
    blocks += gx * gy * gz;
  }
  if (nc == 0) return record_events(ev, st);
  const dim3 grid(blocks);
  const bool hlds = column_box_lds_h(psf) <= (size_t)kColumnBoxMaxLds;
  const size_t lds = hlds ? column_box_lds_h(psf) : column_box_lds(psf);
  switch (psf.nz) {
#define SFW_BOX_CASE(P)                                                                        \
  case P: {                                                                                    \
    static const hipError_t attr = hipFuncSetAttribute(                                        \
        reinterpret_cast<const void*>(&k_column_box<P, true>),                                 \
        hipFuncAttributeMaxDynamicSharedMemorySize, kColumnBoxMaxLds);                         \
    static const hipError_t attr2 = hipFuncSetAttribute(                                       \
        reinterpret_cast<const void*>(&k_column_box<P, false>),                                \
        hipFuncAttributeMaxDynamicSharedMemorySize, kColumnBoxMaxLds);                         \
    if (attr != hipSuccess) return attr;                                                       \
    if (attr2 != hipSuccess) return attr2;                                                     \
    if (hlds)                                                                                  \
      SFW_LAUNCH(ev, (k_column_box<P, true>), grid, dim3(64 * column_box_waves(psf)), lds, st, \
                 bc, nc, H, psf.nx, psf.ny, vol.nx, vol.ny, vol.nz);                           \
    else                                                                                       \
      SFW_LAUNCH(ev, (k_column_box<P, false>), grid, dim3(64 * column_box_waves(psf)), lds,    \
                 st, bc, nc, H, psf.nx, psf.ny, vol.nx, vol.ny, vol.nz);                       \
    return hipGetLastError();                                                                  \
  }
    SFW_BOX_CASE(1) SFW_BOX_CASE(3) SFW_BOX_CASE(5) SFW_BOX_CASE(7) SFW_BOX_CASE(9)
    SFW_BOX_CASE(11) SFW_BOX_CASE(13) SFW_BOX_CASE(15) SFW_BOX_CASE(17) SFW_BOX_CASE(19)
    SFW_BOX_CASE(21) SFW_BOX_CASE(23) SFW_BOX_CASE(25) SFW_BOX_CASE(27) SFW_BOX_CASE(29)
    SFW_BOX_CASE(31) SFW_BOX_CASE(33)
#undef SFW_BOX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_column_box(const AtomK* atom, const float* H, sfw_dims psf, sfw_dims vol,
                             const int box[6], float* out, int* box_out, hipStream_t st) {
  ColumnBoxJob job;
  job.atom = atom;
  job.out = out;
  job.box_out = box_out;
  std::memcpy(job.box, box, sizeof(job.box));
  return launch_column_boxes(&job, 1, H, psf, vol, st);
}

hipError_t launch_conv_mfma_region(const float* in, const float* amat, sfw_dims psf, sfw_dims vol,
                                   const ConvRegion& rg, float* out, hipStream_t st) {
  if (rg.tx1 <= rg.tx0 || rg.ty1 <= rg.ty0 || rg.z1 <= rg.z0 || rg.zchunk < 1)
    return hipSuccess;
  // its own instantiation (same plain epilogue), so profiles tell it from whole-volume launches
  return mfma_e<kEpiColumn>(in, amat, psf, vol, rg, out, nullptr, nullptr, st);
}

int grad_item_tiles(sfw_dims vol) {
  return ((vol.nx + kTile - 1) / kTile) * ((vol.ny + kTile - 1) / kTile) *
         ((vol.nz + kTile - 1) / kTile);
}

hipError_t launch_grad_items(const AtomK* ak, int n, const float* q, sfw_dims vol, float* gpart,
                             int* item_start, int blocks, hipStream_t st,
                             const KernelEvents& ev) {
  if (n <= 0) return record_events(ev, st);
  if (blocks < 1) return hipErrorInvalidValue;
  size_t lds = ((size_t)(n + 1) * sizeof(int) + 15) / 16 * 16;
  if (n <= kItemsLdsAtoms) lds += (size_t)n * (sizeof(AtomK) + sizeof(ItemBox));
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  SFW_LAUNCH(ev, k_grad_items, dim3(blocks), dim3(kGradThreads), lds, st, ak, n, q, vol.nx,
             vol.ny, vol.nz, gpart, item_start);
  return hipGetLastError();
}

hipError_t launch_grad_points(const GradPlan& p, const AtomK* host_atoms, int n, const float* q,
                              sfw_dims vol, float* gpart, int* ticket, double* sums_out,
                              const SigArgs& sig, hipStream_t st, const KernelEvents& ev) {
  if (n <= 0 || n > kAtomArgs) return hipErrorInvalidValue;
  AtomArgs args;
  std::memset(&args, 0, sizeof(args));
  std::memcpy(args.a, host_atoms, sizeof(AtomK) * n);
  dim3 grid(p.ntiles, 1);
  switch (p.vpt) {
#define SFW_GRAD_CASE(V)                                                                       \
  case V:                                                                                      \
    SFW_LAUNCH(ev, (k_grad_points<V>), grid, dim3(kGradThreads), 0, st, args, n, q, vol.nx,     \
               vol.ny, vol.nz, p.ntile_xy, p.rx0, p.ry0, p.rtx, p.rz0, gpart, ticket, sums_out, \
               sig);                                                                            \
    break;
    SFW_GRAD_CASE(64)
    SFW_GRAD_CASE(32)
    SFW_GRAD_CASE(16)
    default:
      return hipErrorInvalidValue;
#undef SFW_GRAD_CASE
  }
  return hipGetLastError();
}

hipError_t launch_grad_finalize(const float* gpart, int ntiles, const int* item_start, int n,
                                const double* loss_part, int nloss, const sfw_atom* atoms,
                                float lambda, double* sums, sfw_atom* grad_out, double* loss_out,
                                hipStream_t st, bool vjp, const SigArgs& sig,
                                const KernelEvents& ev) {
  SFW_LAUNCH(ev, k_grad_finalize, dim3(n + 1), dim3(256), 0, st, gpart, ntiles, item_start, n,
             loss_part, nloss, atoms, lambda, sums, grad_out, loss_out, vjp ? 1 : 0, sig);
  return hipGetLastError();
}

hipError_t launch_argmax_final(const ArgPart* apart, int nparts, sfw_dims vol, int nd,
                               sfw_argmax* best, sfw_argmax* best_host, const SigArgs& sig,
                               hipStream_t st, const KernelEvents& ev) {
  SFW_LAUNCH(ev, k_argmax_final, dim3(1), dim3(1024), 0, st, apart, nparts, vol.nx, vol.ny,
             vol.nz, nd, best, best_host, sig);
  return hipGetLastError();
}

hipError_t launch_dots(const float* a, const int abox[6], const float* cols, const SlotArgs& sa,
                       const int* slots, const int* slot_box, int k, size_t colstride,
                       const float* y, sfw_dims vol, double* dpart, int nblocks, double* out,
                       const SigArgs& sig, hipStream_t st) {
  const Box6 ab{abox[0], abox[1], abox[2], abox[3], abox[4], abox[5]};
  const size_t nvox = (size_t)vol.nx * vol.ny * vol.nz;
  hipLaunchKernelGGL(k_dots, dim3(nblocks), dim3(256), 0, st, a, ab, cols, sa, slots, slot_box, k,
                     colstride, y, vol.nx, vol.ny, nvox, dpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(256), 0, st, dpart, nblocks, k + 1, out, sig);
  return hipGetLastError();
}

int dots_box_blocks(const int box[6]) {
  const int bw4 = (box[1] - box[0]) / 4, nrows = (box[3] - box[2]) * (box[5] - box[4]);
  const int E = nrows * bw4;
  return std::max(1, (E + 256 * kDotsHold - 1) / (256 * kDotsHold));
}

hipError_t launch_dots_box_rows(const GramRowBox* rows, int nr, const float* cols,
                                const SlotArgs& sa, const int* slots, const int* slot_box, int k,
                                size_t colstride, const float* y, sfw_dims vol, double* dpart,
                                int dpart_cap, double* out, size_t out_stride, const SigArgs& sig,
                                hipStream_t st) {
  if (nr < 1 || nr > kDotsRows) return hipErrorInvalidValue;
  DotsRows R;
  std::memset(&R, 0, sizeof(R));
  int part = 0, maxnbx = 0;
  for (int r = 0; r < nr; ++r) {
    const int* box = rows[r].box;
    const int bw4 = (box[1] - box[0]) / 4, bh = box[3] - box[2], nrows = bh * (box[5] - box[4]);
    if (nrows * bw4 <= 0) return hipErrorInvalidValue;
    const int nbx = dots_box_blocks(box);
    R.r[r] = DotsRow{rows[r].a, box[0], bw4, box[2], bh, box[4], nrows, nbx, part};
    part += nbx;
    maxnbx = std::max(maxnbx, nbx);
  }
  if ((size_t)part * (k + 1) > (size_t)dpart_cap) return hipErrorInvalidValue;
  // column chunks: enough blocks to fill the chip, chunks of whole column groups
  const int groups = (k + 1 + kDotsCols - 1) / kDotsCols;
  int chunks = std::max(1, std::min(groups, (1024 + part - 1) / part));
  const int cpb = (groups + chunks - 1) / chunks * kDotsCols;
  chunks = (k + 1 + cpb - 1) / cpb;
  hipLaunchKernelGGL(k_dots_box, dim3(maxnbx, chunks, nr), dim3(256), 0, st, R, cols, sa, slots,
                     slot_box, k, colstride, y, vol.nx, vol.ny, cpb, dpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dots_rows_final, dim3(nr), dim3(256), 0, st, R, k + 1, dpart, out,
                     out_stride, sig);
  return hipGetLastError();
}

hipError_t launch_dots_box(const float* a, const float* cols, const SlotArgs& sa,
                           const int* slots, const int* slot_box, int k, size_t colstride,
                           const float* y, sfw_dims vol, const int box[6], double* dpart,
                           int dpart_cap, double* out, const SigArgs& sig, hipStream_t st) {
  GramRowBox row;
  row.a = a;
  std::memcpy(row.box, box, sizeof(row.box));
  return launch_dots_box_rows(&row, 1, cols, sa, slots, slot_box, k, colstride, y, vol, dpart,
                              dpart_cap, out, 0, sig, st);
}

hipError_t launch_any_nonfinite(const float* v, size_t n, int* flag, hipStream_t st) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_any_nonfinite, dim3((unsigned)blocks), dim3(256), 0, st, v, n, flag);
  return hipGetLastError();
}

}  // namespace sfw
