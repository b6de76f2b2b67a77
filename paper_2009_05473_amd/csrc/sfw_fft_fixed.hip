// Batched 1D FFT passes of compile-time length L = R1 * R2 for the Fourier-domain grid
// certificate (the paper evaluates its convolutions in the Fourier domain, section 2).
//
// Each line is transformed by two Stockham stages: R2 register-resident R1-point DFTs whose
// inputs come straight from global memory, one exchange through LDS, then R1 twiddled
// R2-point DFTs whose outputs go straight to global memory (or to the certificate's
// maximum). With L, R1 and R2 known at compile time, every index and LDS offset folds, so
// the passes cost little beyond the butterflies themselves. Lengths without a two-stage plan
// use the generic runtime-length passes.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "sfw_fft_radix.h"
#include "sfw_internal.h"

namespace sfw {

namespace {

using fftr::cmul;
using fftr::Dft;

// Threads of a block whose C lines need max(C R1, C R2) tasks in one stage, in whole waves.
constexpr int fx_threads(int R1, int R2) {
  const int t = kFxLines * (R1 > R2 ? R1 : R2);
  return (t + 63) / 64 * 64;
}

__device__ __forceinline__ bool arg_better32(float v, int i, float bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// ---------------------------------------------------------------- strided lines (y or z)

// Lines along one axis (element i of column x at o * ostride + i * istride + x) for kFxLines
// adjacent columns x0.. at outer coordinate o = blockIdx.y of batch entry blockIdx.z (arrays
// offset by their batch strides). Reads i < n_in (zero beyond), writes i < n_out.
// tw: exp(-2 pi i m / L), m < L.
template <int R1, int R2>
__global__ __launch_bounds__(fx_threads(R1, R2)) void k_fx_strided(
    const float2* __restrict__ src, size_t src_b, float2* __restrict__ dst, size_t dst_b,
    const float2* __restrict__ twg, int ncols, size_t istride, size_t ostride, int n_in,
    int n_out) {
  constexpr int L = R1 * R2, LS = L | 1, C = kFxLines, NT = fx_threads(R1, R2);
  __shared__ float2 buf[C * LS];
  __shared__ float2 tw[L];
  src += blockIdx.z * src_b;
  dst += blockIdx.z * dst_b;
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = twg[i];
  const int x0 = blockIdx.x * C;
  const size_t obase = (size_t)blockIdx.y * ostride + x0;
  const int cols = min(C, ncols - x0);
  const int t = threadIdx.x;
  // stage 1: task (c, j), j < R2, reads elements j + r R2 and writes LDS slots j R1 + r
  if (t < C * R2) {
    const int c = t % C, j = t / C;
    const bool cok = c < cols;
    float2 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int i = j + r * R2;
      const bool ok = cok && i < n_in;
      const float2 a = src[obase + (ok ? (size_t)i * istride + c : 0)];
      v[r] = ok ? a : make_float2(0.f, 0.f);
    }
    Dft<R1>::run(v);
#pragma unroll
    for (int r = 0; r < R1; ++r) buf[c * LS + j * R1 + r] = v[r];
  }
  __syncthreads();
  // stage 2: task (c, j), j < R1, reads slots j + r R1, twiddles exp(-2 pi i r j / L), and
  // writes elements j + r R1
  if (t < C * R1) {
    const int c = t % C, j = t / C;
    float2 v[R2];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      v[r] = buf[c * LS + j + r * R1];
      if (r > 0) v[r] = cmul(v[r], tw[r * j]);
    }
    Dft<R2>::run(v);
    if (c < cols) {
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int i = j + r * R1;
        if (i < n_out) dst[obase + (size_t)i * istride + c] = v[r];
      }
    }
  }
}

// k <= N / 2 representative of frequency k in [0, N) for spectra even in that axis.
__device__ __forceinline__ int fold(int k, int N) { return 2 * k <= N ? k : N - k; }

// First inverse pass, along z (L = Nz), for every pair: column (x0 + c, y) of Qhat is loaded
// once into LDS (each task keeps its R1 elements there), then for each pair p the input
// conj(Qhat * P_p) (P_p read from its octant) is transformed and rows z < n_out are written to
// work + p * work_b. Keeping Qhat in LDS rather than registers, and fetching a pair's octant
// values where they are used rather than one pair ahead, holds the kernel at 88 VGPRs at L = 81,
// five waves per SIMD, so that the whole grid of the 128 x 128 x 64 workload is resident at once
// (at 120 VGPRs a sixth of its blocks waited for a second round).
//
// Rows y and Ny - y read the same octant rows, as do all x groups of a row. Workgroups go to
// the 8 XCDs round-robin by linear id and each XCD has its own L2, so the 1D grid is remapped:
// the x groups of row y = 0, then of rows 1, Ny - 1, 2, Ny - 2, ... form one sequence, cut
// into 8 contiguous chunks, chunk k running on XCD k. A row and its mirror then share an L2
// and the octants are fetched from memory about once. Blocks past gx * Ny return at once.
template <int R1, int R2>
__global__ __launch_bounds__(fx_threads(R1, R2)) void k_fx_z_inverse(
    const float2* __restrict__ qhat, const float2* __restrict__ oct, size_t oct_b, int hx, int hy,
    float2* __restrict__ work, size_t work_b, const float2* __restrict__ twg, int Nx, int Ny,
    int px, int n_out, int npairs, int gx, int chunk) {
  constexpr int L = R1 * R2, LS = L | 1, C = kFxLines, NT = fx_threads(R1, R2), T1 = C * R2;
  __shared__ float2 buf[C * LS];
  __shared__ float2 tw[L];
  __shared__ float2 qs[R1 * T1];  // the column of Qhat, element r of task t at qs[r T1 + t]
  const int lid = blockIdx.x;
  const int seq = (lid & 7) * chunk + (lid >> 3);
  if (seq >= gx * Ny) return;
  const int rho = seq / gx;
  const int y = rho == 0 ? 0 : ((rho & 1) ? (rho + 1) >> 1 : Ny - (rho >> 1));
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = twg[i];
  const int x0 = (seq - rho * gx) * C;
  const size_t istride = (size_t)px * Ny;
  const size_t obase = (size_t)y * px + x0;
  const int cols = min(C, Nx - x0);
  const int t = threadIdx.x;
  const bool s1 = t < T1;
  const int c1 = t % C, j1 = t / C;
  const bool cok = s1 && c1 < cols;
  // octant offset of this task's element r (any pair): (fold(i) hy + my) hx + mx
  const int mx = fold(min(x0 + c1, Nx - 1), Nx), my = fold(y, Ny);
  auto po = [&](int r) { return (fold(j1 + r * R2, L) * hy + my) * hx + mx; };
  if (s1) {
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int i = j1 + r * R2;  // < L
      const float2 a = qhat[obase + (cok ? (size_t)i * istride + c1 : 0)];
      qs[r * T1 + t] = cok ? a : make_float2(0.f, 0.f);
    }
  }
  for (int p = 0; p < npairs; ++p) {
    if (s1) {
      const float2* P = oct + (size_t)p * oct_b;
      float2 v[R1];
#pragma unroll
      for (int r = 0; r < R1; ++r) v[r] = P[po(r)];
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        v[r] = cmul(qs[r * T1 + t], v[r]);
        v[r].y = -v[r].y;
      }
      Dft<R1>::run(v);
#pragma unroll
      for (int r = 0; r < R1; ++r) buf[c1 * LS + j1 * R1 + r] = v[r];
    }
    __syncthreads();
    if (t < C * R1) {
      const int c = t % C, j = t / C;
      float2 v[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        v[r] = buf[c * LS + j + r * R1];
        if (r > 0) v[r] = cmul(v[r], tw[r * j]);
      }
      Dft<R2>::run(v);
      if (c < cols) {
        float2* dst = work + (size_t)p * work_b + obase;
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          const int i = j + r * R1;
          if (i < n_out) dst[(size_t)i * istride + c] = v[r];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- contiguous lines (x)

// Shared body of the x passes: kFxLines lines (y0 + l, z = blockIdx.y) of length L. Stage 1
// loads through get(l, i) (valid l, i < L); stage 2 hands each task's outputs to
// put(l, j, v), v[r] being element j + r R1 of line l, r < R2.
template <int R1, int R2, class Get, class Put>
__device__ __forceinline__ void fx_xlines(float2* buf, const float2* tw, Get get, Put put) {
  constexpr int L = R1 * R2, LS = L | 1, B = kFxLines;
  const int t = threadIdx.x;
  if (t < B * R2) {
    const int j = t % R2, l = t / R2;  // consecutive lanes: consecutive elements of a line
    float2 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) v[r] = get(l, j + r * R2);
    Dft<R1>::run(v);
#pragma unroll
    for (int r = 0; r < R1; ++r) buf[l * LS + j * R1 + r] = v[r];
  }
  __syncthreads();
  if (t < B * R1) {
    const int j = t % R1, l = t / R1;
    float2 v[R2];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      v[r] = buf[l * LS + j + r * R1];
      if (r > 0) v[r] = cmul(v[r], tw[r * j]);
    }
    Dft<R2>::run(v);
    put(l, j, v);
  }
}

// Forward x pass of the real volume q (lines y < ny of plane z < nz, zero beyond nx) into
// out[(z * Ny + y) * px + i], i < L.
template <int R1, int R2>
__global__ __launch_bounds__(fx_threads(R1, R2)) void k_fx_x_real(
    const float* __restrict__ q, int nx, int ny, const float2* __restrict__ twg, int Ny, int px,
    float2* __restrict__ out) {
  constexpr int L = R1 * R2, LS = L | 1, NT = fx_threads(R1, R2);
  __shared__ float2 buf[kFxLines * LS];
  __shared__ float2 tw[L];
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = twg[i];
  const int y0 = blockIdx.x * kFxLines, z = blockIdx.y;
  const int lines = min(kFxLines, ny - y0);
  const float* base = q + ((size_t)z * ny + y0) * nx;
  float2* obase = out + ((size_t)z * Ny + y0) * px;
  fx_xlines<R1, R2>(
      buf, tw,
      [&](int l, int i) {
        const bool ok = l < lines && i < nx;
        const float v = base[ok ? l * nx + i : 0];
        return make_float2(ok ? v : 0.f, 0.f);
      },
      [&](int l, int j, const float2* v) {
        if (l < lines) {
#pragma unroll
          for (int r = 0; r < R2; ++r) obase[(size_t)l * px + j + r * R1] = v[r];
        }
      });
}

// Last inverse pass of pair p = blockIdx.z: lines (y < ny, z < nz) of its work array, forward
// FFT, conjugated output; the real part is eta of table kernel 2p and the imaginary part eta
// of kernel 2p + 1 (if < nslices), times scale. Writes eta (optional) and the block maxima
// (ties to the lowest flat index).
template <int R1, int R2>
__global__ __launch_bounds__(fx_threads(R1, R2)) void k_fx_x_argmax(
    const float2* __restrict__ work, size_t work_b, int nx, int ny, int nz,
    const float2* __restrict__ twg, int Ny, int px, float scale, int nslices,
    float* __restrict__ eta_out, ArgPart* __restrict__ apart, int nblk) {
  constexpr int L = R1 * R2, LS = L | 1, NT = fx_threads(R1, R2), NW = NT / 64;
  __shared__ float2 buf[kFxLines * LS];
  __shared__ float2 tw[L];
  __shared__ float rv[2][NW];
  __shared__ int ri[2][NW];
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = twg[i];
  const int slice_a = 2 * (int)blockIdx.z;
  const int slice_b = slice_a + 1 < nslices ? slice_a + 1 : -1;
  const int y0 = blockIdx.x * kFxLines, z = blockIdx.y;
  const int lines = min(kFxLines, ny - y0);
  const float2* base = work + blockIdx.z * work_b + ((size_t)z * Ny + y0) * px;
  const size_t V = (size_t)nx * ny * nz;
  const int v0 = (z * ny + y0) * nx;  // flat index of (0, y0, z); V < 2^31
  float bva = -INFINITY, bvb = -INFINITY;
  int bia = 0x7fffffff, bib = 0x7fffffff;
  fx_xlines<R1, R2>(
      buf, tw,
      [&](int l, int i) {
        const bool ok = l < lines;
        const float2 v = base[ok ? (size_t)l * px + i : 0];
        return ok ? v : make_float2(0.f, 0.f);
      },
      [&](int l, int j, const float2* c) {
        // invalid voxels (past the volume) carry (-inf, INT_MAX), which never wins
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          const int i = j + r * R1;
          const bool ok = l < lines && i < nx;
          const int v = ok ? v0 + l * nx + i : 0x7fffffff;
          const float ea = ok ? c[r].x * scale : -INFINITY;
          const float eb = ok ? -c[r].y * scale : -INFINITY;
          if (arg_better32(ea, v, bva, bia)) {
            bva = ea;
            bia = v;
          }
          if (arg_better32(eb, v, bvb, bib)) {
            bvb = eb;
            bib = v;
          }
        }
        if (eta_out && l < lines) {
#pragma unroll
          for (int r = 0; r < R2; ++r) {
            const int i = j + r * R1;
            if (i < nx) {
              const int v = v0 + l * nx + i;
              eta_out[(size_t)slice_a * V + v] = c[r].x * scale;
              if (slice_b >= 0) eta_out[(size_t)slice_b * V + v] = -c[r].y * scale;
            }
          }
        }
      });
  for (int o = 32; o > 0; o >>= 1) {
    const float ova = __shfl_xor(bva, o, 64);
    const int oia = __shfl_xor(bia, o, 64);
    if (arg_better32(ova, oia, bva, bia)) {
      bva = ova;
      bia = oia;
    }
    const float ovb = __shfl_xor(bvb, o, 64);
    const int oib = __shfl_xor(bib, o, 64);
    if (arg_better32(ovb, oib, bvb, bib)) {
      bvb = ovb;
      bib = oib;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    rv[0][threadIdx.x >> 6] = bva;
    ri[0][threadIdx.x >> 6] = bia;
    rv[1][threadIdx.x >> 6] = bvb;
    ri[1][threadIdx.x >> 6] = bib;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int s = threadIdx.x;
    const int slice = s == 0 ? slice_a : slice_b;
    if (slice >= 0) {
      float v = rv[s][0];
      int id = ri[s][0];
      for (int w = 1; w < NW; ++w)
        if (arg_better32(rv[s][w], ri[s][w], v, id)) {
          v = rv[s][w];
          id = ri[s][w];
        }
      ArgPart ap;
      ap.val = v;
      ap.pad = 0;
      // a block with no voxel (cannot happen for launched blocks) keeps idx past every slice
      ap.idx = id == 0x7fffffff ? 0x7fffffffffffffffLL : (long long)slice * (long long)V + id;
      const int blk = blockIdx.y * gridDim.x + blockIdx.x;  // < nblk
      apart[(size_t)slice * nblk + blk] = ap;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- host dispatch

bool fft_fixed_plan(int L, int* r1, int* r2) {
  switch (L) {
#define SFW_FX_CASE(n, a, b) \
  case n:                    \
    *r1 = a;                 \
    *r2 = b;                 \
    return true;
    SFW_FX_LENGTHS(SFW_FX_CASE)
#undef SFW_FX_CASE
    default:
      return false;
  }
}

hipError_t fx_strided(int L, dim3 grid, hipStream_t st, const float2* src, size_t src_b,
                      float2* dst, size_t dst_b, const float2* tw, int ncols, size_t istride,
                      size_t ostride, int n_in, int n_out) {
  switch (L) {
#define SFW_FX_CASE(n, a, b)                                                                 \
  case n:                                                                                    \
    hipLaunchKernelGGL((k_fx_strided<a, b>), grid, dim3(fx_threads(a, b)), 0, st, src, src_b, \
                       dst, dst_b, tw, ncols, istride, ostride, n_in, n_out);                \
    return hipGetLastError();
    SFW_FX_LENGTHS(SFW_FX_CASE)
#undef SFW_FX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t fx_z_inverse(int L, hipStream_t st, const float2* qhat, const float2* oct,
                        size_t oct_b, int hx, int hy, float2* work, size_t work_b,
                        const float2* tw, int Nx, int Ny, int px, int n_out, int npairs,
                        hipEvent_t ev0, hipEvent_t ev1) {
  const int gx = (Nx + kFxLines - 1) / kFxLines;
  const int chunk = (gx * Ny + 7) / 8;  // blocks per XCD
  const dim3 grid(8 * chunk);
  switch (L) {
#define SFW_FX_CASE(n, a, b)                                                                  \
  case n:                                                                                     \
    hipExtLaunchKernelGGL((k_fx_z_inverse<a, b>), grid, dim3(fx_threads(a, b)), 0, st, ev0,   \
                          ev1, 0, qhat, oct, oct_b, hx, hy, work, work_b, tw, Nx, Ny, px,      \
                          n_out, npairs, gx, chunk);                                           \
    return hipGetLastError();
    SFW_FX_LENGTHS(SFW_FX_CASE)
#undef SFW_FX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t fx_x_real(int L, dim3 grid, hipStream_t st, const float* q, int nx, int ny,
                     const float2* tw, int Ny, int px, float2* out) {
  switch (L) {
#define SFW_FX_CASE(n, a, b)                                                                 \
  case n:                                                                                    \
    hipLaunchKernelGGL((k_fx_x_real<a, b>), grid, dim3(fx_threads(a, b)), 0, st, q, nx, ny,  \
                       tw, Ny, px, out);                                                     \
    return hipGetLastError();
    SFW_FX_LENGTHS(SFW_FX_CASE)
#undef SFW_FX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t fx_x_argmax(int L, dim3 grid, hipStream_t st, const float2* work, size_t work_b,
                       int nx, int ny, int nz, const float2* tw, int Ny, int px, float scale,
                       int nslices, float* eta_out, ArgPart* apart, int nblk) {
  switch (L) {
#define SFW_FX_CASE(n, a, b)                                                                 \
  case n:                                                                                    \
    hipLaunchKernelGGL((k_fx_x_argmax<a, b>), grid, dim3(fx_threads(a, b)), 0, st, work,     \
                       work_b, nx, ny, nz, tw, Ny, px, scale, nslices, eta_out, apart, nblk); \
    return hipGetLastError();
    SFW_FX_LENGTHS(SFW_FX_CASE)
#undef SFW_FX_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace sfw
