// Grid certificate through the Fourier domain (the paper computes its convolutions there,
// section 2): eta_ij = correlation of q = Phi^T r with the tabulated unit atom of
// (sigma_i, d_j), for all 12 (or ns * nd) table kernels at once.
//
// q is zero-padded to an Nx x Ny x Nz grid with N_a >= max(n_a + R_max, 2 R_max + 1) on every
// axis, so the circular correlation equals the linear one on the volume. The table kernels are real and
// symmetric, so their spectra are real and two of them ride in one complex spectrum
// P = (K_a + i K_b)^ / N; one inverse transform of Qhat * P then yields eta_a + i eta_b.
// Transforms are separable passes of batched 1D mixed-radix (2, 3, 4, 5) Stockham FFTs in
// LDS; passes skip the rows that are known zero on input or not needed on output, and the
// last pass keeps the running maximum of eta (ties to the lowest flat index).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "sfw_internal.h"

namespace sfw {

namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }

// Forward DFT of size R in place (Y_k = sum_n x_n exp(-2 pi i n k / R)).
template <int R>
__device__ __forceinline__ void dft(float2* v);

template <>
__device__ __forceinline__ void dft<2>(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft<3>(float2* v) {
  const float s = 0.86602540378443865f;  // sin(2 pi / 3)
  const float2 t1 = cadd(v[1], v[2]);
  const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  const float2 d = csub(v[1], v[2]);
  const float2 t3 = make_float2(s * d.y, -s * d.x);  // -i s (x1 - x2)
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}

template <>
__device__ __forceinline__ void dft<4>(float2* v) {
  const float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  const float2 c = cadd(v[1], v[3]), d = mul_mi(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}

template <>
__device__ __forceinline__ void dft<5>(float2* v) {
  const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
  const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
  const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  const float2 x0 = v[0];
  const float2 p1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
  const float2 p2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
  // q1 = -i (s1 b1 + s2 b2), q2 = -i (s2 b1 - s1 b2)
  const float2 q1 = mul_mi(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
  const float2 q2 = mul_mi(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
  v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
  v[1] = cadd(p1, q1);
  v[4] = csub(p1, q1);
  v[2] = cadd(p2, q2);
  v[3] = csub(p2, q2);
}

constexpr int kFftThreads = 256;
constexpr int kFftBatch = 8;  // global loads in flight per thread while filling LDS

// One Stockham stage of radix R over 2^lgB lines of length L held in LDS (src -> dst, line
// pitch LS). Ns = product of the radices of the previous stages; tw[m] = exp(-2 pi i m / L).
// Tasks are mapped line-fastest so that line and butterfly index come from shifts; j / Ns is
// a multiply-high by ceil(2^32 / Ns), exact for j, Ns < 2^16. Each thread takes two tasks per
// round (the second clamped to the last task and not stored when out of range) so that both
// sets of LDS reads are in flight together.
template <int R>
__device__ __forceinline__ void stage(const float2* __restrict__ src, float2* __restrict__ dst,
                                      int L, int LS, int lgB, int Ns, const float2* __restrict__ tw) {
  const int per = L / R;
  const int tasks = per << lgB;
  const int tstep = L / (Ns * R);
  const unsigned mNs = Ns > 1 ? 0xffffffffu / (unsigned)Ns + 1u : 0u;
  const int B1 = (1 << lgB) - 1;
  for (int t0 = threadIdx.x; t0 < tasks; t0 += 2 * kFftThreads) {
    float2 v[2][R];
    int o[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = min(t0 + h * kFftThreads, tasks - 1);
      const int line = t & B1;
      const int j = t >> lgB;
      const int q = Ns > 1 ? (int)__umulhi((unsigned)j, mNs) : j;
      const int k = j - q * Ns;
      const float2* in = src + line * LS + j;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        v[h][r] = in[r * per];
        if (r > 0) v[h][r] = cmul(v[h][r], tw[r * k * tstep]);  // r k tstep < L
      }
      o[h] = line * LS + q * Ns * R + k;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      dft<R>(v[h]);
      if (t0 + h * kFftThreads < tasks) {
#pragma unroll
        for (int r = 0; r < R; ++r) dst[o[h] + r * Ns] = v[h][r];
      }
    }
  }
}

// Runs every stage of the plan; returns the LDS buffer holding the result.
__device__ float2* run_plan(float2* a, float2* b, int LS, int lgB, const FftAxis& ax,
                            const float2* tw) {
  const int L = ax.n;
  int Ns = 1;
  for (int s = 0; s < ax.nstage; ++s) {
    const int R = ax.radix[s];
    __syncthreads();
    switch (R) {
      case 2: stage<2>(a, b, L, LS, lgB, Ns, tw); break;
      case 3: stage<3>(a, b, L, LS, lgB, Ns, tw); break;
      case 4: stage<4>(a, b, L, LS, lgB, Ns, tw); break;
      default: stage<5>(a, b, L, LS, lgB, Ns, tw); break;
    }
    Ns *= R;
    float2* t = a;
    a = b;
    b = t;
  }
  __syncthreads();
  return a;
}

// LDS carve-up shared by the pass kernels: two line buffers of 2^lgB lines at pitch LS (odd,
// so 64-bit accesses of consecutive lines fall in distinct banks) and the twiddle table.
__device__ __forceinline__ int line_pitch(int L) { return L | 1; }

__device__ __forceinline__ float2* load_twiddles(float2* sm, int lgB, int LS, const FftAxis& ax) {
  float2* tw = sm + (2 << lgB) * LS;
  for (int i = threadIdx.x; i < ax.n; i += kFftThreads) tw[i] = ax.tw[i];
  return tw;
}

// e / L for e < 2^16 by multiply-high with ceil(2^32 / L).
__device__ __forceinline__ int div_by(int e, unsigned m) { return (int)__umulhi((unsigned)e, m); }

__device__ __forceinline__ bool arg_better(float v, long long i, float bv, long long bi) {
  return v > bv || (v == bv && i < bi);
}

// Fills LDS with `total` elements: get(e, ok) returns element e, loading from a clamped (always
// valid) address and returning zero when !ok; put(e, v) stores it. The loads of a batch are
// issued before any of them is waited on.
template <class Get, class Put>
__device__ __forceinline__ void fill_lds(int total, Get get, Put put) {
  for (int e0 = threadIdx.x; e0 < total; e0 += kFftBatch * kFftThreads) {
    float2 v[kFftBatch];
#pragma unroll
    for (int u = 0; u < kFftBatch; ++u) v[u] = get(e0 + u * kFftThreads);
#pragma unroll
    for (int u = 0; u < kFftBatch; ++u)
      if (e0 + u * kFftThreads < total) put(e0 + u * kFftThreads, v[u]);
  }
}

// ---------------------------------------------------------------- x passes (contiguous lines)
// Spectrum arrays are [z][y][x] with x pitch px (a multiple of 16 elements, so that the
// 16-column runs of the strided passes are whole 128-byte lines).

// Forward x pass of the real volume q: line (y, z) for y < ny, z < nz, zero beyond nx.
// out[(z * Ny + y) * px + i], i < Nx.
__global__ __launch_bounds__(kFftThreads) void k_fft_x_real(const float* __restrict__ q, int nx,
                                                            int ny, int nz, FftAxis ax, int Ny,
                                                            int px, int lgB,
                                                            float2* __restrict__ out) {
  extern __shared__ float2 sm[];
  const int L = ax.n, LS = line_pitch(L), B = 1 << lgB;
  const unsigned mL = 0xffffffffu / (unsigned)L + 1u;
  float2* a = sm;
  float2* b = sm + B * LS;
  const float2* tw = load_twiddles(sm, lgB, LS, ax);
  const int y0 = blockIdx.x * B, z = blockIdx.y;
  const int lines = min(B, ny - y0);
  const float* base = q + ((size_t)z * ny + y0) * nx;
  fill_lds(
      B * L,
      [&](int e) {
        const int l = div_by(e, mL), i = e - l * L;
        const bool ok = l < lines && i < nx;
        const float v = base[ok ? l * nx + i : 0];
        return make_float2(ok ? v : 0.f, 0.f);
      },
      [&](int e, float2 v) {
        const int l = div_by(e, mL), i = e - l * L;
        a[l * LS + i] = v;
      });
  float2* r = run_plan(a, b, LS, lgB, ax, tw);
  float2* obase = out + ((size_t)z * Ny + y0) * px;
  for (int e = threadIdx.x; e < lines * L; e += kFftThreads) {
    const int l = div_by(e, mL), i = e - l * L;
    obase[l * px + i] = r[l * LS + i];
  }
}

// Forward x pass of a complex array, every line of an Ny x Nz grid.
__global__ __launch_bounds__(kFftThreads) void k_fft_x_c2c(float2* __restrict__ data, FftAxis ax,
                                                           int Ny, int px, int lgB) {
  extern __shared__ float2 sm[];
  const int L = ax.n, LS = line_pitch(L), B = 1 << lgB;
  const unsigned mL = 0xffffffffu / (unsigned)L + 1u;
  float2* a = sm;
  float2* b = sm + B * LS;
  const float2* tw = load_twiddles(sm, lgB, LS, ax);
  const int y0 = blockIdx.x * B, z = blockIdx.y;
  const int lines = min(B, Ny - y0);
  float2* base = data + ((size_t)z * Ny + y0) * px;
  fill_lds(
      B * L,
      [&](int e) {
        const int l = div_by(e, mL), i = e - l * L;
        const bool ok = l < lines;
        const float2 v = base[ok ? l * px + i : 0];
        return ok ? v : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) {
        const int l = div_by(e, mL), i = e - l * L;
        a[l * LS + i] = v;
      });
  float2* r = run_plan(a, b, LS, lgB, ax, tw);
  for (int e = threadIdx.x; e < lines * L; e += kFftThreads) {
    const int l = div_by(e, mL), i = e - l * L;
    base[l * px + i] = r[l * LS + i];
  }
}

// Last inverse pass: line (y < ny, z < nz) of the work array of pair p = blockIdx.z, forward
// FFT, conjugated output; real part is eta of table kernel 2p, imaginary part eta of kernel
// 2p + 1 (if < nslices), times scale. Writes eta (optional) and the block maxima.
__global__ __launch_bounds__(kFftThreads) void k_fft_x_argmax(
    const float2* __restrict__ work, size_t work_bstride, int nx, int ny, int nz, FftAxis ax,
    int Ny, int px, int lgB, float scale, int nslices, float* __restrict__ eta_out,
    ArgPart* __restrict__ apart, int nblk) {
  const int slice_a = 2 * (int)blockIdx.z;
  const int slice_b = slice_a + 1 < nslices ? slice_a + 1 : -1;
  work += blockIdx.z * work_bstride;
  extern __shared__ float2 sm[];
  __shared__ float rv[2][kFftThreads / 64];
  __shared__ long long ri[2][kFftThreads / 64];
  const int L = ax.n, LS = line_pitch(L), B = 1 << lgB;
  const unsigned mL = 0xffffffffu / (unsigned)L + 1u;
  float2* a = sm;
  float2* b = sm + B * LS;
  const float2* tw = load_twiddles(sm, lgB, LS, ax);
  const int y0 = blockIdx.x * B, z = blockIdx.y;
  const int lines = min(B, ny - y0);
  const float2* base = work + ((size_t)z * Ny + y0) * px;
  fill_lds(
      B * L,
      [&](int e) {
        const int l = div_by(e, mL), i = e - l * L;
        const bool ok = l < lines;
        const float2 v = base[ok ? l * px + i : 0];
        return ok ? v : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) {
        const int l = div_by(e, mL), i = e - l * L;
        a[l * LS + i] = v;
      });
  float2* r = run_plan(a, b, LS, lgB, ax, tw);
  const long long V = (long long)nx * ny * nz;
  float bv[2] = {-INFINITY, -INFINITY};
  long long bi[2] = {0x7fffffffffffffffLL, 0x7fffffffffffffffLL};
  const int nxl = lines * nx;
  const unsigned mX = 0xffffffffu / (unsigned)nx + 1u;
  for (int e = threadIdx.x; e < nxl; e += kFftThreads) {
    const int l = div_by(e, mX), i = e - l * nx;
    const long long v = ((long long)z * ny + y0 + l) * nx + i;
    const float2 c = r[l * LS + i];
    const float ea = c.x * scale;
    const float eb = -c.y * scale;
    if (eta_out) {
      eta_out[(size_t)slice_a * V + v] = ea;
      if (slice_b >= 0) eta_out[(size_t)slice_b * V + v] = eb;
    }
    const long long ga = (long long)slice_a * V + v;
    if (arg_better(ea, ga, bv[0], bi[0])) {
      bv[0] = ea;
      bi[0] = ga;
    }
    if (slice_b >= 0) {
      const long long gb = (long long)slice_b * V + v;
      if (arg_better(eb, gb, bv[1], bi[1])) {
        bv[1] = eb;
        bi[1] = gb;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    for (int o = 32; o > 0; o >>= 1) {
      const float ov = __shfl_xor(bv[s], o, 64);
      const long long oi = __shfl_xor(bi[s], o, 64);
      if (arg_better(ov, oi, bv[s], bi[s])) {
        bv[s] = ov;
        bi[s] = oi;
      }
    }
    if ((threadIdx.x & 63) == 0) {
      rv[s][threadIdx.x >> 6] = bv[s];
      ri[s][threadIdx.x >> 6] = bi[s];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;  // < nblk
    for (int s = 0; s < 2; ++s) {
      if (s == 1 && slice_b < 0) break;
      float v = rv[s][0];
      long long id = ri[s][0];
      for (int w = 1; w < kFftThreads / 64; ++w)
        if (arg_better(rv[s][w], ri[s][w], v, id)) {
          v = rv[s][w];
          id = ri[s][w];
        }
      ArgPart ap;
      ap.val = v;
      ap.pad = 0;
      ap.idx = id;
      apart[(size_t)(s == 0 ? slice_a : slice_b) * nblk + blk] = ap;
    }
  }
}

// ---------------------------------------------------------------- strided passes (y or z)

// Lines along one axis with element stride `istride`; a block owns B adjacent x columns at
// one outer coordinate o (address o * ostride + i * istride + x) of batch entry blockIdx.z
// (arrays offset by blockIdx.z times their batch stride). Reads i < n_in (zero beyond), writes
// i < n_out. OCT (first inverse pass, lines along z, o = y): the input is conj(src * P) with P
// the pair spectrum of batch entry p = blockIdx.z read from its octant (hx x hy x hz,
// mulp + p * mul_bstride).
template <bool OCT>
__global__ __launch_bounds__(kFftThreads) void k_fft_strided(
    const float2* __restrict__ src, size_t src_bstride, const float2* __restrict__ mulp,
    size_t mul_bstride, float2* __restrict__ dst, size_t dst_bstride, FftAxis ax, int ncols,
    size_t istride, size_t ostride, int n_in, int n_out, int lgB, int hx, int hy, int Ny) {
  extern __shared__ float2 sm[];
  src += blockIdx.z * src_bstride;
  if (OCT) mulp += blockIdx.z * mul_bstride;
  dst += blockIdx.z * dst_bstride;
  const int L = ax.n, LS = line_pitch(L), B = 1 << lgB;
  float2* a = sm;
  float2* b = sm + B * LS;
  const float2* tw = load_twiddles(sm, lgB, LS, ax);
  const int x0 = blockIdx.x * B;
  const size_t obase = (size_t)blockIdx.y * ostride + x0;
  const int cols = min(B, ncols - x0);
  const int my = OCT ? (2 * (int)blockIdx.y <= Ny ? (int)blockIdx.y : Ny - (int)blockIdx.y) : 0;
  fill_lds(
      B * L,
      [&](int e) {
        const int i = e >> lgB, c = e & (B - 1);  // consecutive threads: consecutive columns
        const bool ok = c < cols && i < n_in;
        float2 v = src[obase + (ok ? (size_t)i * istride + c : 0)];
        if (OCT) {
          const int x = x0 + (ok ? c : 0);
          const int mx = 2 * x <= ncols ? x : ncols - x;
          const int iz = ok ? i : 0;
          const int mz = 2 * iz <= L ? iz : L - iz;
          v = cmul(v, mulp[((size_t)mz * hy + my) * hx + mx]);
          v.y = -v.y;
        }
        return ok ? v : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) {
        const int i = e >> lgB, c = e & (B - 1);
        a[c * LS + i] = v;
      });
  float2* r = run_plan(a, b, LS, lgB, ax, tw);
  for (int e = threadIdx.x; e < B * n_out; e += kFftThreads) {
    const int i = e >> lgB, c = e & (B - 1);
    if (c < cols) dst[obase + (size_t)i * istride + c] = r[c * LS + i];
  }
}

// Packs the k <= N / 2 octant of a full pair spectrum (x pitch px) densely, x fastest.
__global__ __launch_bounds__(256) void k_fft_pack_octant(const float2* __restrict__ full, int px,
                                                         int Ny, int hx, int hy, int hz,
                                                         float2* __restrict__ oct) {
  const size_t n = (size_t)hx * hy * hz;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int x = (int)(e % hx);
  const int y = (int)((e / hx) % hy);
  const int z = (int)(e / ((size_t)hx * hy));
  oct[e] = full[((size_t)z * Ny + y) * px + x];
}

// Kernel pair (a, b) of the table, wrapped around the origin of the Nx x Ny x Nz grid (x pitch
// px, padding columns zero): out = (K_a + i K_b) / N. Tables are [ky][kx][kzp] with radius R
// (2R + 1 taps per axis).
__global__ __launch_bounds__(256) void k_fft_scatter_pair(
    const float* __restrict__ ka, int ra, int kzpa, const float* __restrict__ kb, int rb,
    int kzpb, int Nx, int Ny, int Nz, int px, float inv_n, float2* __restrict__ out) {
  const size_t N = (size_t)px * Ny * Nz;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int x = (int)(i % px);
  const int y = (int)((i / px) % Ny);
  const int z = (int)(i / ((size_t)px * Ny));
  // signed offsets t in (-N/2, N/2]
  const int tx = x <= Nx / 2 ? x : x - Nx;
  const int ty = y <= Ny / 2 ? y : y - Ny;
  const int tz = z <= Nz / 2 ? z : z - Nz;
  float va = 0.f, vb = 0.f;
  if (x < Nx && abs(tx) <= ra && abs(ty) <= ra && abs(tz) <= ra) {
    const int P = 2 * ra + 1;
    va = ka[((size_t)(ty + ra) * P + (tx + ra)) * kzpa + (tz + ra)];
  }
  if (kb && x < Nx && abs(tx) <= rb && abs(ty) <= rb && abs(tz) <= rb) {
    const int P = 2 * rb + 1;
    vb = kb[((size_t)(ty + rb) * P + (tx + rb)) * kzpb + (tz + rb)];
  }
  out[i] = make_float2(va * inv_n, vb * inv_n);
}

}  // namespace

// ---------------------------------------------------------------- host side

static int good_size(int n) {
  for (int m = n;; ++m) {
    int t = m;
    for (int p : {2, 3, 5})
      while (t % p == 0) t /= p;
    if (t == 1) return m;
  }
}

// SFW_FFT=generic keeps every axis on the runtime-length passes (a test switch).
static bool fixed_lengths_enabled() {
  const char* env = std::getenv("SFW_FFT");
  return !(env && std::strcmp(env, "generic") == 0);
}

static bool make_axis_plan(int n, FftAxis& ax) {
  ax.n = n;
  ax.nstage = 0;
  int t = n;
  while (t % 4 == 0 && ax.nstage < kFftMaxStages) {
    ax.radix[ax.nstage++] = 4;
    t /= 4;
  }
  for (int p : {2, 3, 5})
    while (t % p == 0 && ax.nstage < kFftMaxStages) {
      ax.radix[ax.nstage++] = p;
      t /= p;
    }
  if (!fixed_lengths_enabled() || !fft_fixed_plan(n, &ax.r1, &ax.r2)) ax.r1 = ax.r2 = 0;
  return t == 1;
}

// Smallest transform length >= nmin: a fixed-length (two-stage) size when it is at most a
// quarter longer than the smallest 2-3-5-smooth size, whose generic passes cost about twice
// as much per element; else the smooth size.
static int choose_length(int nmin) {
  const int g = good_size(nmin);
  if (!fixed_lengths_enabled()) return g;
  int r1 = 0, r2 = 0;
  for (int L = nmin; L <= g + g / 4; ++L)
    if (fft_fixed_plan(L, &r1, &r2)) return L;
  return g;
}

// log2 of the lines per block and the dynamic LDS bytes of a generic pass over lines of
// length L.
static int fft_lg_lines(int L, bool strided) {
  int lg = strided ? 4 : 3;
  while (lg > 0 && ((size_t)2 * ((size_t)1 << lg) * (L | 1) + L) * sizeof(float2) > 48 * 1024)
    --lg;
  return lg;
}
static size_t fft_lds(int L, int lg) { return ((size_t)2 * ((size_t)1 << lg) * (L | 1) + L) * sizeof(float2); }

// Grid sizes: N >= n + R keeps wrapped reads of q off the volume, N >= 2R + 1 keeps the
// wrapped table kernel from overlapping itself; both make the circular correlation equal the
// linear one on the volume.
bool fft_plan_cert(sfw_dims vol, int rmax, FftPlan& pl) {
  pl.nx = choose_length(std::max(vol.nx + rmax, 2 * rmax + 1));
  pl.ny = choose_length(std::max(vol.ny + rmax, 2 * rmax + 1));
  pl.nz = choose_length(std::max(vol.nz + rmax, 2 * rmax + 1));
  pl.px = (pl.nx + 15) & ~15;
  pl.hx = pl.nx / 2 + 1;
  pl.hy = pl.ny / 2 + 1;
  pl.hz = pl.nz / 2 + 1;
  pl.oct = (size_t)pl.hx * pl.hy * pl.hz;
  if (pl.nx > kFftMaxLen || pl.ny > kFftMaxLen || pl.nz > kFftMaxLen) return false;
  return make_axis_plan(pl.nx, pl.ax[0]) && make_axis_plan(pl.ny, pl.ax[1]) &&
         make_axis_plan(pl.nz, pl.ax[2]);
}

void fft_twiddles(int n, std::vector<float2>& tw) {
  tw.resize(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * 3.14159265358979323846 * (double)m / (double)n;
    tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
}

// One strided pass (lines along y or z): fixed-length kernel when the axis has one.
static hipError_t strided_pass(const FftAxis& ax, unsigned outer, unsigned batch, hipStream_t st,
                               const float2* src, size_t src_b, float2* dst, size_t dst_b,
                               int ncols, size_t istride, size_t ostride, int n_in, int n_out) {
  if (ax.r1 > 0)
    return fx_strided(ax.n, dim3((ncols + kFxLines - 1) / kFxLines, outer, batch), st, src, src_b,
                      dst, dst_b, ax.tw, ncols, istride, ostride, n_in, n_out);
  const int g = fft_lg_lines(ax.n, true), B = 1 << g;
  hipLaunchKernelGGL(k_fft_strided<false>, dim3((ncols + B - 1) / B, outer, batch),
                     dim3(kFftThreads), fft_lds(ax.n, g), st, src, src_b, nullptr, (size_t)0, dst,
                     dst_b, ax, ncols, istride, ostride, n_in, n_out, g, 0, 0, 0);
  return hipGetLastError();
}

// Forward 3D transform of a complex array on the full grid (used for the table spectra).
hipError_t fft_forward_c2c(const FftPlan& pl, float2* data, hipStream_t st) {
  const int gx = fft_lg_lines(pl.nx, false), Bx = 1 << gx;
  hipLaunchKernelGGL(k_fft_x_c2c, dim3((pl.ny + Bx - 1) / Bx, pl.nz), dim3(kFftThreads),
                     fft_lds(pl.nx, gx), st, data, pl.ax[0], pl.ny, pl.px, gx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = strided_pass(pl.ax[1], pl.nz, 1, st, data, 0, data, 0, pl.nx, (size_t)pl.px,
                   (size_t)pl.px * pl.ny, pl.ny, pl.ny);
  if (e != hipSuccess) return e;
  return strided_pass(pl.ax[2], pl.ny, 1, st, data, 0, data, 0, pl.nx, (size_t)pl.px * pl.ny,
                      (size_t)pl.px, pl.nz, pl.nz);
}

hipError_t fft_scatter_pair(const FftPlan& pl, const float* ka, int ra, int kzpa, const float* kb,
                            int rb, int kzpb, float2* out, hipStream_t st) {
  const size_t N = (size_t)pl.nx * pl.ny * pl.nz;
  const size_t Np = (size_t)pl.px * pl.ny * pl.nz;
  hipLaunchKernelGGL(k_fft_scatter_pair, dim3((unsigned)((Np + 255) / 256)), dim3(256), 0, st, ka,
                     ra, kzpa, kb, rb, kzpb, pl.nx, pl.ny, pl.nz, pl.px,
                     (float)(1.0 / (double)N), out);
  return hipGetLastError();
}

// Qhat = FFT(q) with q zero-padded from the volume to the grid.
hipError_t fft_forward_volume(const FftPlan& pl, const float* q, sfw_dims vol, float2* qhat,
                              hipStream_t st) {
  hipError_t e;
  if (pl.ax[0].r1 > 0) {
    e = fx_x_real(pl.nx, dim3((vol.ny + kFxLines - 1) / kFxLines, vol.nz), st, q, vol.nx, vol.ny,
                  pl.ax[0].tw, pl.ny, pl.px, qhat);
  } else {
    const int gx = fft_lg_lines(pl.nx, false), Bx = 1 << gx;
    hipLaunchKernelGGL(k_fft_x_real, dim3((vol.ny + Bx - 1) / Bx, vol.nz), dim3(kFftThreads),
                       fft_lds(pl.nx, gx), st, q, vol.nx, vol.ny, vol.nz, pl.ax[0], pl.ny, pl.px,
                       gx, qhat);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  e = strided_pass(pl.ax[1], vol.nz, 1, st, qhat, 0, qhat, 0, pl.nx, (size_t)pl.px,
                   (size_t)pl.px * pl.ny, vol.ny, pl.ny);
  if (e != hipSuccess) return e;
  return strided_pass(pl.ax[2], pl.ny, 1, st, qhat, 0, qhat, 0, pl.nx, (size_t)pl.px * pl.ny,
                      (size_t)pl.px, vol.nz, pl.nz);
}

int fft_argmax_blocks(const FftPlan& pl, sfw_dims vol) {
  const int Bx = pl.ax[0].r1 > 0 ? kFxLines : 1 << fft_lg_lines(pl.nx, false);
  return ((vol.ny + Bx - 1) / Bx) * vol.nz;
}

hipError_t fft_pack_octant(const FftPlan& pl, const float2* full, float2* oct, hipStream_t st) {
  hipLaunchKernelGGL(k_fft_pack_octant, dim3((unsigned)((pl.oct + 255) / 256)), dim3(256), 0, st,
                     full, pl.px, pl.ny, pl.hx, pl.hy, pl.hz, oct);
  return hipGetLastError();
}

// eta_{2p} + i eta_{2p+1} = IFFT(Qhat * P_p) on the volume for every pair p < npairs at once
// (pair spectra as octants at a stride of pl.oct, work arrays at a stride of `bstride`
// elements), with the block maxima of every slice: the z pass here, then y and x below.
hipError_t fft_inverse_pairs_z(const FftPlan& pl, const float2* qhat, const float2* pairs,
                               float2* work, size_t bstride, int nslices, sfw_dims vol,
                               hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const unsigned np = (unsigned)((nslices + 1) / 2);
  if (pl.ax[2].r1 > 0)
    return fx_z_inverse(pl.nz, st, qhat, pairs, pl.oct, pl.hx, pl.hy, work, bstride,
                        pl.ax[2].tw, pl.nx, pl.ny, pl.px, vol.nz, (int)np, ev0, ev1);
  if (ev0) {
    const hipError_t e = hipEventRecord(ev0, st);
    if (e != hipSuccess) return e;
  }
  const int g = fft_lg_lines(pl.nz, true), B = 1 << g;
  hipLaunchKernelGGL(k_fft_strided<true>, dim3((pl.nx + B - 1) / B, pl.ny, np),
                     dim3(kFftThreads), fft_lds(pl.nz, g), st, qhat, (size_t)0, pairs, pl.oct,
                     work, bstride, pl.ax[2], pl.nx, (size_t)pl.px * pl.ny, (size_t)pl.px,
                     pl.nz, vol.nz, g, pl.hx, pl.hy, pl.ny);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess || !ev1) return e;
  return hipEventRecord(ev1, st);
}

hipError_t fft_inverse_pairs_yx(const FftPlan& pl, float2* work, size_t bstride, int nslices,
                                sfw_dims vol, float scale, float* eta_out, ArgPart* apart,
                                int nblk, hipStream_t st) {
  const unsigned np = (unsigned)((nslices + 1) / 2);
  hipError_t e = strided_pass(pl.ax[1], vol.nz, np, st, work, bstride, work, bstride, pl.nx,
                              (size_t)pl.px, (size_t)pl.px * pl.ny, pl.ny, vol.ny);
  if (e != hipSuccess) return e;
  if (pl.ax[0].r1 > 0)
    return fx_x_argmax(pl.nx, dim3((vol.ny + kFxLines - 1) / kFxLines, vol.nz, np), st, work,
                       bstride, vol.nx, vol.ny, vol.nz, pl.ax[0].tw, pl.ny, pl.px, scale,
                       nslices, eta_out, apart, nblk);
  const int gx = fft_lg_lines(pl.nx, false), Bx = 1 << gx;
  hipLaunchKernelGGL(k_fft_x_argmax, dim3((vol.ny + Bx - 1) / Bx, vol.nz, np), dim3(kFftThreads),
                     fft_lds(pl.nx, gx), st, work, bstride, vol.nx, vol.ny, vol.nz, pl.ax[0],
                     pl.ny, pl.px, gx, scale, nslices, eta_out, apart, nblk);
  return hipGetLastError();
}

}  // namespace sfw
