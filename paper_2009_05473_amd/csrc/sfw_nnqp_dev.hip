// The weights step's non-negative quadratic program on the device (algorithm 1 step 3,
// algorithm 2 step 3: the criterion of section 1.1 restricted to the weights): minimise
// 1/2 w'Gw - c'w over w >= 0 for many independent problems in one launch, one workgroup per
// problem (one wave for small problems in large batches, four waves otherwise), in float64.
//
// The method is the host solver's active-set method: shrink the full set until the solution on
// it is positive, then Lawson-Hanson steps from that feasible point, each solving G_PP z_P = c_P
// on the passive set P by a Cholesky factor (with the same two ridge retries for a singular
// G_PP). G's upper triangle is staged once into LDS and the factor of G_PP is built beside it,
// both packed by rows, so that both fit up to SFW_NNQP_MAX_K atoms. Every decision (which
// coordinate to free, the step back to feasibility, which coordinates leave P) is taken from
// values in LDS after a barrier, so the block's threads follow one control flow. A single problem
// is latency bound (each factor row is a chain of barriers, a square root and a divide); the
// kernel is for batches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "sfw.h"

namespace sfw {

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

namespace {

// NT threads per problem: 256 (four waves) in general, 64 (one wave, so the barriers cost next
// to nothing) for small problems in large batches; the one-wave kernel needs k <= 64.
constexpr int kMaxWaves = 4;
constexpr int kLoadBatch = 16;  // loads of G in flight per thread while it is staged

// Start of row a in the packed upper triangle of an m x m matrix (row a holds columns a..m-1).
__device__ inline int tri(int a, int m) { return a * (2 * m - a + 1) / 2; }

// Per-problem LDS (kmax = the launch's largest size, T = kmax (kmax + 1) / 2): G's upper
// triangle packed for the problem's size k [T], the factor's packed for the passive size n [T],
// then w, z, c and the reciprocal pivots [kmax each], the four waves' row sums [4][kmax], the
// reduction slots and ballot masks, then P and the passive flags [kmax ints each].
struct Lds {
  double *Gp, *Up;
  double *w, *z, *c, *invd, *part;
  double* redv;               // [kMaxWaves]
  unsigned long long* mask;   // [kMaxWaves]
  int* redi;                  // [kMaxWaves]
  int* P;
  int* passive;
  int kmax;
};

__device__ inline Lds carve(unsigned char* base, int kmax) {
  Lds s;
  s.kmax = kmax;
  const int T = kmax * (kmax + 1) / 2;
  double* d = reinterpret_cast<double*>(base);
  s.Gp = d;
  s.Up = d + T;
  d += 2 * (size_t)T;
  s.w = d;
  s.z = d + kmax;
  s.c = d + 2 * kmax;
  s.invd = d + 3 * kmax;
  s.part = d + 4 * kmax;
  s.redv = d + (4 + kMaxWaves) * kmax;
  s.mask = reinterpret_cast<unsigned long long*>(s.redv + kMaxWaves);
  int* i = reinterpret_cast<int*>(s.mask + kMaxWaves);
  s.redi = i;
  s.P = i + kMaxWaves;
  s.passive = s.P + kmax;
  return s;
}

size_t lds_bytes(int kmax) {
  const size_t T = (size_t)kmax * (kmax + 1) / 2;
  return sizeof(double) * (2 * T + (4 + kMaxWaves) * (size_t)kmax + 2 * kMaxWaves) +
         sizeof(int) * (kMaxWaves + 2 * (size_t)kmax);
}

// Lane l's value of a double, on every lane (l uniform).
__device__ inline double readlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Smallest value over the block with its index (ties: the smaller index; NaN never wins).
// Every thread gets the result.
template <int NT>
__device__ void block_argmin(const Lds& s, double v, int idx, double* vout, int* iout) {
  constexpr int kWaves = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (!(v == v)) {
    v = INFINITY;
    idx = 0x7fffffff;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov < v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (lane == 0) {
    s.redv[wave] = v;
    s.redi[wave] = idx;
  }
  __syncthreads();
  double bv = s.redv[0];
  int bi = s.redi[0];
  for (int q = 1; q < kWaves; ++q)
    if (s.redv[q] < bv || (s.redv[q] == bv && s.redi[q] < bi)) {
      bv = s.redv[q];
      bi = s.redi[q];
    }
  __syncthreads();  // the slots are free again
  *vout = bv;
  *iout = bi;
}

// P = the passive coordinates in increasing order (thread i < k owns flag i: k <= NT); returns
// |P| to every thread.
template <int NT>
__device__ int build_passive(const Lds& s, int k) {
  constexpr int kWaves = NT / 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const bool on = t < k && s.passive[t];
  const unsigned long long m = __ballot(on);
  if (lane == 0) s.mask[wave] = m;
  __syncthreads();
  int before = 0, total = 0;
  for (int q = 0; q < kWaves; ++q) {
    const int c = __popcll(s.mask[q]);
    before += q < wave ? c : 0;
    total += c;
  }
  if (on) s.P[before + __popcll(m & ((1ull << lane) - 1ull))] = t;
  __syncthreads();
  return total;
}

// A = U'U for the n x n matrix whose upper triangle is packed in Up, row by row:
// U_ij = (A_ij - sum_{k<i} U_ki U_kj) / U_ii for j > i, with U_ii^2 the same expression at j = i.
// Wave q sums the terms k = q, q + 4, ... of every column; the four sums are added after a
// barrier. Row i overwrites A's row i except the pivot, whose reciprocal goes to invd.
// False (on every thread) if a pivot is not positive.
template <int NT>
__device__ bool cholesky(const Lds& s, int n) {
  constexpr int kWaves = NT / 64;
  const int t = threadIdx.x, lane = t & 63, q = t >> 6, km = s.kmax;
  // the waves' sums of column jj, added in a fixed order
  auto wave_sums = [&](int jj) {
    if (kWaves == 4) return (s.part[jj] + s.part[km + jj]) + (s.part[2 * km + jj] + s.part[3 * km + jj]);
    return s.part[jj];
  };
  double* U = s.Up;
  for (int i = 0; i < n; ++i) {
    const int oi = tri(i, n) - i;  // U_ij at oi + j
    for (int jj = lane; jj < n - i; jj += 64) {
      const int j = i + jj;
      double acc = 0.0;
      // U_kx at ok + x with ok = k (2n - k - 1) / 2, which grows by W (2n - 2k - W - 1) / 2
      // from k to k + W (W = kWaves), that step shrinking by W^2 each time
      int ok = q * (2 * n - q - 1) / 2, dk = kWaves * (2 * n - 2 * q - kWaves - 1) / 2;
      for (int k = q; k < i; k += kWaves) {
        acc += U[ok + i] * U[ok + j];
        ok += dk;
        dk -= kWaves * kWaves;
      }
      s.part[q * km + jj] = acc;
    }
    __syncthreads();
    const double d = U[oi + i] - wave_sums(0);
    if (!(d > 0.0)) return false;
    const double inv = 1.0 / sqrt(d);
    for (int jj = t + 1; jj < n - i; jj += NT) U[oi + i + jj] = (U[oi + i + jj] - wave_sums(jj)) * inv;
    if (t == 0) s.invd[i] = inv;
    __syncthreads();
  }
  return true;
}

// z_P = G_PP^{-1} c_P and z = 0 off P, with the ridges 1e-12 and 1e-6 times the mean diagonal
// added when G_PP is not positive definite (duplicate atoms make it singular).
template <int NT>
__device__ void solve_passive(const Lds& s, int k, int n) {
  constexpr int kWaves = NT / 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int i = t; i < k; i += NT) s.z[i] = 0.0;
  for (int r = 0; r < 3; ++r) {
    double ridge = 0.0;
    if (r > 0) {  // mean diagonal of G_PP (only once a factorisation has failed)
      double tr = 0.0;
      for (int a = 0; a < n; ++a) tr += s.Gp[tri(s.P[a], k)];
      ridge = (r == 1 ? 1e-12 : 1e-6) * (tr / (double)n);
    }
    for (int a = wave; a < n; a += kWaves) {
      const int pa = s.P[a], oa = tri(a, n) - a, ga = tri(pa, k) - pa;
      for (int b = a + lane; b < n; b += 64)
        s.Up[oa + b] = s.Gp[ga + s.P[b]] + (b == a ? ridge : 0.0);
    }
    __syncthreads();
    if (cholesky<NT>(s, n)) break;
    __syncthreads();
  }
  // U' t = c_P, then U x = t, by wave 0 alone: lane l holds unknowns l and l + 64 in registers and
  // each step broadcasts the one just found, so the steps need no barrier.
  if (t < 64) {
    const int l = t;
    double b0 = l < n ? s.c[s.P[l]] : 0.0;
    double b1 = l + 64 < n ? s.c[s.P[l + 64]] : 0.0;
    int oi = 0;  // U_ij at oi + j: i (2n - i - 1) / 2, which grows by n - i - 1 from i to i + 1
    for (int i = 0; i < n; ++i) {
      const double ti = readlane(i < 64 ? b0 : b1, i & 63) * s.invd[i];
      if (l > i && l < n) b0 -= s.Up[oi + l] * ti;
      if (l + 64 > i && l + 64 < n) b1 -= s.Up[oi + l + 64] * ti;
      if (l == (i & 63)) {
        if (i < 64)
          b0 = ti;
        else
          b1 = ti;
      }
      oi += n - i - 1;
    }
    const int ol0 = l * (2 * n - l - 1) / 2, ol1 = (l + 64) * (2 * n - l - 65) / 2;
    for (int i = n - 1; i >= 0; --i) {
      const double xi = readlane(i < 64 ? b0 : b1, i & 63) * s.invd[i];
      if (l < i) b0 -= s.Up[ol0 + i] * xi;
      if (l + 64 < i) b1 -= s.Up[ol1 + i] * xi;
      if (l == (i & 63)) {
        if (i < 64)
          b0 = xi;
        else
          b1 = xi;
      }
    }
    if (l < n) s.z[s.P[l]] = b0;
    if (l + 64 < n) s.z[s.P[l + 64]] = b1;
  }
  __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void k_nnqp(const double* __restrict__ Gall,
                                                   const double* __restrict__ Call,
                                                   const int* __restrict__ ks, int kmax,
                                                   double* __restrict__ Wall,
                                                   int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const Lds s = carve(lds_raw, kmax);
  const int p = blockIdx.x, t = threadIdx.x;
  const int k = ks ? min(max(ks[p], 0), kmax) : kmax;
  const double* G = Gall + (size_t)p * kmax * kmax;
  double* W = Wall + (size_t)p * kmax;
  // stage G's upper triangle, kLoadBatch loads in flight per thread
  for (int base = 0; base < k * k; base += NT * kLoadBatch) {
    double v[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = base + u * NT + t, a = e / k, b = e - a * k;
      v[u] = e < k * k && b >= a ? G[(size_t)a * kmax + b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = base + u * NT + t, a = e / k, b = e - a * k;
      if (e < k * k && b >= a) s.Gp[tri(a, k) + b - a] = v[u];
    }
  }
  for (int i = t; i < kmax; i += NT) {
    s.w[i] = 0.0;
    s.passive[i] = i < k;
    s.c[i] = i < k ? Call[(size_t)p * kmax + i] : 0.0;
  }
  __syncthreads();
  int solves = 0, nP = 0;  // nP: size of the last passive set built (w vanishes off it)
  bool capped = false;
  // Phase 1: from the full set, drop every coordinate whose solution is not positive until the
  // solution on what remains is positive (a feasible point; with nothing dropped, the KKT
  // point of the strictly convex problem).
  for (int round = 0; round < k; ++round) {
    const int n = build_passive<NT>(s, k);
    nP = n;
    if (n == 0) break;
    solve_passive<NT>(s, k, n);
    ++solves;
    int bad = 0;
    for (int q = t; q < n; q += NT) {
      const int i = s.P[q];
      if (!(s.z[i] > 0.0)) {
        s.passive[i] = 0;
        bad = 1;
      }
    }
    if (!__syncthreads_or(bad)) {
      for (int i = t; i < k; i += NT) s.w[i] = s.z[i];
      __syncthreads();
      break;
    }
  }
  // Phase 2: Lawson-Hanson from the feasible point: free the coordinate with the most negative
  // gradient, solve on P and step back to feasibility, until the KKT conditions hold.
  double scale = 0.0;
  for (int i = 0; i < k; ++i) scale = fmax(scale, fabs(s.c[i]));
  const double tol = 1e-13 * fmax(scale, 1e-300);
  const int cap = 4 * k + 20;
  int outer = 0;
  for (; outer < cap; ++outer) {
    // gradient G w - c off P: w vanishes off the last passive set, so the sum runs over it;
    // with 256 threads, threads i and i + 128 take its two halves for coordinate i (k <= 128),
    // with 64, thread i takes all of it (k <= 64)
    constexpr int CH = NT >= 256 ? 128 : NT, HALVES = NT / CH;
    {
      const int i = t % CH, h = t / CH, mid = nP / 2;
      if (i < k && !s.passive[i]) {
        double acc = 0.0;
        const int q0 = HALVES == 2 && h ? mid : 0, q1 = HALVES == 2 && !h ? mid : nP;
        for (int q = q0; q < q1; ++q) {
          const int j = s.P[q], a = min(i, j), b = max(i, j);
          acc += s.Gp[tri(a, k) + b - a] * s.w[j];
        }
        s.part[h * kmax + i] = acc;
      }
    }
    __syncthreads();
    double g = INFINITY;
    int gi = 0x7fffffff;
    if (t < k && !s.passive[t]) {
      const double acc = (HALVES == 2 ? s.part[t] + s.part[kmax + t] : s.part[t]) - s.c[t];
      if (acc < -tol) {
        g = acc;
        gi = t;
      }
    }
    double gbest;
    int jbest;
    block_argmin<NT>(s, g, gi, &gbest, &jbest);
    if (jbest == 0x7fffffff) break;
    if (t == 0) s.passive[jbest] = 1;
    __syncthreads();
    int inner = 0;
    for (; inner < cap; ++inner) {
      const int n = build_passive<NT>(s, k);
      nP = n;
      solve_passive<NT>(s, k, n);
      ++solves;
      int bad = 0;
      double a = 1.0;
      for (int q = t; q < n; q += NT) {
        const int i = s.P[q];
        if (!(s.z[i] > 0.0)) {
          bad = 1;
          const double den = s.w[i] - s.z[i];
          a = fmin(a, den > 0.0 ? s.w[i] / den : 0.0);
        }
      }
      if (!__syncthreads_or(bad)) {
        for (int i = t; i < k; i += NT) s.w[i] = s.z[i];
        __syncthreads();
        break;
      }
      double alpha;
      int unused;
      block_argmin<NT>(s, a, 0, &alpha, &unused);
      for (int i = t; i < k; i += NT) s.w[i] += alpha * (s.z[i] - s.w[i]);
      __syncthreads();
      int moved = 0;
      for (int q = t; q < n; q += NT) {
        const int i = s.P[q];
        if (s.w[i] <= 1e-15 * fmax(1.0, fabs(s.z[i]))) {
          s.passive[i] = 0;
          s.w[i] = 0.0;
          moved = 1;
        }
      }
      if (!__syncthreads_or(moved)) {  // numerically stuck: drop the most negative member
        double zv = INFINITY;
        int zi = 0x7fffffff;
        for (int q = t; q < n; q += NT) {
          const int i = s.P[q];
          if (s.z[i] < zv || (s.z[i] == zv && i < zi)) {
            zv = s.z[i];
            zi = i;
          }
        }
        double zmin;
        int worst;
        block_argmin<NT>(s, zv, zi, &zmin, &worst);
        if (worst == 0x7fffffff) worst = s.P[0];  // every z was NaN
        if (t == 0) {
          s.passive[worst] = 0;
          s.w[worst] = 0.0;
        }
        __syncthreads();
      }
    }
    if (inner == cap) capped = true;
  }
  if (outer == cap) capped = true;
  for (int i = t; i < kmax; i += NT) W[i] = i < k ? s.w[i] : 0.0;
  if (info && t == 0) info[p] = capped ? -solves : solves;
}

}  // namespace

}  // namespace sfw

using namespace sfw;

extern "C" int sfw_nnqp_batch(const double* G, const double* c, const int* k, int kmax,
                              int count, double* w, int* info, hipStream_t stream) {
  try {
    if (count < 0 || kmax < 0) return fail(SFW_EINVAL, "count and kmax must be >= 0");
    if (kmax > SFW_NNQP_MAX_K) return fail(SFW_EINVAL, "kmax above SFW_NNQP_MAX_K");
    if (count == 0 || kmax == 0) return SFW_OK;
    if (!G || !c || !w) return fail(SFW_EINVAL, "G, c or w is NULL");
    const size_t bytes = lds_bytes(kmax);
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_nnqp<256>), hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)lds_bytes(SFW_NNQP_MAX_K));
    if (attr != hipSuccess) return hip_fail(attr, "hipFuncSetAttribute(k_nnqp)");
    static const hipError_t attr64 = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_nnqp<64>), hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)lds_bytes(64));
    if (attr64 != hipSuccess) return hip_fail(attr64, "hipFuncSetAttribute(k_nnqp)");
    // one wave per problem where it is faster (measured, 4,096 problems: 99 against 265 us at 16
    // atoms, 773 against 1,019 at 40, 1,177 against 1,068 at 50; one problem alone: four waves
    // from 24 atoms on)
    const bool one_wave = kmax <= 16 || (kmax <= 40 && count >= 256);
    if (one_wave)
      hipLaunchKernelGGL(k_nnqp<64>, dim3((unsigned)count), dim3(64), bytes, stream, G, c, k,
                         kmax, w, info);
    else
      hipLaunchKernelGGL(k_nnqp<256>, dim3((unsigned)count), dim3(256), bytes, stream, G, c, k,
                         kmax, w, info);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_nnqp");
    return SFW_OK;
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_nnqp_batch");
  }
}
