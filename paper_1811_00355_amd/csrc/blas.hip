// Vector kernels for the Krylov solvers: multi-dot products with a
// deterministic two-stage reduction (per-workgroup partial sums, then a fixed
// order sum), multi-axpy, masked scaling, and the small per-RHS Hessenberg
// kernels (Givens rotations, least-squares back substitution).  All inner
// products accumulate in FP64.
//
// A vector set holds nrhs vectors of `count` complex entries at stride `rs`;
// a basis of such sets is spaced `vstride` pairs apart.
#include "dd_internal.h"
#include "ktimer.h"

namespace {

constexpr int kMaxNv = 16;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The basis kernels take the vector count nv at run time and a compile-time
// bound NV in {1, 2, 4, 8, 16}: loads of vectors past nv are clamped to vector
// nv - 1 (same cache lines) and their results discarded or weighted by zero,
// and each thread handles U = 8 / NV entries per trip (at least one), so all
// NV * U loads of a trip are issued before the first wait.
template <int NV>
constexpr int nv_unroll() { return NV >= 8 ? 1 : 8 / NV; }

// partial[r][i][blk] = <V_i[r], w[r]> over the blk-th of nblk equal chunks
template <int NV, typename Tv, typename Tw>
__global__ void __launch_bounds__(256) k_dots(int nrhs, long long count, long long rs, const Tv* __restrict__ V, int nv,
                                              long long vstride, const Tw* __restrict__ w, double* __restrict__ partial,
                                              int nblk, Gate gt) {
  if (gate_closed(gt)) return;
  constexpr int U = nv_unroll<NV>();
  __shared__ double red[4][2 * NV];
  const int r = blockIdx.y, blk = blockIdx.x;
  const long long chunk = (count + nblk - 1) / nblk;
  const long long e0 = (long long)blk * chunk, e1 = e0 + chunk < count ? e0 + chunk : count;
  cx<double> acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = {0.0, 0.0};
  const Tw* wr = w + (long long)r * rs;
  const Tv* vr = V + (long long)r * rs;
  for (long long b = e0 + threadIdx.x; b < e1; b += 256LL * U) {
    long long ek[U];
    Tw wraw[U];
    Tv vraw[NV][U];
#pragma unroll
    for (int u = 0; u < U; ++u) ek[u] = b + 256LL * u < e1 ? b + 256LL * u : e1 - 1;
#pragma unroll
    for (int u = 0; u < U; ++u) wraw[u] = wr[ek[u]];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const Tv* vi = vr + (long long)(i < nv ? i : nv - 1) * vstride;
#pragma unroll
      for (int u = 0; u < U; ++u) vraw[i][u] = vi[ek[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const cx<double> x = b + 256LL * u < e1 ? ld<double, Tw>(&wraw[u]) : cx<double>{0.0, 0.0};
#pragma unroll
      for (int i = 0; i < NV; ++i) cfma_conj(acc[i], ld<double, Tv>(&vraw[i][u]), x);
    }
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nv) {
      double a = wave_sum(acc[i].re), b = wave_sum(acc[i].im);
      if (lane == 0) {
        red[wv][2 * i] = a;
        red[wv][2 * i + 1] = b;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * nv) {
    double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    int i = threadIdx.x >> 1, c = threadIdx.x & 1;
    partial[(((long long)r * nv + i) * nblk + blk) * 2 + c] = s;
  }
}

// out[r * ldo + off + i] = sum over blocks of partial[r][i][blk]
__global__ void __launch_bounds__(256) k_reduce(int nv, int nblk, const double* __restrict__ partial,
                                                double2* __restrict__ out, int ldo, int off, Gate gt) {
  if (gate_closed(gt)) return;
  __shared__ double red[2][256];
  const int q = blockIdx.x;   // r * nv + i
  const int r = q / nv, i = q % nv;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    a += partial[((long long)q * nblk + k) * 2];
    b += partial[((long long)q * nblk + k) * 2 + 1];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(long long)r * ldo + off + i] = make_double2(red[0][0], red[1][0]);
}

// w[r] += sign * sum_{i < nv} coef[r * ldc + coff + i] * V_i[r]
template <int NV, typename Tv, typename Tw>
__global__ void __launch_bounds__(256) k_multi_axpy(int nrhs, long long count, long long rs, const Tv* __restrict__ V,
                                                    int nv, long long vstride, const double2* __restrict__ coef, int ldc,
                                                    int coff, double sign, Tw* __restrict__ w, Gate gt) {
  if (gate_closed(gt)) return;
  constexpr int U = nv_unroll<NV>();
  __shared__ cx<double> c[NV];
  const int r = blockIdx.y;
  if (threadIdx.x < NV) {
    const double2 v = threadIdx.x < nv ? coef[(long long)r * ldc + coff + threadIdx.x] : make_double2(0.0, 0.0);
    c[threadIdx.x] = {sign * v.x, sign * v.y};
  }
  __syncthreads();
  const Tv* vr = V + (long long)r * rs;
  Tw* wr = w + (long long)r * rs;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < count; b += stride * U) {
    long long ek[U];
    Tw wraw[U];
    Tv vraw[NV][U];
#pragma unroll
    for (int u = 0; u < U; ++u) ek[u] = b + stride * u < count ? b + stride * u : count - 1;
#pragma unroll
    for (int u = 0; u < U; ++u) wraw[u] = wr[ek[u]];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const Tv* vi = vr + (long long)(i < nv ? i : nv - 1) * vstride;
#pragma unroll
      for (int u = 0; u < U; ++u) vraw[i][u] = vi[ek[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cx<double> acc = ld<double, Tw>(&wraw[u]);
#pragma unroll
      for (int i = 0; i < NV; ++i) cfma(acc, c[i], ld<double, Tv>(&vraw[i][u]));
      if (b + stride * u < count) st<Tw, double>(wr + ek[u], acc);
    }
  }
}

// Fused CGS pieces for one sweep of the basis: w <- w - sum_i c_i V_i with the
// V_i kept in registers, then either the inner products <V_i, w> (NORM = false)
// or |w|^2 (NORM = true) of the updated w, reduced like k_dots.
template <int NV, typename Tv, typename Tw, bool NORM>
__global__ void __launch_bounds__(256) k_axpy_dots(int nrhs, long long count, long long rs, const Tv* __restrict__ V,
                                                   int nv, long long vstride, const double2* __restrict__ coef, int ldc,
                                                   Tw* __restrict__ w, double* __restrict__ partial, int nblk, Gate gt) {
  if (gate_closed(gt)) return;
  constexpr int U = nv_unroll<NV>();
  __shared__ double red[4][2 * NV];
  __shared__ cx<double> c[NV];
  const int r = blockIdx.y, blk = blockIdx.x;
  if (threadIdx.x < NV) {
    const double2 v = threadIdx.x < nv ? coef[(long long)r * ldc + threadIdx.x] : make_double2(0.0, 0.0);
    c[threadIdx.x] = {v.x, v.y};
  }
  __syncthreads();
  const long long chunk = (count + nblk - 1) / nblk;
  const long long e0 = (long long)blk * chunk, e1 = e0 + chunk < count ? e0 + chunk : count;
  cx<double> acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = {0.0, 0.0};
  Tw* wr = w + (long long)r * rs;
  const Tv* vr = V + (long long)r * rs;
  for (long long b = e0 + threadIdx.x; b < e1; b += 256LL * U) {
    long long ek[U];
    Tw wraw[U];
    Tv vraw[NV][U];
#pragma unroll
    for (int u = 0; u < U; ++u) ek[u] = b + 256LL * u < e1 ? b + 256LL * u : e1 - 1;
#pragma unroll
    for (int u = 0; u < U; ++u) wraw[u] = wr[ek[u]];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const Tv* vi = vr + (long long)(i < nv ? i : nv - 1) * vstride;
#pragma unroll
      for (int u = 0; u < U; ++u) vraw[i][u] = vi[ek[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = b + 256LL * u < e1;
      cx<double> x = ld<double, Tw>(&wraw[u]);
#pragma unroll
      for (int i = 0; i < NV; ++i) x = x - c[i] * ld<double, Tv>(&vraw[i][u]);
      if (ok) st<Tw, double>(wr + ek[u], x);
      if (!ok) x = {0.0, 0.0};
      if (NORM) {
        acc[0].re += x.re * x.re + x.im * x.im;
      } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) cfma_conj(acc[i], ld<double, Tv>(&vraw[i][u]), x);
      }
    }
  }
  const int nout = NORM ? 1 : nv;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nout) {
      double a = wave_sum(acc[i].re), b = wave_sum(acc[i].im);
      if (lane == 0) {
        red[wv][2 * i] = a;
        red[wv][2 * i + 1] = b;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * nout) {
    double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    int i = threadIdx.x >> 1, cc = threadIdx.x & 1;
    partial[(((long long)r * nout + i) * nblk + blk) * 2 + cc] = s;
  }
}

// Classical Gram-Schmidt against a whole basis (nv <= kGsMaxNv) in two passes:
// k_gs_dots forms <V_i, w> for every i, k_gs_axpy_norm then w <- w - sum c_i V_i
// and |w|^2.  A workgroup owns a fixed tile of 256 EPT entries (so the
// reduction tree depends on the vector length only); each thread keeps EPT
// entries of w in registers and streams kGsGroup basis vectors at a time, and
// a wave folds the 2 kGsGroup sums of its lanes with a butterfly that halves
// the set at every exchange.  Long vectors take EPT = 8; short ones (the
// coarse lattices of small volumes, the level-3 lattice) EPT = 1, so that
// they still spread over a few hundred workgroups.
constexpr int kGsGroup = 4, kGsMaxNv = 128;
constexpr long long kGsShort = 1LL << 17;   // entries per right-hand side up to which EPT = 1

// a[0..7] of every lane -> value (lane >> 3) summed over the wave (10 exchanges)
__device__ __forceinline__ double fold8(double* a, int lane) {
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double keep = hi ? a[4 + j] : a[j], send = hi ? a[j] : a[4 + j];
      a[j] = keep + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double keep = hi ? a[2 + j] : a[j], send = hi ? a[j] : a[2 + j];
      a[j] = keep + __shfl_xor(send, 16, 64);
    }
  }
  {
    const bool hi = lane & 8;
    const double keep = hi ? a[1] : a[0], send = hi ? a[0] : a[1];
    a[0] = keep + __shfl_xor(send, 8, 64);
  }
  double v = a[0];
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 1, 64);
  return v;
}

// The loads of a group carry no conditions (indices are clamped into the
// vectors and out-of-range terms are multiplied by zero), so a thread has all
// EPT * kGsGroup of them in flight at once.
template <typename Tv, typename Tw, int EPT>
__global__ void __launch_bounds__(256) k_gs_dots(int nrhs, long long count, long long rs, const Tv* __restrict__ V,
                                                 int nv, long long vstride, const Tw* __restrict__ w,
                                                 double* __restrict__ partial, int nblk, Gate gt) {
  if (gate_closed(gt)) return;
  static_assert(kGsGroup == 4, "fold8 folds 2 x 4 values");
  __shared__ double red[4][2 * kGsMaxNv];
  const int r = blockIdx.y, blk = blockIdx.x, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long e0 = (long long)blk * (256 * EPT) + threadIdx.x;
  const Tw* wr = w + (long long)r * rs;
  const Tv* vr = V + (long long)r * rs;
  cx<double> x[EPT];
  long long ek[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const long long e = e0 + 256LL * k;
    ek[k] = e < count ? e : count - 1;
    const cx<double> v = ld<double, Tw>(wr + ek[k]);
    x[k] = e < count ? v : cx<double>{0.0, 0.0};   // entries past the end contribute zero
  }
  for (int i0 = 0; i0 < nv; i0 += kGsGroup) {
    Tv raw[kGsGroup][EPT];
#pragma unroll
    for (int g = 0; g < kGsGroup; ++g) {
      const Tv* vi = vr + (long long)(i0 + g < nv ? i0 + g : nv - 1) * vstride;   // past nv: discarded below
#pragma unroll
      for (int k = 0; k < EPT; ++k) raw[g][k] = vi[ek[k]];
    }
    double a[2 * kGsGroup];
#pragma unroll
    for (int g = 0; g < kGsGroup; ++g) {
      cx<double> acc = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < EPT; ++k) cfma_conj(acc, ld<double, Tv>(&raw[g][k]), x[k]);
      a[2 * g] = acc.re;
      a[2 * g + 1] = acc.im;
    }
    const double s = fold8(a, lane);
    const int t = 2 * i0 + (lane >> 3);
    if ((lane & 7) == 0 && t < 2 * nv) red[wv][t] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 2 * nv; t += blockDim.x)
    partial[(((long long)r * nv + (t >> 1)) * nblk + blk) * 2 + (t & 1)] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

// w[r] <- w[r] - sum_{i < nv} coef[r * ldc + i] V_i[r], partial sums of |w|^2 over the same tiles
template <typename Tv, typename Tw, int EPT>
__global__ void __launch_bounds__(256) k_gs_axpy_norm(int nrhs, long long count, long long rs,
                                                      const Tv* __restrict__ V, int nv, long long vstride,
                                                      const double2* __restrict__ coef, int ldc, Tw* __restrict__ w,
                                                      double* __restrict__ partial, int nblk, Gate gt) {
  if (gate_closed(gt)) return;
  __shared__ cx<double> c[kGsMaxNv + kGsGroup];
  __shared__ double red[4];
  const int r = blockIdx.y, blk = blockIdx.x, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nvp = (nv + kGsGroup - 1) / kGsGroup * kGsGroup;
  for (int i = threadIdx.x; i < nvp; i += blockDim.x) {
    const double2 v = i < nv ? coef[(long long)r * ldc + i] : make_double2(0.0, 0.0);   // padding: zero weight
    c[i] = {v.x, v.y};
  }
  __syncthreads();
  const long long e0 = (long long)blk * (256 * EPT) + threadIdx.x;
  Tw* wr = w + (long long)r * rs;
  const Tv* vr = V + (long long)r * rs;
  cx<double> x[EPT];
  long long ek[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const long long e = e0 + 256LL * k;
    ek[k] = e < count ? e : count - 1;
    x[k] = ld<double, Tw>(wr + ek[k]);
  }
  for (int i0 = 0; i0 < nv; i0 += kGsGroup) {
    Tv raw[kGsGroup][EPT];
#pragma unroll
    for (int g = 0; g < kGsGroup; ++g) {
      const Tv* vi = vr + (long long)(i0 + g < nv ? i0 + g : nv - 1) * vstride;   // past nv: weight zero
#pragma unroll
      for (int k = 0; k < EPT; ++k) raw[g][k] = vi[ek[k]];
    }
#pragma unroll
    for (int g = 0; g < kGsGroup; ++g) {
      const cx<double> cg = c[i0 + g];
#pragma unroll
      for (int k = 0; k < EPT; ++k) x[k] = x[k] - cg * ld<double, Tv>(&raw[g][k]);
    }
  }
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const long long e = e0 + 256LL * k;
    if (e < count) {
      st<Tw, double>(wr + e, x[k]);
      n2 += x[k].re * x[k].re + x[k].im * x[k].im;
    }
  }
  n2 = wave_sum(n2);
  if (lane == 0) red[wv] = n2;
  __syncthreads();
  if (threadIdx.x < 2)
    partial[((long long)r * nblk + blk) * 2 + threadIdx.x] =
        threadIdx.x == 0 ? red[0] + red[1] + red[2] + red[3] : 0.0;
}

// dst[r] = src[r] / sqrt(nrm[r].x) where mask[r] != 0 (mask may be null); zero norm gives zero,
// and so does a masked-off r: whatever a finished or unused slot held before,
// the preconditioner then sees zeros there, never stale or uninitialised words
// (which x += 0 * M(v) would carry into a finished solution as NaN)
template <typename Ts, typename Td>
__global__ void __launch_bounds__(256) k_normalize(int nrhs, long long count, long long rs, const Ts* __restrict__ src,
                                                   const double2* __restrict__ nrm2, const double* __restrict__ nrm,
                                                   const int* __restrict__ mask, Td* __restrict__ dst,
                                                   float2* __restrict__ copy32, Gate gt) {
  if (gate_closed(gt)) return;
  const int r = blockIdx.y;
  const bool on = !(mask && !mask[r]);
  double n = nrm ? nrm[r] : sqrt(nrm2[r].x);
  double s = n > 0.0 ? 1.0 / n : 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (long long)gridDim.x * blockDim.x) {
    cx<double> v = on ? s * ld<double, Ts>(src + (long long)r * rs + e) : cx<double>{0.0, 0.0};
    Td q;
    st<Td, double>(&q, v);
    dst[(long long)r * rs + e] = q;
    if (copy32) {   // the stored (rounded) value, widened to FP32
      const cx<float> f = ld<float, Td>(&q);
      copy32[(long long)r * rs + e] = make_float2(f.re, f.im);
    }
  }
}

// out = a - b   (elementwise, same layout)
template <typename Tv>
__global__ void k_sub(long long n, const Tv* __restrict__ a, const Tv* __restrict__ b, Tv* __restrict__ out, Gate gt) {
  if (gate_closed(gt)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    cx<double> x = ld<double, Tv>(a + i), y = ld<double, Tv>(b + i);
    st<Tv, double>(out + i, x - y);
  }
}

// zero fill in 4-byte words (a kernel, so that it can sit inside a captured graph)
__global__ void k_zero(long long nwords, unsigned* __restrict__ p) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

template <typename Tv>
__global__ void k_add(long long n, const Tv* __restrict__ a, Tv* __restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    cx<double> x = ld<double, Tv>(a + i), y = ld<double, Tv>(out + i);
    st<Tv, double>(out + i, x + y);
  }
}

// ---------------------------------------------------------------------------
// per-RHS Hessenberg kernels (one thread per RHS)
// ---------------------------------------------------------------------------
// start of a cycle: g = (beta, 0, ...), active if beta > tolabs and not finished
__global__ void k_cycle_init(int nrhs, int m, const double2* __restrict__ nrm2, const double* __restrict__ tolabs,
                             const int* __restrict__ finished, double2* __restrict__ gv, double* __restrict__ beta,
                             int* __restrict__ active, int* __restrict__ kcyc, Gate gt) {
  if (gate_closed(gt)) return;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double b = sqrt(nrm2[r].x);
  beta[r] = b;
  for (int i = 0; i <= m; ++i) gv[r * (m + 1) + i] = make_double2(i == 0 ? b : 0.0, 0.0);
  active[r] = (!finished[r] && b > tolabs[r]) ? 1 : 0;
  kcyc[r] = 0;
}

// column j of the Hessenberg matrix from the two CGS passes and the norm, Givens update
__global__ void k_arnoldi(int nrhs, int m, int j, const double2* __restrict__ h1, const double2* __restrict__ h2,
                          const double2* __restrict__ nrm2, double2* __restrict__ H, double* __restrict__ cs,
                          double2* __restrict__ sn, double2* __restrict__ gv, const double* __restrict__ tolabs,
                          int* __restrict__ active, int* __restrict__ kcyc, double* __restrict__ est,
                          double* __restrict__ hnext, Gate gt) {
  if (gate_closed(gt)) return;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs || !active[r]) return;
  double2* Hc = H + ((long long)r * m + j) * (m + 1);   // column j
  for (int i = 0; i <= j; ++i) {
    double2 a = h1[r * (m + 1) + i], b = h2 ? h2[r * (m + 1) + i] : make_double2(0.0, 0.0);
    Hc[i] = make_double2(a.x + b.x, a.y + b.y);
  }
  double hn = sqrt(nrm2[r].x);
  Hc[j + 1] = make_double2(hn, 0.0);
  hnext[r] = hn;
  // previous rotations
  for (int i = 0; i < j; ++i) {
    cx<double> a = {Hc[i].x, Hc[i].y}, b = {Hc[i + 1].x, Hc[i + 1].y};
    cx<double> s = {sn[r * m + i].x, sn[r * m + i].y};
    double c = cs[r * m + i];
    cx<double> na = c * a + s * b;
    cx<double> nb = c * b - conj(s) * a;
    Hc[i] = make_double2(na.re, na.im);
    Hc[i + 1] = make_double2(nb.re, nb.im);
  }
  // new rotation zeroing H[j+1][j]: c real, [c s; -conj(s) c] [a; b] = [rho; 0]
  cx<double> a = {Hc[j].x, Hc[j].y};
  double bn = hn;
  double c;
  cx<double> s;
  double aa = sqrt(a.re * a.re + a.im * a.im);
  if (bn == 0.0) {
    c = 1.0;
    s = {0.0, 0.0};
  } else if (aa == 0.0) {
    c = 0.0;
    s = {1.0, 0.0};
  } else {
    double t = sqrt(aa * aa + bn * bn);
    c = aa / t;
    s = (bn / t) * cx<double>{a.re / aa, a.im / aa};   // (a/|a|) conj(b)/t with b = hn real
  }
  cs[r * m + j] = c;
  sn[r * m + j] = make_double2(s.re, s.im);
  cx<double> rho = c * a + s * cx<double>{bn, 0.0};
  Hc[j] = make_double2(rho.re, rho.im);
  Hc[j + 1] = make_double2(0.0, 0.0);
  cx<double> gj = {gv[r * (m + 1) + j].x, gv[r * (m + 1) + j].y};
  cx<double> g1 = -(conj(s) * gj);
  cx<double> g0 = c * gj;
  gv[r * (m + 1) + j] = make_double2(g0.re, g0.im);
  gv[r * (m + 1) + j + 1] = make_double2(g1.re, g1.im);
  double e = sqrt(g1.re * g1.re + g1.im * g1.im);
  est[r] = e;
  kcyc[r] = j + 1;
  if (e <= tolabs[r] || hn == 0.0 || j + 1 == m) active[r] = 0;
}

// y = R^-1 g over the kcyc[r] leading entries; y beyond kcyc is zero
__global__ void k_lsq(int nrhs, int m, const double2* __restrict__ H, const double2* __restrict__ gv,
                      const int* __restrict__ kcyc, double2* __restrict__ y, Gate gt) {
  if (gate_closed(gt)) return;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  int k = kcyc[r];
  for (int i = m - 1; i >= k; --i) y[r * m + i] = make_double2(0.0, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    cx<double> acc = {gv[r * (m + 1) + i].x, gv[r * (m + 1) + i].y};
    for (int q = i + 1; q < k; ++q) {
      double2 h = H[((long long)r * m + q) * (m + 1) + i];
      double2 yq = y[r * m + q];
      acc = acc - cx<double>{h.x, h.y} * cx<double>{yq.x, yq.y};
    }
    double2 d = H[((long long)r * m + i) * (m + 1) + i];
    double den = d.x * d.x + d.y * d.y;
    cx<double> inv = den > 0.0 ? cx<double>{d.x / den, -d.y / den} : cx<double>{0.0, 0.0};
    cx<double> v = acc * inv;
    y[r * m + i] = make_double2(v.re, v.im);
  }
}

// Wave-per-RHS forms of k_arnoldi and k_lsq for m <= 64: lane i holds entry i
// of the column, the rotations and the right-hand side, so the column is read
// and written once in parallel and only the recurrences run lane by lane
// (register exchanges instead of dependent global loads).
__device__ __forceinline__ cx<double> lane_get(cx<double> v, int i) {
  return {__shfl(v.re, i, 64), __shfl(v.im, i, 64)};
}

__global__ void __launch_bounds__(64) k_arnoldi_w(int m, int j, const double2* __restrict__ h1,
                                                  const double2* __restrict__ h2, const double2* __restrict__ nrm2,
                                                  double2* __restrict__ H, double* __restrict__ cs,
                                                  double2* __restrict__ sn, double2* __restrict__ gv,
                                                  const double* __restrict__ tolabs, int* __restrict__ active,
                                                  int* __restrict__ kcyc, double* __restrict__ est,
                                                  double* __restrict__ hnext, Gate gt) {
  if (gate_closed(gt)) return;
  const int r = blockIdx.x, lane = threadIdx.x;
  if (!active[r]) return;   // uniform per wave
  double2* Hc = H + ((long long)r * m + j) * (m + 1);   // column j
  cx<double> hc = {0.0, 0.0}, sl = {0.0, 0.0};
  double cl = 1.0;
  if (lane <= j) {
    const double2 a = h1[r * (m + 1) + lane], b = h2 ? h2[r * (m + 1) + lane] : make_double2(0.0, 0.0);
    hc = {a.x + b.x, a.y + b.y};
  }
  if (lane < j) {
    cl = cs[r * m + lane];
    const double2 v = sn[r * m + lane];
    sl = {v.x, v.y};
  }
  const double hn = sqrt(nrm2[r].x);
  // previous rotations, in order: (H_i, H_{i+1}) <- (c H_i + s H_{i+1}, c H_{i+1} - conj(s) H_i)
  cx<double> carry = lane_get(hc, 0), res = hc;
  for (int i = 0; i < j; ++i) {
    const cx<double> b = lane_get(hc, i + 1), s = lane_get(sl, i);
    const double c = __shfl(cl, i, 64);
    const cx<double> na = c * carry + s * b;
    carry = c * b - conj(s) * carry;
    if (lane == i) res = na;
  }
  // new rotation zeroing H[j+1][j]: c real, [c s; -conj(s) c] [a; b] = [rho; 0]
  const cx<double> a = carry;
  const double bn = hn;
  double c;
  cx<double> s;
  const double aa = sqrt(a.re * a.re + a.im * a.im);
  if (bn == 0.0) {
    c = 1.0;
    s = {0.0, 0.0};
  } else if (aa == 0.0) {
    c = 0.0;
    s = {1.0, 0.0};
  } else {
    const double t = sqrt(aa * aa + bn * bn);
    c = aa / t;
    s = (bn / t) * cx<double>{a.re / aa, a.im / aa};
  }
  const cx<double> rho = c * a + s * cx<double>{bn, 0.0};
  if (lane == j) res = rho;
  if (lane <= j) Hc[lane] = make_double2(res.re, res.im);
  if (lane == 0) {
    hnext[r] = hn;
    Hc[j + 1] = make_double2(0.0, 0.0);
    cs[r * m + j] = c;
    sn[r * m + j] = make_double2(s.re, s.im);
    const cx<double> gj = {gv[r * (m + 1) + j].x, gv[r * (m + 1) + j].y};
    const cx<double> g1 = -(conj(s) * gj);
    const cx<double> g0 = c * gj;
    gv[r * (m + 1) + j] = make_double2(g0.re, g0.im);
    gv[r * (m + 1) + j + 1] = make_double2(g1.re, g1.im);
    const double e = sqrt(g1.re * g1.re + g1.im * g1.im);
    est[r] = e;
    kcyc[r] = j + 1;
    if (e <= tolabs[r] || hn == 0.0 || j + 1 == m) active[r] = 0;
  }
}

// y = R^-1 g over the kcyc[r] leading entries (column-oriented back substitution); y beyond kcyc is zero
__global__ void __launch_bounds__(64) k_lsq_w(int m, const double2* __restrict__ H, const double2* __restrict__ gv,
                                              const int* __restrict__ kcyc, double2* __restrict__ y, Gate gt) {
  if (gate_closed(gt)) return;
  const int r = blockIdx.x, lane = threadIdx.x;
  const int k = kcyc[r];
  cx<double> g = {0.0, 0.0}, yl = {0.0, 0.0};
  if (lane < k) g = {gv[r * (m + 1) + lane].x, gv[r * (m + 1) + lane].y};
  for (int i = k - 1; i >= 0; --i) {
    const double2* Hi = H + ((long long)r * m + i) * (m + 1);   // column i
    const double2 d = Hi[i];
    const double den = d.x * d.x + d.y * d.y;
    const cx<double> inv = den > 0.0 ? cx<double>{d.x / den, -d.y / den} : cx<double>{0.0, 0.0};
    const cx<double> yi = lane_get(g, i) * inv;
    if (lane == i) yl = yi;
    if (lane < i) {
      const double2 h = Hi[lane];
      g = g - cx<double>{h.x, h.y} * yi;
    }
  }
  if (lane < m) y[r * m + lane] = make_double2(yl.re, yl.im);
}

// Device-side controls of the coarse GMRES when no host round trip is taken:
// the tolerance from |rhs'|, the finished marks after a cycle, a vector copy.
__global__ void k_set_tol(int nrhs, double tol, const double2* __restrict__ nrm2, double* __restrict__ tolabs,
                          int* __restrict__ finished, int* __restrict__ active) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  tolabs[r] = tol * sqrt(nrm2[r].x);
  finished[r] = 0;
  active[r] = 1;
}

// after a cycle: a right-hand side whose residual estimate met its tolerance is
// finished; the activity flags become "not finished" (the gate of the next
// cycle's residual kernels); the cycle's longest Arnoldi run is added to iters
__global__ void k_finish(int nrhs, const double* __restrict__ est, const double* __restrict__ tolabs,
                         int* __restrict__ finished, int* __restrict__ active, const int* __restrict__ kcyc,
                         int* __restrict__ iters, Gate gt) {
  if (gate_closed(gt)) return;
  __shared__ int kmax;
  if (threadIdx.x == 0) kmax = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < nrhs; r += blockDim.x) {
    if (est[r] <= tolabs[r]) finished[r] = 1;
    active[r] = finished[r] ? 0 : 1;
    atomicMax(&kmax, kcyc[r]);
  }
  __syncthreads();
  if (threadIdx.x == 0) *iters += kmax;
}

template <typename Tv>
__global__ void k_copy(long long n, const Tv* __restrict__ a, Tv* __restrict__ out, Gate gt) {
  if (gate_closed(gt)) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i];
}

inline unsigned grid1(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b > 65535 ? 65535 : b);
}

}  // namespace

// Workgroups per right-hand side for the two-stage reductions.  It depends on
// the vector length only, never on the number of right-hand sides, so the
// summation order of every RHS is the same alone and in a batch.
int dots_blocks(long long count, int /*nrhs*/) {
  long long per = 512;     // entries per workgroup, at least (2 per thread): short coarse vectors still fill the chip
  long long nb = (count + per - 1) / per;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return (int)nb;
}

namespace {
// BODY(NV) for the smallest bucket NV >= n (n <= 16)
#define DD_NV_BUCKET(n, BODY) \
  if ((n) <= 1) {             \
    BODY(1);                  \
  } else if ((n) <= 2) {      \
    BODY(2);                  \
  } else if ((n) <= 4) {      \
    BODY(4);                  \
  } else if ((n) <= 8) {      \
    BODY(8);                  \
  } else {                    \
    BODY(16);                 \
  }

template <typename Tv, typename Tw>
void dots_typed(dim3 grid, hipStream_t st, int nrhs, long long count, long long rs, const void* V, int n,
                long long vstride, const void* w, double* partial, int nblk) {
#define DD_DOTS(NV) \
  k_dots<NV, Tv, Tw><<<grid, 256, 0, st>>>(nrhs, count, rs, (const Tv*)V, n, vstride, (const Tw*)w, partial, nblk, current_gate())
  DD_NV_BUCKET(n, DD_DOTS)
#undef DD_DOTS
}

template <typename Tv, typename Tw>
void multi_axpy_typed(dim3 grid, hipStream_t st, int nrhs, long long count, long long rs, const void* V, int n,
                      long long vstride, const double2* coef, int ldc, int coff, double sign, void* w) {
#define DD_MAXPY(NV)                                                                                          \
  k_multi_axpy<NV, Tv, Tw><<<grid, 256, 0, st>>>(nrhs, count, rs, (const Tv*)V, n, vstride, coef, ldc, coff, sign, \
                                                  (Tw*)w, current_gate())
  DD_NV_BUCKET(n, DD_MAXPY)
#undef DD_MAXPY
}

template <typename Tv, typename Tw, bool NORM>
void axpy_dots_typed(dim3 grid, hipStream_t st, int nrhs, long long count, long long rs, const void* V, int n,
                     long long vstride, const double2* coef, int ldc, void* w, double* partial, int nblk) {
#define DD_AXD(NV)                                                                                                \
  k_axpy_dots<NV, Tv, Tw, NORM><<<grid, 256, 0, st>>>(nrhs, count, rs, (const Tv*)V, n, vstride, coef, ldc, (Tw*)w, \
                                                       partial, nblk, current_gate())
  DD_NV_BUCKET(n, DD_AXD)
#undef DD_AXD
}
#undef DD_NV_BUCKET
}  // namespace

void launch_dots(dd_dtype vt, dd_dtype wt, int nrhs, long long count, long long rs, const void* V, int nv,
                 long long vstride, const void* w, double* partial, int nblk, double2* out, int ldo, int off,
                 hipStream_t st) {
  for (int i0 = 0; i0 < nv; i0 += kMaxNv) {
    int n = nv - i0 < kMaxNv ? nv - i0 : kMaxNv;
    dim3 grid(nblk, nrhs);
    size_t es = vt == DD_F64 ? sizeof(double2) : vt == DD_F16 ? sizeof(__half2) : sizeof(float2);
    size_t ew = wt == DD_F64 ? sizeof(double2) : sizeof(float2);
    const void* Vi = (const char*)V + (size_t)i0 * vstride * es;
    // a norm (V = w, one vector) reads the vector once
    const double bytes = (double)nrhs * count * (Vi == w && n == 1 ? ew : n * es + ew), flops = 8.0 * nrhs * count * n;
    const bool timed = ktimer_enabled("k_dots");
    if (timed) ktimer_begin("k_dots", st);
    if (vt == DD_F64 && wt == DD_F64)
      dots_typed<double2, double2>(grid, st, nrhs, count, rs, Vi, n, vstride, w, partial, nblk);
    else if (vt == DD_F16 && wt == DD_F32)
      dots_typed<__half2, float2>(grid, st, nrhs, count, rs, Vi, n, vstride, w, partial, nblk);
    else if (vt != DD_F64 && wt != DD_F64)
      dots_typed<float2, float2>(grid, st, nrhs, count, rs, Vi, n, vstride, w, partial, nblk);
    else if (vt == DD_F64)
      dots_typed<double2, float2>(grid, st, nrhs, count, rs, Vi, n, vstride, w, partial, nblk);
    else
      dots_typed<float2, double2>(grid, st, nrhs, count, rs, Vi, n, vstride, w, partial, nblk);
    if (timed) ktimer_end("k_dots", st, bytes, flops);
    ktimer_account(bytes, flops);
    k_reduce<<<nrhs * n, 256, 0, st>>>(n, nblk, partial, out, ldo, off + i0, current_gate());
  }
}

void launch_multi_axpy(dd_dtype vt, dd_dtype wt, int nrhs, long long count, long long rs, const void* V, int nv,
                       long long vstride, const double2* coef, int ldc, int coff, double sign, void* w,
                       hipStream_t st) {
  for (int i0 = 0; i0 < nv; i0 += kMaxNv) {
    int n = nv - i0 < kMaxNv ? nv - i0 : kMaxNv;
    dim3 grid(grid1(count), nrhs);
    size_t es = vt == DD_F64 ? sizeof(double2) : vt == DD_F16 ? sizeof(__half2) : sizeof(float2);
    size_t ew = wt == DD_F64 ? sizeof(double2) : sizeof(float2);
    const void* Vi = (const char*)V + (size_t)i0 * vstride * es;
    const double bytes = (double)nrhs * count * (n * es + 2 * ew), flops = 8.0 * nrhs * count * n;
    const bool timed = ktimer_enabled("k_multi_axpy");
    if (timed) ktimer_begin("k_multi_axpy", st);
    if (vt == DD_F64 && wt == DD_F64)
      multi_axpy_typed<double2, double2>(grid, st, nrhs, count, rs, Vi, n, vstride, coef, ldc, coff + i0, sign, w);
    else if (vt == DD_F16 && wt == DD_F32)
      multi_axpy_typed<__half2, float2>(grid, st, nrhs, count, rs, Vi, n, vstride, coef, ldc, coff + i0, sign, w);
    else if (vt != DD_F64 && wt != DD_F64)
      multi_axpy_typed<float2, float2>(grid, st, nrhs, count, rs, Vi, n, vstride, coef, ldc, coff + i0, sign, w);
    else if (vt != DD_F64)
      multi_axpy_typed<float2, double2>(grid, st, nrhs, count, rs, Vi, n, vstride, coef, ldc, coff + i0, sign, w);
    else
      multi_axpy_typed<double2, float2>(grid, st, nrhs, count, rs, Vi, n, vstride, coef, ldc, coff + i0, sign, w);
    if (timed) ktimer_end("k_multi_axpy", st, bytes, flops);
    ktimer_account(bytes, flops);
  }
}

// basis V of dtype bt (DD_F16 only with FP32 vectors), vectors w of dtype vt
#define DD_BASIS_DISPATCH(NORMV)                                                                                    \
  if (vt == DD_F64)                                                                                                  \
    axpy_dots_typed<double2, double2, NORMV>(grid, st, nrhs, count, rs, V, nv, vstride, coef, ldc, w, partial, nblk); \
  else if (bt == DD_F16)                                                                                             \
    axpy_dots_typed<__half2, float2, NORMV>(grid, st, nrhs, count, rs, V, nv, vstride, coef, ldc, w, partial, nblk);  \
  else                                                                                                               \
    axpy_dots_typed<float2, float2, NORMV>(grid, st, nrhs, count, rs, V, nv, vstride, coef, ldc, w, partial, nblk);

void launch_axpy_dots(dd_dtype vt, int nrhs, long long count, long long rs, const void* V, int nv, long long vstride,
                      const double2* coef, int ldc, void* w, double* partial, int nblk, double2* out, int ldo,
                      hipStream_t st, dd_dtype bt) {
  dim3 grid(nblk, nrhs);
  const size_t es = vt == DD_F64 ? sizeof(double2) : sizeof(float2), eb = bt == DD_F16 ? 4 : es;
  const double bytes = (double)nrhs * count * (nv * eb + 2 * es), flops = 16.0 * nrhs * count * nv;
  DD_TIMED("k_axpy_dots", st, bytes, flops, DD_BASIS_DISPATCH(false));
  k_reduce<<<nrhs * nv, 256, 0, st>>>(nv, nblk, partial, out, ldo, 0, current_gate());
}

void launch_axpy_norm(dd_dtype vt, int nrhs, long long count, long long rs, const void* V, int nv, long long vstride,
                      const double2* coef, int ldc, void* w, double* partial, int nblk, double2* out, hipStream_t st,
                      dd_dtype bt) {
  dim3 grid(nblk, nrhs);
  const size_t es = vt == DD_F64 ? sizeof(double2) : sizeof(float2), eb = bt == DD_F16 ? 4 : es;
  const double bytes = (double)nrhs * count * (nv * eb + 2 * es), flops = 8.0 * nrhs * count * (nv + 1);
  DD_TIMED("k_axpy_norm", st, bytes, flops, DD_BASIS_DISPATCH(true));
  k_reduce<<<nrhs, 256, 0, st>>>(1, nblk, partial, out, 1, 0, current_gate());
}
#undef DD_BASIS_DISPATCH

int gs_max_nv() { return kGsMaxNv; }
static int gs_ept(long long count) { return count <= kGsShort ? 1 : 8; }
int gs_blocks(long long count) {
  const long long tile = 256LL * gs_ept(count);
  return (int)((count + tile - 1) / tile);
}

// basis V of dtype bt (DD_F16 only with FP32 vectors), vector w of dtype vt, EPT entries per thread
#define DD_GS_LAUNCH(KERNEL, EPT, ...)                                                                          \
  if (vt == DD_F64)                                                                                             \
    KERNEL<double2, double2, EPT><<<grid, 256, 0, st>>>(nrhs, count, rs, (const double2*)V, nv, vstride,        \
                                                        __VA_ARGS__, (double2*)w, partial, nblk, current_gate()); \
  else if (bt == DD_F16)                                                                                        \
    KERNEL<__half2, float2, EPT><<<grid, 256, 0, st>>>(nrhs, count, rs, (const __half2*)V, nv, vstride,         \
                                                       __VA_ARGS__, (float2*)w, partial, nblk, current_gate());  \
  else                                                                                                          \
    KERNEL<float2, float2, EPT><<<grid, 256, 0, st>>>(nrhs, count, rs, (const float2*)V, nv, vstride,           \
                                                      __VA_ARGS__, (float2*)w, partial, nblk, current_gate());
#define DD_GS_DISPATCH(KERNEL, ...)            \
  if (gs_ept(count) == 1) {                    \
    DD_GS_LAUNCH(KERNEL, 1, __VA_ARGS__)       \
  } else {                                     \
    DD_GS_LAUNCH(KERNEL, 8, __VA_ARGS__)       \
  }

void launch_gs_dots(dd_dtype bt, dd_dtype vt, int nrhs, long long count, long long rs, const void* V, int nv,
                    long long vstride, const void* w, double* partial, double2* out, int ldo, hipStream_t st) {
  const int nblk = gs_blocks(count);
  dim3 grid(nblk, nrhs);
  const size_t es = vt == DD_F64 ? sizeof(double2) : sizeof(float2), eb = bt == DD_F16 ? 4 : es;
  const double bytes = (double)nrhs * count * (nv * eb + es), flops = 8.0 * nrhs * count * nv;
#define DD_GS_DOTS(EPT)                                                                                          \
  if (vt == DD_F64)                                                                                              \
    k_gs_dots<double2, double2, EPT><<<grid, 256, 0, st>>>(nrhs, count, rs, (const double2*)V, nv, vstride,      \
                                                           (const double2*)w, partial, nblk, current_gate());     \
  else if (bt == DD_F16)                                                                                         \
    k_gs_dots<__half2, float2, EPT><<<grid, 256, 0, st>>>(nrhs, count, rs, (const __half2*)V, nv, vstride,       \
                                                          (const float2*)w, partial, nblk, current_gate());       \
  else                                                                                                           \
    k_gs_dots<float2, float2, EPT><<<grid, 256, 0, st>>>(nrhs, count, rs, (const float2*)V, nv, vstride,         \
                                                         (const float2*)w, partial, nblk, current_gate());
  if (gs_ept(count) == 1)
    DD_TIMED("k_gs_dots", st, bytes, flops, DD_GS_DOTS(1));
  else
    DD_TIMED("k_gs_dots", st, bytes, flops, DD_GS_DOTS(8));
#undef DD_GS_DOTS
  k_reduce<<<nrhs * nv, 256, 0, st>>>(nv, nblk, partial, out, ldo, 0, current_gate());
}

void launch_gs_axpy_norm(dd_dtype bt, dd_dtype vt, int nrhs, long long count, long long rs, const void* V, int nv,
                         long long vstride, const double2* coef, int ldc, void* w, double* partial, double2* out,
                         hipStream_t st) {
  const int nblk = gs_blocks(count);
  dim3 grid(nblk, nrhs);
  const size_t es = vt == DD_F64 ? sizeof(double2) : sizeof(float2), eb = bt == DD_F16 ? 4 : es;
  const double bytes = (double)nrhs * count * (nv * eb + 2 * es), flops = 8.0 * nrhs * count * (nv + 1);
  DD_TIMED("k_gs_axpy_norm", st, bytes, flops, DD_GS_DISPATCH(k_gs_axpy_norm, coef, ldc));
  k_reduce<<<nrhs, 256, 0, st>>>(1, nblk, partial, out, 1, 0, current_gate());
}
#undef DD_GS_DISPATCH
#undef DD_GS_LAUNCH

void launch_normalize(dd_dtype vt, int nrhs, long long count, long long rs, const void* src, const double2* nrm2,
                      const double* nrm, const int* mask, void* dst, hipStream_t st, dd_dtype dt, void* copy32) {
  dim3 grid(grid1(count), nrhs);
  if (vt == DD_F64)
    k_normalize<double2, double2><<<grid, 256, 0, st>>>(nrhs, count, rs, (const double2*)src, nrm2, nrm, mask,
                                                        (double2*)dst, (float2*)copy32, current_gate());
  else if (dt == DD_F16)
    k_normalize<float2, __half2><<<grid, 256, 0, st>>>(nrhs, count, rs, (const float2*)src, nrm2, nrm, mask,
                                                       (__half2*)dst, (float2*)copy32, current_gate());
  else
    k_normalize<float2, float2><<<grid, 256, 0, st>>>(nrhs, count, rs, (const float2*)src, nrm2, nrm, mask,
                                                      (float2*)dst, (float2*)copy32, current_gate());
}

void launch_sub(dd_dtype vt, long long n, const void* a, const void* b, void* out, hipStream_t st) {
  unsigned nb = (unsigned)((n + 255) / 256);
  if (vt == DD_F64)
    k_sub<double2><<<nb, 256, 0, st>>>(n, (const double2*)a, (const double2*)b, (double2*)out, current_gate());
  else
    k_sub<float2><<<nb, 256, 0, st>>>(n, (const float2*)a, (const float2*)b, (float2*)out, current_gate());
}

void launch_set_tol(int nrhs, double tol, const double2* nrm2, double* tolabs, int* finished, int* active,
                    hipStream_t st) {
  k_set_tol<<<(nrhs + 63) / 64, 64, 0, st>>>(nrhs, tol, nrm2, tolabs, finished, active);
}

void launch_finish(int nrhs, const double* est, const double* tolabs, int* finished, int* active, const int* kcyc,
                   int* iters, hipStream_t st) {
  k_finish<<<1, 64, 0, st>>>(nrhs, est, tolabs, finished, active, kcyc, iters, current_gate());
}

void launch_copy(dd_dtype vt, long long n, const void* a, void* out, hipStream_t st) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (vt == DD_F64) k_copy<double2><<<nb, 256, 0, st>>>(n, (const double2*)a, (double2*)out, current_gate());
  else k_copy<float2><<<nb, 256, 0, st>>>(n, (const float2*)a, (float2*)out, current_gate());
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  const long long nw = (long long)(bytes / 4);
  if (nw <= 0) return;
  k_zero<<<(unsigned)((nw + 255) / 256), 256, 0, st>>>(nw, (unsigned*)p);
}

void launch_add(dd_dtype vt, long long n, const void* a, void* out, hipStream_t st) {
  unsigned nb = (unsigned)((n + 255) / 256);
  if (vt == DD_F64)
    k_add<double2><<<nb, 256, 0, st>>>(n, (const double2*)a, (double2*)out);
  else
    k_add<float2><<<nb, 256, 0, st>>>(n, (const float2*)a, (float2*)out);
}

void launch_cycle_init(int nrhs, int m, const double2* nrm2, const double* tolabs, const int* finished, double2* gv,
                       double* beta, int* active, int* kcyc, hipStream_t st) {
  k_cycle_init<<<(nrhs + 63) / 64, 64, 0, st>>>(nrhs, m, nrm2, tolabs, finished, gv, beta, active, kcyc, current_gate());
}

void launch_arnoldi(int nrhs, int m, int j, const double2* h1, const double2* h2, const double2* nrm2, double2* H,
                    double* cs, double2* sn, double2* gv, const double* tolabs, int* active, int* kcyc, double* est,
                    double* hnext, hipStream_t st) {
  if (m <= 64)
    k_arnoldi_w<<<nrhs, 64, 0, st>>>(m, j, h1, h2, nrm2, H, cs, sn, gv, tolabs, active, kcyc, est, hnext, current_gate());
  else
    k_arnoldi<<<(nrhs + 63) / 64, 64, 0, st>>>(nrhs, m, j, h1, h2, nrm2, H, cs, sn, gv, tolabs, active, kcyc, est, hnext, current_gate());
}

void launch_lsq(int nrhs, int m, const double2* H, const double2* gv, const int* kcyc, double2* y, hipStream_t st) {
  if (m <= 64)
    k_lsq_w<<<nrhs, 64, 0, st>>>(m, H, gv, kcyc, y, current_gate());
  else
    k_lsq<<<(nrhs + 63) / 64, 64, 0, st>>>(nrhs, m, H, gv, kcyc, y, current_gate());
}

Gate& current_gate() {
  static thread_local Gate g;
  return g;
}
