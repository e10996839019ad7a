// Inter-grid transfer and coarse-operator construction (Sec. 2).
//   restriction,  Eq. (3): b_c(X, s, i) = <lambda_i(X, s) | b>
//   prolongation, Eq. (4): x = sum_{X,s,i} x_c(X, s, i) lambda_i(X, s)
//   Gram-Schmidt of every chirality-split aggregate of the test vectors (FP64)
//   Galerkin operator, Eq. (2): D_c(X,s,i; Y,t,j) = <lambda_i(X,s)| D |lambda_j(Y,t)>
//
// Test vectors are stored like n packed fine vectors ([n][12][V] pairs); the
// aggregate X is the contiguous site range of block slot X, chirality s covers
// spin components 6s..6s+5.  Coarse vectors are [rhs][Vc][2n] pairs with
// component s*n + i; coarse-operator blocks are [Vc][9][col][row] (column major).
#include <type_traits>

#include "dslash.h"
#include "ktimer.h"

namespace {

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// restriction: one workgroup per (aggregate, rhs), one thread per site
// ---------------------------------------------------------------------------
template <int N, typename R, typename Sp, typename Tv, typename To>
__global__ void __launch_bounds__(256) k_restrict(GeomDev g, const Sp* __restrict__ P, int nrhs, const Tv* __restrict__ fine,
                                                  To* __restrict__ out, long long rstride, long long sstride) {
  __shared__ R red[4][4 * N];
  int slot, r;
  xcd_tile_rhs(nrhs, slot, r);
  if (slot >= g.Vc) return;
  const int j = threadIdx.x;
  const long long V = g.V;
  cx<R> d[2 * N];
#pragma unroll
  for (int k = 0; k < 2 * N; ++k) d[k] = {(R)0, (R)0};
  if (j < g.Bv) {
    const long long I = ((long long)slot << g.lBv) + j;
    cx<R> v[12];
    load_spinor<R, Tv>(fine + (long long)r * 12 * V, V, I, v);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const Sp* li = P + (long long)i * 12 * V + I;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        cx<R> l = ld<R, Sp>(li + (long long)c * V);
        cfma_conj(d[(c < 6 ? 0 : N) + i], l, v[c]);
      }
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < 2 * N; ++k) {
    R a = wave_sum(d[k].re), b = wave_sum(d[k].im);
    if (lane == 0) {
      red[w][2 * k] = a;
      red[w][2 * k + 1] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * N) {
    int k = threadIdx.x;
    R a = 0, b = 0;
    for (int q = 0; q < nw; ++q) {
      a += red[q][2 * k];
      b += red[q][2 * k + 1];
    }
    st<To, R>(out + r * rstride + slot * sstride + k, cx<R>{a, b});
  }
}

// ---------------------------------------------------------------------------
// restriction on matrix cores (4^4 aggregates, FP32 vectors): one workgroup per
// aggregate for up to 16 right-hand sides at a time, so the aggregate's test
// vectors are read once.  Per chirality s the result is the complex product
// (n x 6*256) . (6*256 x rhs) of conj(lambda) and the fine vector.  Wave w takes
// sites 64w .. 64w+63; per spin-colour component c the wave stages the 64 sites
// of v (16 RHS) and of the n test vectors in LDS with coalesced loads, then runs
// 16 k-steps of v_mfma_f32_16x16x4f32 over the sites, three real products per
// complex one (Gauss: with conj(lambda) = a + ib, v = c + id: a (c + d),
// (a + b)(-d), (b - a) c).  The four waves' partial sums are added in wave order.
// Each wave stages into LDS of its own and synchronises with itself only, so the
// four waves' load and product phases interleave; the FP64 form (Galerkin
// build) stages 32 sites per step, the two lane halves taking half of the
// right-hand sides and of the test vectors each.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename R> struct Mfma4;
// Output layouts differ: element v of lane group lk holds row 4 lk + v (FP32 form)
// or row lk + 4 v (FP64 form) of column lane % 16.
template <> struct Mfma4<float> {
  typedef f32x4 acc;
  typedef float2 vec;
  __device__ static acc op(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct Mfma4<double> {
  typedef f64x4 acc;
  typedef double2 vec;
  __device__ static acc op(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int v) { return lk + 4 * v; }
};

// order LDS accesses of one wave: its writes are visible to its later reads, and
// its reads are done before its later writes (a wave's LDS instructions
// complete in order; this keeps the compiler from moving them across)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// R: FP32 (inner solve) or FP64 (Galerkin build); SW: sites per staging step of a wave
template <int N, typename Sp, typename R, int SW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_restrict_mfma(GeomDev g, const Sp* __restrict__ P, int nrhs,
                                                       const typename Mfma4<R>::vec* __restrict__ fine,
                                                       typename Mfma4<R>::vec* __restrict__ out, long long rstride,
                                                       long long sstride) {
  typedef Mfma4<R> M;
  typedef typename M::acc acc_t;
  typedef typename M::vec Tv;
  constexpr int MT = (N + 15) / 16, SP = SW + 1;   // row tiles of the n test vectors; padded site stride
  constexpr int KU = SW == 32 ? 2 : 4;             // k-steps unrolled (FP64: fewer LDS values in flight)
  // staging of v and lambda; after each chirality the same bytes hold the waves' partial sums [w][row][rhs]
  constexpr size_t kVs = sizeof(Tv) * 4 * 16 * SP, kPs = sizeof(Sp) * 4 * N * SP, kRed = sizeof(Tv) * 4 * N * 16;
  __shared__ __align__(16) char smem[kVs + kPs > kRed ? kVs + kPs : kRed];
  Tv(*vs)[16][SP] = reinterpret_cast<Tv(*)[16][SP]>(smem);
  Sp(*ps)[N][SP] = reinterpret_cast<Sp(*)[N][SP]>(smem + kVs);
  Tv(*red)[N][16] = reinterpret_cast<Tv(*)[N][16]>(smem);
  const int slot = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const long long V = g.V, base = ((long long)slot << g.lBv) + 64 * w;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = nrhs - r0 < 16 ? nrhs - r0 : 16;
    const bool rhs_ok = li < nr;
    for (int s = 0; s < 2; ++s) {
      acc_t k1[MT], k2[MT], k3[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) k1[t] = k2[t] = k3[t] = acc_t{0, 0, 0, 0};
      for (int cc = 0; cc < 6; ++cc) {
        const int c = 6 * s + cc;
        for (int h = 0; h < 64 / SW; ++h) {
          if constexpr (SW == 32) {
            // 32 sites per step: lane half hf stages right-hand sides 8 hf .. 8 hf + 7 and
            // test vectors hf N/2 .. (hf + 1) N/2 - 1 of site lane % 32
            const int hf = lane >> 5, sl = lane & 31;
            const long long site = base + h * SW + sl;
            Tv xv[8];
            Sp pv[N / 2];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int r = 8 * hf + q;
              xv[q] = fine[(long long)(r0 + (r < nr ? r : 0)) * 12 * V + (long long)c * V + site];
            }
#pragma unroll
            for (int q = 0; q < N / 2; ++q) pv[q] = P[((long long)(hf * (N / 2) + q) * 12 + c) * V + site];
#pragma unroll
            for (int q = 0; q < 8; ++q) vs[w][8 * hf + q][sl] = xv[q];
#pragma unroll
            for (int q = 0; q < N / 2; ++q) ps[w][hf * (N / 2) + q][sl] = pv[q];
          } else {
            const long long site = base + h * SW + (lane < SW ? lane : 0);
            Tv xv[16];
            Sp pv[N];
#pragma unroll
            for (int r = 0; r < 16; ++r)
              xv[r] = fine[(long long)(r0 + (r < nr ? r : 0)) * 12 * V + (long long)c * V + site];
#pragma unroll
            for (int i = 0; i < N; ++i) pv[i] = P[((long long)i * 12 + c) * V + site];
            if (lane < SW) {
#pragma unroll
              for (int r = 0; r < 16; ++r) vs[w][r][lane] = xv[r];
#pragma unroll
              for (int i = 0; i < N; ++i) ps[w][i][lane] = pv[i];
            }
          }
          wave_sync();   // the staging is this wave's own: the other waves go at their own pace
#pragma unroll(KU)
          for (int ks = 0; ks < SW / 4; ++ks) {
            const Tv xb = vs[w][li][4 * ks + lk];
            const R xc = rhs_ok ? xb.x : (R)0, xd = rhs_ok ? xb.y : (R)0;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
              const int i = 16 * t + li;
              const cx<R> l = i < N ? ld<R, Sp>(&ps[w][i < N ? i : 0][4 * ks + lk]) : cx<R>{(R)0, (R)0};
              const R a = l.re, b = -l.im;   // conj(lambda)
              k1[t] = M::op(a, xc + xd, k1[t]);
              k2[t] = M::op(a + b, -xd, k2[t]);
              k3[t] = M::op(b - a, xc, k3[t]);
            }
          }
          wave_sync();   // every read of this wave's staging is done before it is refilled
        }
      }
      __syncthreads();   // the partial sums below reuse every wave's staging bytes
      // this wave's partial result: lane holds rows 16t + M::row(lk, v) of right-hand side li
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * t + M::row(lk, v);
          if (row < N) red[w][row][li] = Tv{k1[t][v] + k2[t][v], k1[t][v] + k3[t][v]};
        }
      __syncthreads();
      for (int e = threadIdx.x; e < N * 16; e += blockDim.x) {
        const int r = e / N, row = e - r * N;
        if (r < nr) {
          const Tv a = red[0][row][r], b = red[1][row][r], c = red[2][row][r], d = red[3][row][r];
          out[(long long)(r0 + r) * rstride + (long long)slot * sstride + s * N + row] =
              Tv{((a.x + b.x) + c.x) + d.x, ((a.y + b.y) + c.y) + d.y};
        }
      }
      __syncthreads();   // the staging buffer is refilled next
    }
  }
}

// ---------------------------------------------------------------------------
// prolongation on matrix cores (4^4 aggregates, FP32 vectors): one workgroup per
// aggregate for up to 16 right-hand sides at a time.  Per spin-colour component
// c (chirality s = c / 6) the fine values of the aggregate's sites are the
// complex product (sites x n) . (n x rhs) of lambda_i(site, c) and the coarse
// vector's chirality-s block.  Wave w takes sites 64w .. 64w+63 as four 16-row
// tiles; the n test-vector values of its sites are staged in LDS per component
// (coalesced), the coarse vectors once per pass.  Three real MFMAs per complex
// product as in the restriction.
// ---------------------------------------------------------------------------
template <int N, typename Sp>
__global__ void __launch_bounds__(256) k_prolong_mfma(GeomDev g, const Sp* __restrict__ P, int nrhs,
                                                      const float2* __restrict__ coarse, float2* __restrict__ fine) {
  constexpr int KS = (N + 3) / 4, SP = 65;
  __shared__ Sp ps[4][N][SP];
  __shared__ float2 xs[16][2 * N + 1];
  const int slot = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const long long V = g.V, base = ((long long)slot << g.lBv) + 64 * w;
  const int nc = 2 * N;
  for (int r0 = 0; r0 < nrhs; r0 += 16) {
    const int nr = nrhs - r0 < 16 ? nrhs - r0 : 16;
    __syncthreads();   // the previous pass's reads of xs are done
    for (int e = threadIdx.x; e < 16 * nc; e += blockDim.x) {
      const int r = e / nc, k = e - r * nc;
      xs[r][k] = r < nr ? coarse[((long long)(r0 + r) * g.Vc + slot) * nc + k] : make_float2(0.f, 0.f);
    }
    for (int c = 0; c < 12; ++c) {
      const int s = c / 6;
      Sp pv[N];
#pragma unroll
      for (int i = 0; i < N; ++i) pv[i] = P[((long long)i * 12 + c) * V + base + lane];
      __syncthreads();   // xs is written (first component); the previous component's reads of ps are done
#pragma unroll
      for (int i = 0; i < N; ++i) ps[w][i][lane] = pv[i];
      __syncthreads();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 k1 = {0.f, 0.f, 0.f, 0.f}, k2 = k1, k3 = k1;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int i = 4 * ks + lk;
          const cx<float> l = i < N ? ld<float, Sp>(&ps[w][i < N ? i : 0][16 * t + li]) : cx<float>{0.f, 0.f};
          const float2 xb = i < N ? xs[li][s * N + i] : make_float2(0.f, 0.f);
          k1 = __builtin_amdgcn_mfma_f32_16x16x4f32(l.re, xb.x + xb.y, k1, 0, 0, 0);
          k2 = __builtin_amdgcn_mfma_f32_16x16x4f32(l.re + l.im, -xb.y, k2, 0, 0, 0);
          k3 = __builtin_amdgcn_mfma_f32_16x16x4f32(l.im - l.re, xb.x, k3, 0, 0, 0);
        }
        // lane holds sites 16t + 4lk + v of right-hand side li
        if (li < nr) {
          float2* o = fine + (long long)(r0 + li) * 12 * V + (long long)c * V + base + 16 * t + 4 * lk;
#pragma unroll
          for (int v = 0; v < 4; ++v) o[v] = make_float2(k1[v] + k2[v], k1[v] + k3[v]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// prolongation: one workgroup per (aggregate, rhs), one thread per site
// ---------------------------------------------------------------------------
template <typename R, typename Sp, typename Tv>
__global__ void __launch_bounds__(256) k_prolong(GeomDev g, int n, const Sp* __restrict__ P, int nrhs,
                                                 const Tv* __restrict__ coarse, Tv* __restrict__ fine) {
  __shared__ cx<R> c[128];
  int slot, r;
  xcd_tile_rhs(nrhs, slot, r);
  if (slot >= g.Vc) return;
  const int j = threadIdx.x;
  const int nc = 2 * n;
  const long long V = g.V;
  if (j < nc) c[j] = ld<R, Tv>(coarse + ((long long)r * g.Vc + slot) * nc + j);
  __syncthreads();
  if (j >= g.Bv) return;
  const long long I = ((long long)slot << g.lBv) + j;
  cx<R> o[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) o[q] = {(R)0, (R)0};
  for (int i = 0; i < n; ++i) {
    const Sp* li = P + (long long)i * 12 * V + I;
    cx<R> cp = c[i], cm = c[n + i];
#pragma unroll
    for (int q = 0; q < 12; ++q) cfma(o[q], q < 6 ? cp : cm, ld<R, Sp>(li + (long long)q * V));
  }
  store_spinor<R, Tv>(fine + (long long)r * 12 * V, V, I, o);
}

// ---------------------------------------------------------------------------
// two-pass modified Gram-Schmidt per (aggregate, chirality), FP64, in place
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  a = b = 0.0;
  for (int q = 0; q < nw; ++q) {
    a += red[2 * q];
    b += red[2 * q + 1];
  }
}

__global__ void __launch_bounds__(256) k_gram_schmidt(GeomDev g, int n, double2* __restrict__ P, int* bad) {
  __shared__ double red[16];
  const int slot = blockIdx.x >> 1, s = blockIdx.x & 1;
  const int j = threadIdx.x;
  const bool act = j < g.Bv;
  const long long V = g.V;
  const long long I = ((long long)slot << g.lBv) + (act ? j : 0);
  for (int i = 0; i < n; ++i) {
    cx<double> v[6];
    double2* vi = P + (long long)i * 12 * V + (long long)(6 * s) * V + I;
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = act ? ld<double, double2>(vi + c * V) : cx<double>{0.0, 0.0};
    double n0 = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) n0 += v[c].re * v[c].re + v[c].im * v[c].im;
    double dummy = 0.0;
    block_sum2(n0, dummy, red);
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < i; ++q) {
        const double2* vq = P + (long long)q * 12 * V + (long long)(6 * s) * V + I;
        cx<double> u[6];
        cx<double> dt = {0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          u[c] = act ? ld<double, double2>(vq + c * V) : cx<double>{0.0, 0.0};
          cfma_conj(dt, u[c], v[c]);
        }
        block_sum2(dt.re, dt.im, red);
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = v[c] - dt * u[c];
      }
    double nn = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) nn += v[c].re * v[c].re + v[c].im * v[c].im;
    block_sum2(nn, dummy, red);
    double nrm = sqrt(nn);
    if (nrm <= 1e-12 * sqrt(n0)) {
      if (threadIdx.x == 0) atomicCAS(bad, -1, 2 * slot + s);
      nrm = 1.0;
    }
    double inv = 1.0 / nrm;
    if (act)
#pragma unroll
      for (int c = 0; c < 6; ++c) st<double2, double>(vi + c * V, inv * v[c]);
  }
}

// ---------------------------------------------------------------------------
// pieces of D applied to the chirality-split test vectors, for the Galerkin build.
// Column col = t*n + jv is phi = Pi_t lambda_jv.  Piece d = 0: the operator kept
// inside every domain (clover + hops between sites of the same domain); d = 1..4:
// the forward hop in direction d-1 from sites whose neighbour lies in the next
// domain; d = 5..8: the backward hop in direction d-5 across the domain face.
// ---------------------------------------------------------------------------
template <typename R, typename Sp>
__device__ __forceinline__ void load_phi(const Sp* P, long long V, int jv, int t, long long J, cx<R>* p) {
  const Sp* l = P + (long long)jv * 12 * V + J;
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = ((c < 6) == (t == 0)) ? ld<R, Sp>(l + (long long)c * V) : cx<R>{(R)0, (R)0};
}

template <int MU, int SGN, typename R, typename S>
__device__ __forceinline__ void face_hop(const GeomDev& g, const S* links, const SiteLoc& s, long long I,
                                         const cx<R>* psi_nb, long long J, bool wrap, cx<R>* acc) {
  cx<R> h[6], uh[6], u[9];
  project<MU, (SGN > 0 ? -1 : +1), R>(psi_nb, h);
  load_link<R, S>(links, g.V, MU, SGN > 0 ? I : J, u);
  if (SGN > 0) su3_mul_half<R>(u, h, uh);
  else su3_dag_mul_half<R>(u, h, uh);
  reconstruct_acc<MU, (SGN > 0 ? -1 : +1), R>(uh, (R)(wrap ? -0.5 * g.bc_t : -0.5), acc);
}

template <int MU, int SGN, typename R, typename S, typename Sp>
__device__ __forceinline__ void face_piece(const GeomDev& g, const S* links, const Sp* P, int jv, int t,
                                           const SiteLoc& s, long long I, cx<R>* acc) {
  bool wrap, inside;
  long long J = neighbor(g, s, MU, SGN, wrap, inside);
  if (inside) return;
  cx<R> psi[12];
  load_phi<R, Sp>(P, g.V, jv, t, J, psi);
  face_hop<MU, SGN, R, S>(g, links, s, I, psi, J, wrap, acc);
}

template <typename R, typename S, typename Sp>
__global__ void __launch_bounds__(256) k_coarse_piece(GeomDev g, const S* __restrict__ links, const S* __restrict__ clov,
                                                      const Sp* __restrict__ P, int n, int col0, int ncol, int d,
                                                      double2* __restrict__ W) {
  int tile, cl;
  xcd_tile_rhs(ncol, tile, cl);
  const int col = col0 + cl;
  const long long I = (long long)tile * blockDim.x + threadIdx.x;
  if (I >= g.V) return;
  const int t = col / n, jv = col % n;
  SiteLoc s = decode_site(g, I);
  cx<R> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {(R)0, (R)0};
  if (d == 0) {
    cx<R> phi[12];
    load_phi<R, Sp>(P, g.V, jv, t, I, phi);
    clover_mul<R, S, false>(clov, g.V, I, phi, acc);
    auto fetch = [&](long long J, bool, cx<R>* p) { load_phi<R, Sp>(P, g.V, jv, t, J, p); };
    hop_all<R, S>(g, links, s, I, true, fetch, acc);
  } else {
    switch (d) {
      case 1: face_piece<0, +1, R, S, Sp>(g, links, P, jv, t, s, I, acc); break;
      case 2: face_piece<1, +1, R, S, Sp>(g, links, P, jv, t, s, I, acc); break;
      case 3: face_piece<2, +1, R, S, Sp>(g, links, P, jv, t, s, I, acc); break;
      case 4: face_piece<3, +1, R, S, Sp>(g, links, P, jv, t, s, I, acc); break;
      case 5: face_piece<0, -1, R, S, Sp>(g, links, P, jv, t, s, I, acc); break;
      case 6: face_piece<1, -1, R, S, Sp>(g, links, P, jv, t, s, I, acc); break;
      case 7: face_piece<2, -1, R, S, Sp>(g, links, P, jv, t, s, I, acc); break;
      default: face_piece<3, -1, R, S, Sp>(g, links, P, jv, t, s, I, acc); break;
    }
  }
  store_spinor<R, double2>(W + (long long)cl * 12 * g.V, g.V, I, acc);
}

// ---------------------------------------------------------------------------
// inverses of the odd-site self blocks: Gauss-Jordan with partial pivoting in FP64
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_coarse_invert(GeomDev g, int nc, const double2* __restrict__ Dc,
                                                       double2* __restrict__ Dinv, int* bad) {
  extern __shared__ double2 M[];   // [nc][2 nc] row major, augmented with the identity
  __shared__ int piv_s;
  __shared__ double2 fac[64];
  const int oslot = blockIdx.x;             // odd site index in [0, Vch)
  const int X = g.Vch + oslot;
  const int w2 = 2 * nc;
  const double2* A = Dc + (long long)X * 9 * nc * nc;   // self block, [col][row]
  for (int e = threadIdx.x; e < nc * w2; e += blockDim.x) {
    int r = e / w2, c = e % w2;
    M[e] = (c < nc) ? A[(long long)c * nc + r] : make_double2(c - nc == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < nc; ++k) {
    if (threadIdx.x == 0) {
      int p = k;
      double best = -1.0;
      for (int r = k; r < nc; ++r) {
        double2 v = M[r * w2 + k];
        double a = v.x * v.x + v.y * v.y;
        if (a > best) { best = a; p = r; }
      }
      if (best == 0.0) atomicCAS(bad, -1, X);
      piv_s = p;
    }
    __syncthreads();
    int p = piv_s;
    if (p != k)
      for (int c = threadIdx.x; c < w2; c += blockDim.x) {
        double2 t = M[k * w2 + c];
        M[k * w2 + c] = M[p * w2 + c];
        M[p * w2 + c] = t;
      }
    __syncthreads();
    double2 pv = M[k * w2 + k];
    double den = pv.x * pv.x + pv.y * pv.y;
    cx<double> pinv = den > 0.0 ? cx<double>{pv.x / den, -pv.y / den} : cx<double>{0.0, 0.0};
    __syncthreads();
    for (int c = threadIdx.x; c < w2; c += blockDim.x) {
      cx<double> v = ld<double, double2>(&M[k * w2 + c]);
      st<double2, double>(&M[k * w2 + c], v * pinv);
    }
    for (int r = threadIdx.x; r < nc; r += blockDim.x) fac[r] = M[r * w2 + k];
    __syncthreads();
    for (int e = threadIdx.x; e < nc * w2; e += blockDim.x) {
      int r = e / w2, c = e % w2;
      if (r == k) continue;
      cx<double> f = {fac[r].x, fac[r].y};
      cx<double> v = ld<double, double2>(&M[e]);
      cx<double> kk = ld<double, double2>(&M[k * w2 + c]);
      st<double2, double>(&M[e], v - f * kk);
    }
    __syncthreads();
  }
  double2* out = Dinv + (long long)oslot * nc * nc;
  for (int e = threadIdx.x; e < nc * nc; e += blockDim.x) {
    int c = e / nc, r = e % nc;   // column major output
    out[e] = M[r * w2 + nc + c];
  }
}

template <int N>
struct RestrictDispatch {
  template <typename R, typename Sp, typename Tv, typename To>
  static void run(const GeomDev& g, const void* P, int nrhs, const void* fine, void* out, long long rstride,
                  long long sstride, hipStream_t st) {
    int threads = g.Bv < 64 ? 64 : g.Bv;
    // test vectors once, fine input per RHS, coarse output per RHS
    const double bytes = (double)g.V * 12 * (N * sizeof(Sp) + nrhs * sizeof(Tv)) + (double)g.Vc * 2 * N * nrhs * sizeof(To);
    const double flops = 8.0 * g.V * 12 * N * nrhs;
    if constexpr (std::is_same<R, double>::value && std::is_same<Tv, double2>::value && std::is_same<To, double2>::value) {
      if (g.Bv == 256) {   // FP64 matrix cores, 32 sites per staging step (two workgroups per CU)
        DD_TIMED("k_restrict", st, bytes, flops,
                 (k_restrict_mfma<N, Sp, double, 32><<<g.Vc, 256, 0, st>>>(g, (const Sp*)P, nrhs, (const double2*)fine,
                                                                           (double2*)out, rstride, sstride)));
        return;
      }
    }
    DD_TIMED("k_restrict", st, bytes, flops,
             (k_restrict<N, R, Sp, Tv, To><<<xcd_grid(g.Vc, nrhs), threads, 0, st>>>(g, (const Sp*)P, nrhs, (const Tv*)fine,
                                                                                      (To*)out, rstride, sstride)));
  }
};

template <typename R, typename Sp, typename Tv, typename To>
void restrict_n(const GeomDev& g, int n, const void* P, int nrhs, const void* fine, void* out, long long rstride,
                long long sstride, hipStream_t st) {
  switch (n) {
    case 6: RestrictDispatch<6>::run<R, Sp, Tv, To>(g, P, nrhs, fine, out, rstride, sstride, st); break;
    case 8: RestrictDispatch<8>::run<R, Sp, Tv, To>(g, P, nrhs, fine, out, rstride, sstride, st); break;
    case 12: RestrictDispatch<12>::run<R, Sp, Tv, To>(g, P, nrhs, fine, out, rstride, sstride, st); break;
    case 16: RestrictDispatch<16>::run<R, Sp, Tv, To>(g, P, nrhs, fine, out, rstride, sstride, st); break;
    case 20: RestrictDispatch<20>::run<R, Sp, Tv, To>(g, P, nrhs, fine, out, rstride, sstride, st); break;
    case 24: RestrictDispatch<24>::run<R, Sp, Tv, To>(g, P, nrhs, fine, out, rstride, sstride, st); break;
  }
}

}  // namespace

bool supported_nvec(int n) { return n == 6 || n == 8 || n == 12 || n == 16 || n == 20 || n == 24; }

void launch_restrict(const GeomDev& g, dd_dtype vt, dd_dtype pst, int n, const void* P, int nrhs, const void* fine,
                     void* coarse, hipStream_t st) {
  long long nc = 2 * n, rs = (long long)g.Vc * nc;
  if (vt == DD_F64) {
    restrict_n<double, double2, double2, double2>(g, n, P, nrhs, fine, coarse, rs, nc, st);
    return;
  }
  if (g.Bv == 256 && pst != DD_F64) {   // matrix-core form
    const double bytes = (double)g.V * 12 * (n * storage_pair_bytes(pst) + nrhs * sizeof(float2)) +
                         (double)g.Vc * 2 * n * nrhs * sizeof(float2);
    const double flops = 8.0 * g.V * 12 * n * nrhs;
#define DD_RM(NN, SP)                                                                                     \
  DD_TIMED("k_restrict", st, bytes, flops,                                                                \
           (k_restrict_mfma<NN, SP, float, 64><<<g.Vc, 256, 0, st>>>(g, (const SP*)P, nrhs,                \
                                                                     (const float2*)fine, (float2*)coarse, rs, nc)))
#define DD_RMN(SP)                  \
  switch (n) {                      \
    case 6: DD_RM(6, SP); break;    \
    case 8: DD_RM(8, SP); break;    \
    case 12: DD_RM(12, SP); break;  \
    case 16: DD_RM(16, SP); break;  \
    case 20: DD_RM(20, SP); break;  \
    default: DD_RM(24, SP); break;  \
  }
    switch (pst) {
      case DD_F32: DD_RMN(float2) break;
      case DD_F16: DD_RMN(__half2) break;
      default: DD_RMN(bf16x2) break;
    }
#undef DD_RMN
#undef DD_RM
    return;
  }
  switch (pst) {
    case DD_F64: restrict_n<float, double2, float2, float2>(g, n, P, nrhs, fine, coarse, rs, nc, st); break;
    case DD_F32: restrict_n<float, float2, float2, float2>(g, n, P, nrhs, fine, coarse, rs, nc, st); break;
    case DD_F16: restrict_n<float, __half2, float2, float2>(g, n, P, nrhs, fine, coarse, rs, nc, st); break;
    case DD_BF16: restrict_n<float, bf16x2, float2, float2>(g, n, P, nrhs, fine, coarse, rs, nc, st); break;
  }
}

static void prolong_dispatch(const GeomDev& g, dd_dtype vt, dd_dtype pst, int n, const void* P, int nrhs,
                             const void* coarse, void* fine, hipStream_t st) {
  if (vt != DD_F64 && g.Bv == 256 && pst != DD_F64) {   // matrix-core form
#define DD_PM(NN, SP)                                                                                        \
  k_prolong_mfma<NN, SP><<<g.Vc, 256, 0, st>>>(g, (const SP*)P, nrhs, (const float2*)coarse, (float2*)fine)
#define DD_PMN(SP)                  \
  switch (n) {                      \
    case 6: DD_PM(6, SP); break;    \
    case 8: DD_PM(8, SP); break;    \
    case 12: DD_PM(12, SP); break;  \
    case 16: DD_PM(16, SP); break;  \
    case 20: DD_PM(20, SP); break;  \
    default: DD_PM(24, SP); break;  \
  }
    switch (pst) {
      case DD_F32: DD_PMN(float2) break;
      case DD_F16: DD_PMN(__half2) break;
      default: DD_PMN(bf16x2) break;
    }
#undef DD_PMN
#undef DD_PM
    return;
  }
  int threads = g.Bv < 64 ? 64 : g.Bv;
  unsigned nb = xcd_grid(g.Vc, nrhs);
  if (vt == DD_F64) {
    k_prolong<double, double2, double2><<<nb, threads, 0, st>>>(g, n, (const double2*)P, nrhs, (const double2*)coarse,
                                                               (double2*)fine);
    return;
  }
  switch (pst) {
    case DD_F64:
      k_prolong<float, double2, float2><<<nb, threads, 0, st>>>(g, n, (const double2*)P, nrhs, (const float2*)coarse,
                                                               (float2*)fine);
      break;
    case DD_F32:
      k_prolong<float, float2, float2><<<nb, threads, 0, st>>>(g, n, (const float2*)P, nrhs, (const float2*)coarse,
                                                              (float2*)fine);
      break;
    case DD_F16:
      k_prolong<float, __half2, float2><<<nb, threads, 0, st>>>(g, n, (const __half2*)P, nrhs, (const float2*)coarse,
                                                               (float2*)fine);
      break;
    case DD_BF16:
      k_prolong<float, bf16x2, float2><<<nb, threads, 0, st>>>(g, n, (const bf16x2*)P, nrhs, (const float2*)coarse,
                                                              (float2*)fine);
      break;
  }
}

void launch_prolong(const GeomDev& g, dd_dtype vt, dd_dtype pst, int n, const void* P, int nrhs, const void* coarse,
                    void* fine, hipStream_t st) {
  const size_t sp = pst == DD_F64 ? 16 : (pst == DD_F32 ? 8 : 4), sv = vt == DD_F64 ? 16 : 8;
  const double bytes = (double)g.V * 12 * (n * sp + nrhs * sv) + (double)g.Vc * 2 * n * nrhs * sv;
  const double flops = 8.0 * g.V * 12 * n * nrhs;
  DD_TIMED("k_prolong", st, bytes, flops, prolong_dispatch(g, vt, pst, n, P, nrhs, coarse, fine, st));
}

void launch_gram_schmidt(const GeomDev& g, int n, double2* P, int* bad_flag, hipStream_t st) {
  int threads = g.Bv < 64 ? 64 : g.Bv;
  k_gram_schmidt<<<(unsigned)g.Vc * 2, threads, 0, st>>>(g, n, P, bad_flag);
}

// D_c = P^dag D P in FP64 from the stored test vectors (pst) and the FP64 operator.
// W is scratch for `chunk` fine FP64 vectors.
void launch_coarse_build(const GeomDev& g, const OpSet& ops64, dd_dtype pst, int n, const void* P, double2* Dc64,
                         double2* W, int chunk, hipStream_t st) {
  const int nc = 2 * n;
  const double2* L = (const double2*)ops64.links;
  const double2* C = (const double2*)ops64.clover;
  for (int d = 0; d < 9; ++d)
    for (int c0 = 0; c0 < nc; c0 += chunk) {
      int ncol = nc - c0 < chunk ? nc - c0 : chunk;
      unsigned nb = xcd_grid((g.V + 255) / 256, ncol);
      switch (pst) {
        case DD_F64:
          k_coarse_piece<double, double2, double2><<<nb, 256, 0, st>>>(g, L, C, (const double2*)P, n, c0, ncol, d, W);
          break;
        case DD_F32:
          k_coarse_piece<double, double2, float2><<<nb, 256, 0, st>>>(g, L, C, (const float2*)P, n, c0, ncol, d, W);
          break;
        case DD_F16:
          k_coarse_piece<double, double2, __half2><<<nb, 256, 0, st>>>(g, L, C, (const __half2*)P, n, c0, ncol, d, W);
          break;
        case DD_BF16:
          k_coarse_piece<double, double2, bf16x2><<<nb, 256, 0, st>>>(g, L, C, (const bf16x2*)P, n, c0, ncol, d, W);
          break;
      }
      // rows of D_c(X, d)[:, col] = restriction of the piece: out[col][X][row] with strides
      double2* out = Dc64 + (long long)d * nc * nc + (long long)c0 * nc;
      long long rstride = nc, sstride = 9LL * nc * nc;
      switch (pst) {
        case DD_F64: restrict_n<double, double2, double2, double2>(g, n, P, ncol, W, out, rstride, sstride, st); break;
        case DD_F32: restrict_n<double, float2, double2, double2>(g, n, P, ncol, W, out, rstride, sstride, st); break;
        case DD_F16: restrict_n<double, __half2, double2, double2>(g, n, P, ncol, W, out, rstride, sstride, st); break;
        case DD_BF16: restrict_n<double, bf16x2, double2, double2>(g, n, P, ncol, W, out, rstride, sstride, st); break;
      }
    }
}

void launch_coarse_invert(const GeomDev& g, int nc, const double2* Dc64, double2* Dinv64, int* bad_flag, hipStream_t st) {
  size_t shm = sizeof(double2) * nc * 2 * nc;
  k_coarse_invert<<<(unsigned)g.Vch, 256, shm, st>>>(g, nc, Dc64, Dinv64, bad_flag);
}
