// Internal declarations shared by the libdd translation units: handle
// structs, the packed-layout geometry, device complex arithmetic, storage
// types and the host-side kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/dd.h"

// ---------------------------------------------------------------------------
// Packed geometry
//
// Sites are stored block-major: packed index I = slot * Bv + p * Bvh + j, where
//   slot : block ("domain") slot; red blocks (sum of block coordinates even)
//          take slots [0, Vc/2), black blocks [Vc/2, Vc); inside a colour the
//          slot is (lexicographic block index) / 2,
//   p    : site parity (block origins are even, so local parity = global parity),
//   j    : (lexicographic position inside the block) / 2.
// A domain is a contiguous range of Bv sites with its even sites first, and the
// coarse lattice uses the same slots (even coarse sites = red blocks first).
// Block edges are powers of two, so local coordinates come from shifts.
// ---------------------------------------------------------------------------
struct GeomDev {
  int L[4];
  int b[4];
  int lb[4];      // log2 of the block edges
  int lBv;        // log2(Bv)
  int Bv, Bvh;    // sites per block, half of it
  int Vc, Vch;    // blocks (coarse sites), half of it
  long long V;
  const int* blk_nbr;    // [8][Vc]: slot of the neighbouring block; bit 30 set when the hop wraps in t
  const int* blk_coord;  // [Vc]: block coordinates packed as bx | by<<8 | bz<<16 | bt<<24
  const int* lex_slot;   // [Vc]: slot of the block with lexicographic block index l (x fastest)
  double bc_t;
};

#define DD_WRAP_BIT (1 << 30)
#define DD_SLOT_MASK ((1 << 30) - 1)

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cx<R> cmul_conj(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc += a * b
template <typename R>
__host__ __device__ __forceinline__ void cfma(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}
// acc += conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ void cfma_conj(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.re * b.im - a.im * b.re;
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }

// ---------------------------------------------------------------------------
// storage types: a complex number stored as a pair
// ---------------------------------------------------------------------------
struct bf16x2 {
  uint32_t u;  // low 16 bits: real part, high 16 bits: imaginary part
};

template <typename S>
struct StoreTraits;
template <>
struct StoreTraits<double2> {
  typedef double R;
};
template <>
struct StoreTraits<float2> {
  typedef float R;
};
template <>
struct StoreTraits<__half2> {
  typedef float R;
};
template <>
struct StoreTraits<bf16x2> {
  typedef float R;
};

template <typename R, typename S>
__device__ __forceinline__ cx<R> ld(const S* p);
template <>
__device__ __forceinline__ cx<double> ld<double, double2>(const double2* p) {
  double2 v = *p;
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ cx<float> ld<float, float2>(const float2* p) {
  float2 v = *p;
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ cx<float> ld<float, __half2>(const __half2* p) {
  float2 v = __half22float2(*p);
  return {v.x, v.y};
}
template <>
__device__ __forceinline__ cx<float> ld<float, bf16x2>(const bf16x2* p) {
  uint32_t u = p->u;
  return {__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u)};
}
template <>
__device__ __forceinline__ cx<float> ld<float, double2>(const double2* p) {
  double2 v = *p;
  return {(float)v.x, (float)v.y};
}
template <>
__device__ __forceinline__ cx<double> ld<double, float2>(const float2* p) {
  float2 v = *p;
  return {(double)v.x, (double)v.y};
}
template <>
__device__ __forceinline__ cx<double> ld<double, __half2>(const __half2* p) {
  float2 v = __half22float2(*p);
  return {(double)v.x, (double)v.y};
}
template <>
__device__ __forceinline__ cx<double> ld<double, bf16x2>(const bf16x2* p) {
  uint32_t u = p->u;
  return {(double)__uint_as_float(u << 16), (double)__uint_as_float(u & 0xffff0000u)};
}

template <typename S, typename R>
__device__ __forceinline__ void st(S* p, cx<R> v);
template <>
__device__ __forceinline__ void st<double2, double>(double2* p, cx<double> v) { *p = make_double2(v.re, v.im); }
template <>
__device__ __forceinline__ void st<float2, float>(float2* p, cx<float> v) { *p = make_float2(v.re, v.im); }
template <>
__device__ __forceinline__ void st<float2, double>(float2* p, cx<double> v) {
  *p = make_float2((float)v.re, (float)v.im);
}
template <>
__device__ __forceinline__ void st<__half2, double>(__half2* p, cx<double> v) {
  *p = __floats2half2_rn((float)v.re, (float)v.im);
}
template <>
__device__ __forceinline__ void st<double2, float>(double2* p, cx<float> v) {
  *p = make_double2((double)v.re, (double)v.im);
}

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// ---------------------------------------------------------------------------
// packed-geometry helpers (device)
// ---------------------------------------------------------------------------
struct SiteLoc {
  int slot;
  int l[4];
};

__host__ __device__ __forceinline__ SiteLoc decode_site(const GeomDev& g, long long I) {
  SiteLoc s;
  s.slot = (int)(I >> g.lBv);
  int loc = (int)(I & (g.Bv - 1));
  int p = loc >> (g.lBv - 1);
  int lex2 = (loc & (g.Bvh - 1)) << 1;
  int lx0 = lex2 & (g.b[0] - 1);
  s.l[1] = (lex2 >> g.lb[0]) & (g.b[1] - 1);
  s.l[2] = (lex2 >> (g.lb[0] + g.lb[1])) & (g.b[2] - 1);
  s.l[3] = lex2 >> (g.lb[0] + g.lb[1] + g.lb[2]);
  s.l[0] = lx0 + ((p + s.l[1] + s.l[2] + s.l[3]) & 1);
  return s;
}

__host__ __device__ __forceinline__ int encode_local(const GeomDev& g, const int l[4]) {
  int lex = l[0] + ((l[1] + ((l[2] + (l[3] << g.lb[2])) << g.lb[1])) << g.lb[0]);
  int p = (l[0] + l[1] + l[2] + l[3]) & 1;
  return p * g.Bvh + (lex >> 1);
}

// Neighbour of a site in direction mu (sign +1/-1).  Returns the packed index
// and sets `wrap` when the hop crosses the t boundary, `inside` when the
// neighbour lies in the same block.
__host__ __device__ __forceinline__ long long neighbor(const GeomDev& g, const SiteLoc& s, int mu, int sign,
                                              bool& wrap, bool& inside) {
  int l[4] = {s.l[0], s.l[1], s.l[2], s.l[3]};
  int v = l[mu] + sign;
  int slot = s.slot;
  wrap = false;
  inside = (v >= 0 && v < g.b[mu]);
  if (!inside) {
    int e = g.blk_nbr[(sign > 0 ? mu : 4 + mu) * g.Vc + slot];
    wrap = (e & DD_WRAP_BIT) != 0;
    slot = e & DD_SLOT_MASK;
    v = (sign > 0) ? 0 : g.b[mu] - 1;
  }
  l[mu] = v;
  return ((long long)slot << g.lBv) + encode_local(g, l);
}

// XCD-aware work mapping.  Consecutive workgroups are dealt round-robin to the
// eight XCDs, each with its own L2.  Workgroups that handle the same tile for
// different right-hand sides share the tile's operator, so they are given the
// same XCD: workgroup b runs on XCD b % 8 and takes tile (b % 8) + 8 * (k / nrhs),
// rhs k % nrhs, with k = b / 8.  Launch xcd_grid(ntiles, nrhs) workgroups and
// skip tiles >= ntiles.
__device__ __forceinline__ void xcd_tile_rhs(int nrhs, int& tile, int& rhs) {
  const int b = blockIdx.x, x = b & 7, k = b >> 3;
  tile = x + 8 * (k / nrhs);
  rhs = k % nrhs;
}
inline unsigned xcd_grid(long long ntiles, int nrhs) { return (unsigned)(8 * ((ntiles + 7) / 8) * nrhs); }

// Contiguous ranges per XCD: the k-th workgroup of XCD x = b % 8 takes right-hand
// side k % nrhs of tile x * (ntiles / 8) + k / nrhs (ntiles a multiple of 8), so
// each XCD works through one contiguous eighth of the tiles.  Launch
// xcd_grid(ntiles, nrhs) workgroups.
__device__ __forceinline__ void xcd_range_tile(int ntiles, int nrhs, int& tile, int& rhs) {
  const int b = blockIdx.x, x = b & 7, k = b >> 3;
  rhs = k % nrhs;
  tile = x * (ntiles / 8) + k / nrhs;
}

// Slab order for kernels whose halo comes from neighbouring blocks.  The tiles
// (per_blk of them per block) are taken in lexicographic block order, both
// colours interleaved, and each XCD gets a contiguous eighth of that order (a
// slab of the lattice): the k-th workgroup of XCD x = b % 8 takes right-hand
// side k % nrhs of tile x * (ntiles / 8) + k / nrhs of the order.  Neighbouring
// blocks are then processed together on one L2.  Launch xcd_grid(Vc * per_blk,
// nrhs) workgroups; Vc is a multiple of 16.  Returns false for workgroups past
// the end.
__device__ __forceinline__ bool xcd_slab_tile(const GeomDev& g, int per_blk, int nrhs, int& tile, int& rhs) {
  const int b = blockIdx.x, x = b & 7, k = b >> 3;
  const int per_x = g.Vc * per_blk / 8;
  const int kk = k / nrhs;
  rhs = k % nrhs;
  if (kk >= per_x) return false;
  const int tl = x * per_x + kk;
  tile = g.lex_slot[tl / per_blk] * per_blk + tl % per_blk;
  return true;
}

// Device-side gate of a launch: the kernel returns at once unless some entry
// of `flags` (one per right-hand side) equals `open_on`.  With the Arnoldi
// activity flags (open_on 1) the steps of a coarse GMRES cycle become no-ops
// once every right-hand side has converged; with the finished flags
// (open_on 0) so do the cycle-level kernels once every right-hand side is done.
// A null gate is always open.  The host sets the gate launches take through
// GateScope (per host thread), so the launchers keep their signatures.
struct Gate {
  const int* flags = nullptr;
  int n = 0;
  int open_on = 1;
};
__device__ __forceinline__ bool gate_closed(const Gate& g) {
  if (!g.flags) return false;
  for (int r = 0; r < g.n; ++r)
    if (g.flags[r] == g.open_on) return false;
  return true;
}
Gate& current_gate();
struct GateScope {
  Gate saved;
  explicit GateScope(const Gate& g) : saved(current_gate()) { current_gate() = g; }
  ~GateScope() { current_gate() = saved; }
};

// lexicographic site index of a packed site
__host__ __device__ __forceinline__ long long lex_site(const GeomDev& g, const SiteLoc& s) {
  int bc = g.blk_coord[s.slot];
  int x = (bc & 255) * g.b[0] + s.l[0];
  int y = ((bc >> 8) & 255) * g.b[1] + s.l[1];
  int z = ((bc >> 16) & 255) * g.b[2] + s.l[2];
  int t = ((bc >> 24) & 255) * g.b[3] + s.l[3];
  return x + (long long)g.L[0] * (y + (long long)g.L[1] * (z + (long long)g.L[2] * t));
}

// ---------------------------------------------------------------------------
// host-side objects
// ---------------------------------------------------------------------------
struct dd_ctx {
  int device;
  size_t budget;
  size_t in_use;             // guarded by mu: threads that drive different solvers share one context
  std::mutex mu;
  void* scratch = nullptr;   // device address of this device's static scratch array (allocation-free calls)
};

// Size of the static per-device scratch array that the allocation-free entry
// point carves its workspace from (api_core.hip).
constexpr size_t kStaticScratchBytes = 128ULL << 20;

// Operand copies of one storage type (links, clover, clover inverse).
struct OpSet {
  bool ready = false;
  void* links = nullptr;    // [4][9][V]   complex pairs of the storage type
  void* clover = nullptr;   // [36][V]     packed Hermitian blocks, pairs of the storage type
  void* cinv = nullptr;     // [36][V]     same layout, inverse
};

// Launch shapes picked per gauge field (problem shape) by the autotuner; every
// choice gives bit-identical results.
struct Tuning {
  int sap_wpe = 2;          // SAP layout: 2 (registers, 2 waves per SIMD) or 3 (lean LDS, 3)
  int sap_persist = 0;      // domain-resident SAP: all sweeps in one cooperative launch (same bits)
  int sap_dom_rhs = 2;      // 4^4 domains, FP16/BF16 operands: RHS per workgroup of the domain-resident
                            // SAP (operator staged in LDS once per domain), 2 or 4; 0 = one workgroup per
                            // (domain, RHS)
  int dirac_threads = 256;  // D apply workgroup size: 64, 128 or 256
  int coarse_spw = 4;       // FP32 coarse apply: coarse sites (waves) per workgroup, 2, 4 or 8
  int coarse_half = 0;        // with half-precision storage: 1 = coarse blocks in that type, 0 = FP32 blocks
  int coarse_basis_half = 0;  // FP32 coarse GMRES: Krylov basis stored in FP16 (1) or FP32 (0)
  int coarse_mfma_half = 0;   // half-precision blocks: FP16 / BF16 MFMA with x rounded to that type
};

struct dd_gauge {
  dd_ctx* ctx;
  Tuning tune;
  dd_problem prob;
  GeomDev geo;
  int* d_blk_nbr = nullptr;
  int* d_blk_coord = nullptr;
  int* d_lex_slot = nullptr;
  std::vector<int> h_blk_nbr, h_blk_coord;
  OpSet ops[4];   // indexed by dd_dtype: F64 master, F32, F16, BF16
  int refcount = 0;
};

struct Workspace;
struct Level3;

struct dd_mg {
  dd_ctx* ctx;
  dd_gauge* g;
  dd_mg_params p;
  int n;          // test vectors
  int nc;         // 2n
  dd_dtype vstore;  // storage of P inside M
  // test vectors: FP64 master of the orthonormalised P (packed fine layout, n vectors)
  double2* P64 = nullptr;
  void* Pst = nullptr;       // P in the storage dtype (float2 / __half2 / bf16x2)
  void* tv = nullptr;        // working test vectors lambda_i (inner dtype)
  // coarse operator: [Vc][9][col][row] complex (column-major blocks), FP64 master and FP32
  double2* Dc64 = nullptr;
  float2* Dc32 = nullptr;
  void* Dch = nullptr;       // half-precision copy (storage dtype F16/BF16) used by the FP32 inner solve
  // odd-site inverses of the self blocks: [Vch][col][row]
  double2* Dinv64 = nullptr;
  float2* Dinv32 = nullptr;
  void* Dinvh = nullptr;
  Workspace* ws = nullptr;
  int graphs = 0;   // 0: launches; 1: coarse GMRES chunks replayed from graphs; 2: all of M from one graph
  dd_solve_state* live = nullptr;   // the stepwise solve that holds the workspace, if any
  Level3* l3 = nullptr;             // third level: coarse solves by a two-level cycle on D_c, when added
};

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
dd_status dd_fail(dd_ctx* ctx, dd_status s, const std::string& msg);
size_t ctx_in_use(dd_ctx* ctx);   // bytes reserved against the budget (locked read)
dd_status dd_hip_check(dd_ctx* ctx, hipError_t e, const char* what);
#define DD_HIP(ctx, call)                                            \
  do {                                                               \
    hipError_t _e = (call);                                          \
    if (_e != hipSuccess) return dd_hip_check((ctx), _e, #call);    \
  } while (0)

dd_status dd_alloc(dd_ctx* ctx, void** p, size_t bytes);
void dd_free(dd_ctx* ctx, void* p, size_t bytes);

inline size_t storage_pair_bytes(dd_dtype dt) {
  switch (dt) {
    case DD_F64: return 16;
    case DD_F32: return 8;
    default: return 4;
  }
}
inline size_t vector_pair_bytes(dd_dtype dt) { return dt == DD_F64 ? 16 : 8; }

// ---------------------------------------------------------------------------
// kernel launchers (each defined next to its kernels)
// ---------------------------------------------------------------------------
// geometry / packing / conversion / random vectors
void launch_pack_fine(const GeomDev& g, dd_dtype vt, int nrhs, const double2* canon, void* packed,
                      hipStream_t st);
void launch_unpack_fine(const GeomDev& g, dd_dtype vt, int nrhs, const void* packed, double2* canon,
                        hipStream_t st);
void launch_pack_links(const GeomDev& g, const double2* canon, double2* links64, hipStream_t st);
// FP64 source for DD_F64 / DD_F32 targets, FP32 source for DD_F16 / DD_BF16 targets
void launch_convert_pairs(dd_dtype to, const double2* src64, const float2* src32, void* dst, long long count,
                          hipStream_t st);
void launch_vec_convert(dd_dtype from, dd_dtype to, const void* src, void* dst, long long count,
                        hipStream_t st);
void launch_gauss(unsigned long long seed, long long n, double2* out, hipStream_t st);
// clover
void launch_clover_build(const GeomDev& g, const double2* links64, double m0, double csw,
                         double2* clover64, double2* cinv64, hipStream_t st);
// Dirac operator
void launch_dirac(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, const void* in, void* out,
                  hipStream_t st, int threads = 256);
// FP64 operator applied to an FP32 vector (FP64 result)
void launch_dirac_f32_in(const GeomDev& g, const OpSet& ops64, int nrhs, const float2* in, double2* out,
                         hipStream_t st, int threads = 256);
// SAP smoother
void launch_sap(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, int sweeps, int mr_iters,
                const void* b, void* x, int wpe, int dom_rhs, int persist, hipStream_t st);
bool sap_dom_supported(const GeomDev& g, dd_dtype dt);
void launch_sap_dom(const GeomDev& g, dd_dtype dt, const OpSet& ops, int nrhs, int sweeps, int mr_iters,
                    const void* b, void* x, int rhs_group, bool persist, hipStream_t st);
// transfer and coarse construction
bool supported_nvec(int n);
void launch_restrict(const GeomDev& g, dd_dtype vt, dd_dtype pst, int n, const void* P, int nrhs,
                     const void* fine, void* coarse, hipStream_t st);
void launch_prolong(const GeomDev& g, dd_dtype vt, dd_dtype pst, int n, const void* P, int nrhs,
                    const void* coarse, void* fine, hipStream_t st);
void launch_gram_schmidt(const GeomDev& g, int n, double2* P, int* bad_flag, hipStream_t st);
void launch_coarse_build(const GeomDev& g, const OpSet& ops64, dd_dtype pst, int n, const void* P,
                         double2* Dc64, double2* W, int chunk, hipStream_t st);
void launch_coarse_invert(const GeomDev& g, int nc, const double2* Dc64, double2* Dinv64, int* bad_flag,
                          hipStream_t st);
// coarse operator: out = a_self M xs + a_hop sum_d D_c(d) xh(X+d) + beta z on sites [begin, begin+count)
void launch_coarse_mv(const GeomDev& g, dd_dtype vt, int nc, const void* Dc, const void* Minv, int use_inv,
                      int nrhs, int site_begin, int count, double a_self, const void* xs, double a_hop,
                      const void* xh, double beta, const void* z, void* out, hipStream_t st, int spw = 4,
                      dd_dtype bt = DD_F32, bool hmfma = false);   // hmfma: half blocks on half-precision MFMA
// vector kernels
int dots_blocks(long long count, int nrhs);
void launch_dots(dd_dtype vt, dd_dtype wt, int nrhs, long long count, long long ld, const void* V, int nv,
                 long long vstride, const void* w, double* partial, int nblk, double2* out, int ldo, int off,
                 hipStream_t st);
void launch_multi_axpy(dd_dtype vt, dd_dtype wt, int nrhs, long long count, long long ld, const void* V, int nv,
                       long long vstride, const double2* coef, int ldc, int coff, double sign, void* w,
                       hipStream_t st);
// w -= sum_i coef_i V_i, then out = <V_i, w> (fused, nv <= 16)
void launch_axpy_dots(dd_dtype vt, int nrhs, long long count, long long ld, const void* V, int nv, long long vstride,
                      const double2* coef, int ldc, void* w, double* partial, int nblk, double2* out, int ldo,
                      hipStream_t st,
                      dd_dtype bt = DD_F32);
// w -= sum_i coef_i V_i, then out[r].x = |w|^2 (fused, nv <= 16)
void launch_axpy_norm(dd_dtype vt, int nrhs, long long count, long long ld, const void* V, int nv, long long vstride,
                      const double2* coef, int ldc, void* w, double* partial, int nblk, double2* out, hipStream_t st,
                      dd_dtype bt = DD_F32);
// whole-basis classical Gram-Schmidt (nv <= gs_max_nv()), partial sums over gs_blocks(count) tiles:
// out[r * ldo + i] = <V_i, w> for i < nv
int gs_max_nv();
int gs_blocks(long long count);
void launch_gs_dots(dd_dtype bt, dd_dtype vt, int nrhs, long long count, long long ld, const void* V, int nv,
                    long long vstride, const void* w, double* partial, double2* out, int ldo, hipStream_t st);
// w -= sum_{i < nv} coef_i V_i, then out[r].x = |w|^2
void launch_gs_axpy_norm(dd_dtype bt, dd_dtype vt, int nrhs, long long count, long long ld, const void* V, int nv,
                         long long vstride, const double2* coef, int ldc, void* w, double* partial, double2* out,
                         hipStream_t st);
void launch_normalize(dd_dtype vt, int nrhs, long long count, long long ld, const void* src, const double2* nrm2,
                      const double* nrm, const int* mask, void* dst, hipStream_t st,
                      dd_dtype dt = DD_F32, void* copy32 = nullptr);   // dt: dtype of dst (F16 basis)
void launch_sub(dd_dtype vt, long long n, const void* a, const void* b, void* out, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);   // bytes: multiple of 4
// device-side controls of the coarse GMRES (no host round trip)
void launch_set_tol(int nrhs, double tol, const double2* nrm2, double* tolabs, int* finished, int* active,
                    hipStream_t st);
void launch_finish(int nrhs, const double* est, const double* tolabs, int* finished, int* active, const int* kcyc,
                   int* iters, hipStream_t st);
void launch_copy(dd_dtype vt, long long n, const void* a, void* out, hipStream_t st);
// FP32 (and, when half is DD_F16 / DD_BF16, half) copies of nblk FP64 coarse
// blocks in the order the matrix-core apply reads
void launch_coarse_tile(int nc, const double2* src64, long long nblk, float2* dst32, dd_dtype half, void* dsth,
                        hipStream_t st);
void launch_add(dd_dtype vt, long long n, const void* a, void* out, hipStream_t st);
void launch_cycle_init(int nrhs, int m, const double2* nrm2, const double* tolabs, const int* finished,
                       double2* gv, double* beta, int* active, int* kcyc, hipStream_t st);
// h2: second Gram-Schmidt pass, or null after a single pass
void launch_arnoldi(int nrhs, int m, int j, const double2* h1, const double2* h2, const double2* nrm2,
                    double2* H, double* cs, double2* sn, double2* gv, const double* tolabs, int* active,
                    int* kcyc, double* est, double* hnext, hipStream_t st);
void launch_lsq(int nrhs, int m, const double2* H, const double2* gv, const int* kcyc, double2* y,
                hipStream_t st);

// third level (blocks of 2^4 coarse sites, chirality-split aggregates)
void launch_gs2(int Vc, int Vc3, int n, int n2, const int* slot_of, const double2* tv, double2* P2, int* bad,
                hipStream_t st);
void launch_restrict2(dd_dtype vt, int Vc, int Vc3, int n, int n2, const int* slot_of, const void* P2, int nrhs,
                      const void* v, void* out, hipStream_t st);
void launch_prolong2(dd_dtype vt, int Vc, int Vc3, int n, int n2, const int* l3_of, const int* loc_of,
                     const void* P2, int nrhs, const void* y, void* out, hipStream_t st);
void launch_galerkin3(const GeomDev& g2, int Vc3, int n, int n2, const int* slot_of, const int* l3_of,
                      const int* loc_of, const double2* Dc64, const double2* P2, double2* D3, hipStream_t st);
void launch_mr_alpha(int nrhs, const double2* num, const double2* den, double2* alpha, hipStream_t st);

dd_status ensure_opset(dd_gauge* g, dd_dtype dt);
dd_status gauge_set_mass(dd_gauge* g, double m0);
