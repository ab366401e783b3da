// Device side of the implicit filter on gfx950: matrix upload, the
// Jacobi-preconditioned CG kernels and the per-column solve driver.
//
// The solve of Sect. 2.2.2 is CG on S x = M phi from x0 = phi (the residual
// form: r0 = M phi - S phi = -c K_n phi), with S = diag(M) + c K_n and the
// Jacobi preconditioner diag(S)^-1. Everything is bandwidth bound, so the
// kernels are organised around HBM traffic:
//
//  * K_n's off-diagonal entries are streamed in sliced-ELL form (slices of
//    64 rows = one wavefront, column-major inside a slice) so that column
//    indices and values are read with fully coalesced 256 / 512 B wavefront
//    loads; the diagonal of S = M + c diag(K_n) is formed once per solve and
//    doubles as the Jacobi preconditioner.
//  * One CG iteration is one kernel (k_cg): the residual update of the
//    previous iteration is applied on the fly to the gathered operand
//    (z' = z - alpha u, with u = diag(S)^-1 S p kept in place of S p), then
//    x += alpha p, p' = z' + beta p and u' = diag(S)^-1 S p', with the block
//    partials of the next iteration's sums: one grid-level reduction per
//    iteration.
//  * Reductions are deterministic two-level sums: every block writes one
//    partial per quantity; the next kernel's blocks each finish the sums in
//    the same fixed order (all quantities in one pass), so all blocks agree
//    bitwise on alpha / beta and on the stopping test without atomics or
//    cross-XCD fences.
//  * Logical blocks own contiguous row ranges and are mapped so that the
//    blocks of one XCD (hardware dispatches workgroups round-robin over the
//    8 XCDs) hold neighbouring ranges: neighbouring rows' gathers then hit
//    the same XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <limits>
#include <string>
#include <vector>

#include "batch.h"
#include "internal.h"

namespace ifl {

#define IFL_HIP(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(IFL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

constexpr int kWave = 64;
constexpr int kBlock = 512;                 // 8 wavefronts
constexpr int kWavesPerBlock = kBlock / kWave;
// logical blocks (partials per quantity). Every block reduces the previous
// kernel's partials in its prologue, so more blocks cost more there: on a
// 2.6 M-row mesh 512 beat 256, 1024 and 2048 (FP32 SpMV 38 vs 46-50 us).
constexpr int kMaxBlocks = 512;
constexpr int kXcd = 8;
constexpr int kMaxDevices = 64;
constexpr int kUnroll = 8;                  // sliced-ELL entries loaded together per row

// Per-column device state of the one-column path, in two copies: launch L
// reads copy L & 1 and its block 0 writes copy (L + 1) & 1 (so no block of
// a launch reads what that launch writes).
struct Scalars {
  double tol2;      // rtol^2 ||M phi||^2
  double rr_ref;    // ||r||^2 of the last FP64 true residual (mixed: replacement trigger)
  double c;         // gamma / k^(2n)
  double rr_last;   // ||r||^2 seen by the last stopping test
  double res2;      // final true ||b - S x||^2 (FP64)
  double bb;        // ||b||^2
  double energy2;   // sum M x^2
  double rho;       // (r, z) of the z a replacement superseded (beta after the replacement)
  int32_t iters;    // CG iterations performed
  int32_t done;     // 0 running, 1 converged, 2 breakdown, 3 max_iter
  int32_t updates;  // FP64 residual replacements
  int32_t mode;     // what the launch that wrote this copy did (M_INIT, M_ITER, M_REPLACE, M_DONE)
  uint32_t fused_bits;  // bit L % 32: launch L iterated with alpha != 0 (profiling)
  int32_t xbuf;     // after a stop: the x buffer that holds the solution
  int32_t pad1[2];
};

// The fields of Scalars that a k_cg launch changes; the others pass through
// from the copy it read. Keeping only these live (and re-reading the rest
// when the copy is written) keeps the whole struct out of scratch memory.
struct ScalarsMut {
  double rr_ref, rr_last, rho;
  int32_t iters, done, updates, mode, xbuf;
  uint32_t fused_bits;
};

__device__ __forceinline__ ScalarsMut mut_of(const Scalars& s) {
  return ScalarsMut{s.rr_ref, s.rr_last, s.rho, s.iters, s.done, s.updates, s.mode, s.xbuf, s.fused_bits};
}

// *dst = *src with the changed fields of m (one thread).
__device__ __forceinline__ void put_scalars(Scalars* dst, const Scalars* src, const ScalarsMut& m) {
  Scalars t = *src;
  t.rr_ref = m.rr_ref;
  t.rr_last = m.rr_last;
  t.rho = m.rho;
  t.iters = m.iters;
  t.done = m.done;
  t.updates = m.updates;
  t.mode = m.mode;
  t.xbuf = m.xbuf;
  t.fused_bits = m.fused_bits;
  *dst = t;
}

struct DevMatrix {
  int64_t n = 0, n_slices = 0, n_pad = 0;
  int64_t nnz_stored = 0;   // padded sliced-ELL entries
  int64_t offdiag = 0;      // true off-diagonal entries
  int64_t* sptr = nullptr;
  int32_t* col = nullptr;
  double* val64 = nullptr;
  float* val32 = nullptr;
  double* kdiag64 = nullptr;
  float* kdiag32 = nullptr;
  double* mass64 = nullptr;
  int64_t* entity = nullptr;
  int32_t* row_of = nullptr;  // caller index -> row, -1 for entries without a dof (field_len)
  int64_t field_len = 0;
  double mass_sum = 0.0;
  int head = 6;  // entries per row the gathering kernels load together (6, 12 or 20)
  // two-component operators: the 2 x 2-block sliced ELL of the batched
  // gathering kernels (PairPack); psptr == nullptr otherwise
  int64_t nb = 0, nb_slices = 0, pnnz = 0;
  int64_t* psptr = nullptr;
  int32_t* pcol = nullptr;
  double* pval64 = nullptr;
  float* pval32 = nullptr;
  int phead = 6;  // blocks per block row in the pipelined head
};

struct ColWork {
  double* x[2] = {nullptr, nullptr};  // FP64 solution (both precisions)
  // FP64 path vectors
  double *z[2] = {nullptr, nullptr}, *u[2] = {nullptr, nullptr}, *p[2] = {nullptr, nullptr}, *d = nullptr;
  // mixed path vectors
  float *z32[2] = {nullptr, nullptr}, *u32[2] = {nullptr, nullptr}, *p32[2] = {nullptr, nullptr}, *d32 = nullptr;
  double* phi = nullptr;   // field in internal order
  double* part = nullptr;  // partials, see offsets below
  Scalars* sc = nullptr;       // two copies (see Scalars)
  Scalars* sc_host = nullptr;  // pinned, 2 slots
  int* flag = nullptr;         // device: non-finite input detected
  double* stage_in = nullptr;  // field staging (caller numbering)
  double* stage_out = nullptr;
  int64_t stage_len = 0;
};

// ---- first-order shifted solves (IFL_SOLVER_SHIFTED) ----
// Complex vectors are interleaved (re, im) pairs of n_pad entries.
// Partial sums of a complex launch (units of G): two parities of nine sums
// (the complex (p, q), (q, z), (q, d^-1 q), (r, z) and the real ||r||^2),
// then the floor norm, ||M phi||^2 and the two finish sums.
constexpr int kCPqR = 0, kCPqI = 1, kCZuR = 2, kCZuI = 3, kCUuR = 4, kCUuI = 5, kCRzR = 6, kCRzI = 7, kCRr = 8,
              kCPerParity = 9;
__host__ __device__ constexpr int cidx(int parity, int q) { return parity * kCPerParity + q; }
enum { CP_FL = 2 * kCPerParity, CP_BB, CP_RES, CP_EN, CP_COUNT };

// State of one complex-shifted solve, two copies as for Scalars.
struct CScalars {
  double tol2, rr_ref, rr_last, bb;
  double sr, si;          // the shift sigma = sr + i si of M + sigma K
  double rho_r, rho_i;    // (r, z) of the z a replacement superseded
  int32_t iters, done, updates, mode;
  uint32_t fused_bits;
  int32_t xbuf;
  int32_t pad[2];
};

// The first-order operator K of a handle of order >= 2 (sliced ELL, the
// rows of K_n).
struct DevK1 {
  int64_t nnz_stored = 0;
  int64_t* sptr = nullptr;
  int32_t* col = nullptr;
  double* val64 = nullptr;
  float* val32 = nullptr;
  double* kdiag64 = nullptr;
  float* kdiag32 = nullptr;
  int head = 6;
};

// Work space of the shifted solves (made on first use).
struct ShiftWork {
  double* x[2] = {nullptr, nullptr};  // complex FP64 solution
  double *z64[2] = {nullptr, nullptr}, *u64[2] = {nullptr, nullptr}, *p64[2] = {nullptr, nullptr}, *d64 = nullptr;
  float *z32[2] = {nullptr, nullptr}, *u32[2] = {nullptr, nullptr}, *p32[2] = {nullptr, nullptr}, *d32 = nullptr;
  double* acc = nullptr;   // the weighted sum of the shifted solutions (real), n_pad
  double* part = nullptr;  // CP_COUNT x G
  CScalars* sc = nullptr;  // two copies
  CScalars* sc_host = nullptr;  // pinned, two slots
};

struct DeviceState {
  int device = 0;
  int order = 1;  // the handle's order n
  hipStream_t own_stream = nullptr;
  DevMatrix m;
  ColWork w;
  int G = 1;          // logical blocks
  int spb = 1;        // slices per logical block
  // completion events of the one-column path's chunks (made with the handle)
  hipEvent_t done_ev[2] = {nullptr, nullptr};
  // profiling
  std::vector<hipEvent_t> ev;
  int64_t prof_launches = 0;
  double prof_ms = 0.0;
  double prof_bytes = 0.0;  // summed algorithmic bytes of the timed launches
  std::string prof_kernel;  // the kernel those launches ran
  // batched engine work space (allocated on first use), and narrower tiles
  // that the last columns of a call move to
  DevK1 k1;
  ShiftWork sw;
  BatchWork bw;
  std::deque<BatchWork> spare;  // a deque: adding a tile leaves the others where they are
  BatchWork bwc;                 // complex tile of the shifted solves (order 2)
  double k1_gnorm = 0.0;         // g >= ||K M^-1||_2 of the first-order operator (order >= 2)
  double* zero_rows = nullptr;   // n_pad zeros: the imaginary part of a field
  // grid sizes picked by the autotuner, per (tile size, precision), and the
  // tile size it found best per precision (0 = not tuned)
  struct TunedGrid {
    int R;
    bool mixed;
    int G, Gu;
  };
  std::vector<TunedGrid> tuned;
  int tuned_R[2] = {0, 0};
  double* field_stage = nullptr;  // device copy of host fields
  int64_t field_stage_len = 0;
  double* field_rows = nullptr;   // the call's fields in row order (n_fields x n_pad)
  int64_t field_rows_len = 0;
  double* col_stage = nullptr;    // per-slot outputs for host destinations
  int64_t col_stage_len = 0;
  // cell -> vertex projection of vertex-vector handles (uploaded on first use)
  int64_t* proj_ptr = nullptr;
  int32_t* proj_tri = nullptr;
  double* proj_w = nullptr;
  double* proj_in = nullptr;      // device copy of a host cell field
};

// Partial sums of a one-column launch (units of G): two parities of five
// iteration sums, then the floor norm of a replacement, ||M phi||^2 and the
// finish sums. Launch L writes parity L & 1 and its successor reads it.
constexpr int kPq = 0, kZu = 1, kUu = 2, kRz = 3, kRr = 4, kPerParity = 5;
__host__ __device__ constexpr int pidx(int parity, int q) { return parity * kPerParity + q; }
enum { P_FL = 2 * kPerParity, P_BB, P_RES, P_EN, P_COUNT };

// Work space of ifl_filter_noalloc: the one-column path's block partials
// (P_COUNT x G doubles) followed by its Scalars, in a file-scope device
// array, so that the call allocates nothing. Each GPU holds its own copy
// for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns on that device (noalloc_scratch_addr),
// never through the symbol's name.
constexpr size_t kNoallocScratchBytes = 64 * 1024;
constexpr size_t kNoallocScalarsOffset = kNoallocScratchBytes - 256;  // Scalars in the last 256 bytes
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
static_assert(2 * sizeof(Scalars) <= 256, "both Scalars copies must fit the scratch tail");

// Attainable accuracy of an FP64 residual r = b - S x: its rounding error is
// bounded by a small multiple of u ||(|b| + |S| |x|)||, u = 2^-53. A true
// residual at or below kFloorUnits * u times that norm cannot be reduced
// further in FP64 and counts as converged.
constexpr double kUnitRoundoff = 1.1102230246251565e-16;
constexpr double kFloorUnits = 8.0;
// Reliable updates: an FP64 residual replacement whenever the recursive
// residual fell by 100x since the last true residual (delta^2 = 1e-4), in
// both precisions, and the CG directions continue across it. Replacing only
// when the recursive residual meets the tolerance lets it drift so far at
// cond(S) ~ 1e6-1e7 that the continued iteration stagnates (a 10^4 fall
// already stalls the circumcentre n = 2 system at lambda = 32h); restarting
// instead converges, but 20-100% slower there.
constexpr double kReplaceDelta2 = 1e-4;

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int logical_block(int G) {
  const int b = blockIdx.x;
  if (G % kXcd) return b;
  return (b % kXcd) * (G / kXcd) + b / kXcd;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sum of NV values, fixed order; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[kWavesPerBlock]) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = wave_sum(v[i]);
    if (lane == 0) lds[i][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < kWavesPerBlock; ++w) s += lds[i][w];
      v[i] = s;
    }
  }
}

// Sum of a partial array a[0..G) by the whole block, fixed order; every
// thread returns the same value.
__device__ __forceinline__ double reduce_partials(const double* a, int G, double* lds_w, double* lds_out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < G; i += kBlock) s += a[i];
  s = wave_sum(s);
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  if (lane == 0) lds_w[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWavesPerBlock; ++w) t += lds_w[w];
    *lds_out = t;
  }
  __syncthreads();
  return *lds_out;
}

template <typename T>
struct alignas(2 * sizeof(T)) Pack2 {
  T a, b;
};

// Vectors of a one-column solve; x, z, u = diag(S)^-1 S p and p alternate
// between two buffers (a launch gathers the ones it reads while it writes
// the others).
template <typename T>
struct CgVecs {
  T* z[2];
  T* u[2];
  T* p[2];
  T* d;
  double* x[2];
};

struct Mat {
  int64_t n, n_slices;
  const int64_t* sptr;
  const int32_t* col;
  const double* val64;
  const float* val32;
  const double* kdiag64;
  const float* kdiag32;
  const double* mass64;
};

template <typename T>
__device__ __forceinline__ const T* mval(const Mat& m);
template <>
__device__ __forceinline__ const double* mval<double>(const Mat& m) { return m.val64; }
template <>
__device__ __forceinline__ const float* mval<float>(const Mat& m) { return m.val32; }

// Only an FP64 true residual r = M phi - S x may stop a solve, in both
// precisions: a recursive residual drifts from the true one when S is badly
// conditioned (an FP64 solve stopped on it at cond(S) ~ 1e6 was accurate to
// ~1e-7 only).

// Modes of a one-column launch, decided in its prologue (the same in every
// block, from the same partials) and recorded for the next launch.
enum { M_INIT = 0, M_ITER = 1, M_REPLACE = 2, M_DONE = 3 };

// ---------------------------------------------------------------- kernels
// Start of a solve: x0 = phi, r0 = M phi - S phi = -c K_n phi (FP64 values),
// diag(S) stored, x0 and z0 = r0 / diag(S) into buffers 0, and the sums of (r, z),
// (r, r) (as parity 1, read by launch 0) and ||M phi||^2. Scalars copy 0 is
// the state launch 0 reads.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(Mat m, CgVecs<T> v, const double* phi, double* part, Scalars* sc,
                                                  double c, int G, int spb) {
  __shared__ double lds[3][kWavesPerBlock];
  const int lb = logical_block(G);
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  double acc3[3] = {0.0, 0.0, 0.0};
  const int64_t s_end = min((int64_t)(lb + 1) * spb, m.n_slices);
  for (int64_t s = (int64_t)lb * spb + wid; s < s_end; s += kWavesPerBlock) {
    const int64_t row = s * kWave + lane;
    if (row >= m.n) continue;
    const int64_t base = m.sptr[s];
    const int w = (int)((m.sptr[s + 1] - base) / kWave);
    double a = 0.0;
    for (int k = 0; k < w; ++k) {
      const int64_t e = base + (int64_t)k * kWave + lane;
      a += m.val64[e] * phi[m.col[e]];
    }
    const double ph = phi[row];
    const double kd = m.kdiag64[row];
    const double r64 = -c * (kd * ph + a);
    const double d64 = m.mass64[row] + c * kd;
    const T rt = (T)r64, dt = (T)d64;
    const T zt = rt / dt;
    v.x[0][row] = ph;
    v.z[0][row] = zt;
    v.d[row] = dt;
    acc3[0] += (double)rt * (double)zt;
    acc3[1] += r64 * r64;
    const double b = m.mass64[row] * ph;
    acc3[2] += b * b;
  }
  block_sum<3>(acc3, lds);
  if (threadIdx.x == 0) {
    part[pidx(1, kRz) * G + lb] = acc3[0];
    part[pidx(1, kRr) * G + lb] = acc3[1];
    part[P_BB * G + lb] = acc3[2];
    part[P_FL * G + lb] = 0.0;
    if (lb == 0) {
      Scalars s0{};
      s0.c = c;
      s0.mode = M_INIT;
      sc[0] = s0;
    }
  }
}

// One block: tolerance and reference norms from the init sums.
__global__ __launch_bounds__(kBlock) void k_setup(double* part, Scalars* sc, double rtol, int G) {
  __shared__ double lw[kWavesPerBlock];
  __shared__ double lo;
  const double bb = reduce_partials(part + P_BB * G, G, lw, &lo);
  if (threadIdx.x == 0) {
    sc[0].bb = bb;
    sc[0].tol2 = rtol * rtol * bb;
  }
}

// Sums of NQ partial arrays src[q][0..G) by the whole block in one pass
// (fixed order); every thread returns the same values.
template <int NQ>
__device__ __forceinline__ void reduce_many(const double* const (&src)[NQ], int G, double (&out)[NQ],
                                            double (*lds)[kWavesPerBlock]) {
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += kBlock) s += src[q][i];
    v[q] = wave_sum(s);
  }
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[q][wid] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double t = 0.0;
    for (int w = 0; w < kWavesPerBlock; ++w) t += lds[q][w];
    out[q] = t;
  }
}

// One CG iteration per launch (or, when due, the FP64 residual
// replacement), with u = diag(S)^-1 S p in place of q = S p (d = diag(S);
// z = d^-1 r is the residual state; r = d z is formed where needed).
//
// The prologue finishes the previous launch's sums and decides, in every
// block alike:
//  * after the start or a replacement (an FP64 true residual): stop if it
//    meets max(tol, attainable-accuracy floor); else iterate with alpha = 0
//    and beta = 0 after the start, beta = rho_true / rho_prev after a
//    replacement (the directions continue: the residual is replaced, the
//    Krylov directions are kept);
//  * after an iteration: alpha = rho / (p, q) (breakdown if (p, q) <= 0);
//    replace if the recursive residual meets the tolerance or fell by
//    100x since the last true residual; else iterate
//    with beta = rho_next / rho, rho_next = rho - 2 alpha (q, z) + alpha^2
//    (q, d^-1 q) (the rho of z - alpha d^-1 q, known before that z exists).
//
// Iterate (buffers: read x, z, u, p [L & 1], write [(L + 1) & 1]):
//    z' = z - alpha u          (own row and every gathered neighbour)
//    x += alpha p              (FP64)
//    p' = z' + beta p
//    u' = z' + d^-1 c K_off z' + beta u   (= d^-1 S p')
//  with the sums (p', q'), (q', z'), (q', d^-1 q'), (r', z'), (r', r').
// Replace: x' = x + alpha p (own row and gathered neighbours, FP64), r =
//  M phi - S x' with FP64 values, z = r / d, p and u carried to the other
//  buffers, with the sums (r, z), (r, r) and the floor norm
//  || |M phi| + |M x'| + c |K_n| |x'| ||^2.
// Block 0 writes the state copy (L + 1) & 1, which no block of launch L
// reads; a stopping launch records the buffer that holds the final x.
// 'launch' is the host's index of this launch.
template <typename T, bool MIXED, int U>
__global__ __launch_bounds__(kBlock) void k_cg(Mat m, CgVecs<T> v, const double* phi, double* part, Scalars* sc,
                                                int launch, int G, int spb, int max_iter) {
  __shared__ double lds6[6][kWavesPerBlock];
  __shared__ double lds5[5][kWavesPerBlock];
  const int cur = launch & 1, nxt = cur ^ 1;
  const Scalars s0 = sc[cur];
  const int lb = logical_block(G);
  const bool leader = lb == 0 && threadIdx.x == 0;
  if (s0.done) {
    if (leader) {
      ScalarsMut s1 = mut_of(s0);
      s1.fused_bits &= ~(1u << (launch & 31));
      put_scalars(&sc[nxt], &sc[cur], s1);
    }
    return;
  }
  // previous launch's sums (parity nxt = (launch - 1) & 1)
  double q[6];
  {
    const double* const src[6] = {part + pidx(nxt, kPq) * G, part + pidx(nxt, kZu) * G, part + pidx(nxt, kUu) * G,
                                  part + pidx(nxt, kRz) * G, part + pidx(nxt, kRr) * G, part + P_FL * G};
    reduce_many<6>(src, G, q, lds6);
  }
  const double pq = q[0], zu = q[1], uu = q[2], rz = q[3], rr = q[4], fl = q[5];
  ScalarsMut s1 = mut_of(s0);
  s1.fused_bits &= ~(1u << (launch & 31));
  int mode;
  double alpha = 0.0, beta = 0.0;
  bool restart = false;
  if (s0.mode != M_ITER) {
    // a true residual: stop or (re)start
    const double floor2 = fl * (kFloorUnits * kUnitRoundoff) * (kFloorUnits * kUnitRoundoff);
    s1.rr_last = rr;
    s1.rr_ref = rr;
    if (rr <= fmax(s0.tol2, floor2)) {
      s1.done = 1;
      mode = M_DONE;
    } else if (s0.iters >= max_iter) {
      s1.done = 3;
      mode = M_DONE;
    } else {
      mode = M_ITER;
      restart = s0.mode == M_INIT;
      beta = restart ? 0.0 : rz / s0.rho;
    }
  } else {
    alpha = rz / pq;
    s1.rr_last = rr;
    if (!(pq > 0.0) || !isfinite(alpha)) {
      s1.done = 2;
      mode = M_DONE;
    } else if (rr <= s0.tol2 || rr <= kReplaceDelta2 * s0.rr_ref) {
      mode = M_REPLACE;
      s1.rho = rz;  // rho of the z this replacement supersedes (beta after it)
      s1.updates += 1;
    } else if (s0.iters >= max_iter) {
      s1.done = 3;
      mode = M_DONE;
    } else {
      mode = M_ITER;
      beta = (rz - 2.0 * alpha * zu + alpha * alpha * uu) / rz;
    }
  }
  if (mode == M_DONE) s1.xbuf = cur;
  if (mode == M_ITER) {
    s1.iters += 1;
    if (alpha != 0.0) s1.fused_bits |= 1u << (launch & 31);
  }
  s1.mode = mode;
  if (mode == M_DONE) {
    if (leader) put_scalars(&sc[nxt], &sc[cur], s1);
    return;
  }
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int64_t s_end = min((int64_t)(lb + 1) * spb, m.n_slices);
  const T* __restrict__ zin = v.z[cur];
  const T* __restrict__ uin = v.u[cur];
  const T* __restrict__ pin = v.p[cur];
  T* __restrict__ zout = v.z[nxt];
  T* __restrict__ uout = v.u[nxt];
  T* __restrict__ pout = v.p[nxt];
  const double* __restrict__ xin = v.x[cur];
  double* __restrict__ xout = v.x[nxt];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (mode == M_REPLACE) {
    const double c = s0.c;
    for (int64_t s = (int64_t)lb * spb + wid; s < s_end; s += kWavesPerBlock) {
      const int64_t row = s * kWave + lane;
      if (row >= m.n) continue;
      const int64_t base = m.sptr[s];
      const int w = (int)((m.sptr[s + 1] - base) / kWave);
      double a = 0.0, aa = 0.0;
      for (int k0 = 0; k0 < w; k0 += U) {
        int32_t cu[U];
        double vu[U], xu[U];
        T pu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t e = base + (int64_t)(k0 + u) * kWave + lane;
          cu[u] = m.col[e];
          const double vv = m.val64[e];
          vu[u] = k0 + u < w ? vv : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          xu[u] = xin[cu[u]];
          pu[u] = pin[cu[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double xn = fma(alpha, (double)pu[u], xu[u]);
          a = fma(vu[u], xn, a);
          aa = fma(fabs(vu[u]), fabs(xn), aa);
        }
      }
      const T pi = pin[row], ui = uin[row];
      const double xi = fma(alpha, (double)pi, xin[row]);
      const double mi = m.mass64[row], kd = m.kdiag64[row], ph = phi[row];
      const double r64 = mi * (ph - xi) - c * (kd * xi + a);
      const double mag = fabs(mi * ph) + fabs(mi * xi) + c * (fabs(kd * xi) + aa);
      const T rt = (T)r64;
      const T zt = rt / v.d[row];
      xout[row] = xi;
      zout[row] = zt;
      pout[row] = pi;
      uout[row] = ui;
      acc[0] += (double)rt * (double)zt;
      acc[1] += r64 * r64;
      acc[2] += mag * mag;
    }
  } else {
    const T at = (T)alpha, bt = (T)beta, c = (T)s0.c;
    const T* __restrict__ val = mval<T>(m);
    const bool step = alpha != 0.0;  // z moves (and x); else z' = z, and u is not gathered
    for (int64_t s = (int64_t)lb * spb + wid; s < s_end; s += kWavesPerBlock) {
      const int64_t row = s * kWave + lane;
      if (row >= m.n) continue;
      const int64_t base = m.sptr[s];
      const int w = (int)((m.sptr[s + 1] - base) / kWave);
      // entries U at a time: index / value loads, then the gathers, then
      // the FMAs in entry order; loads past the row's end stay in bounds
      // (the next slice or the zero tail) and their values are replaced by 0
      T a = (T)0;
      for (int k0 = 0; k0 < w; k0 += U) {
        int32_t cu[U];
        T vu[U], zu_[U], uu_[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t e = base + (int64_t)(k0 + u) * kWave + lane;
          cu[u] = m.col[e];
          const T vv = val[e];
          vu[u] = k0 + u < w ? vv : (T)0;
        }
        if (step) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            zu_[u] = zin[cu[u]];
            uu_[u] = uin[cu[u]];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) a = fma(vu[u], fma(-at, uu_[u], zu_[u]), a);
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) zu_[u] = zin[cu[u]];
#pragma unroll
          for (int u = 0; u < U; ++u) a = fma(vu[u], zu_[u], a);
        }
      }
      const T zi = zin[row], di = v.d[row];
      const T ui = restart ? (T)0 : uin[row];
      const T pi = restart ? (T)0 : pin[row];
      const T zn = step ? fma(-at, ui, zi) : zi;
      const double xi = xin[row];
      xout[row] = step ? fma(alpha, (double)pi, xi) : xi;
      const T pn = fma(bt, pi, zn);
      const T un = fma(bt, ui, zn + (c * a) / di);
      zout[row] = zn;
      pout[row] = pn;
      uout[row] = un;
      const double dd = (double)di, zz = (double)zn, uv = (double)un;
      acc[0] += dd * (double)pn * uv;
      acc[1] += dd * zz * uv;
      acc[2] += dd * uv * uv;
      acc[3] += dd * zz * zz;
      acc[4] += (dd * zz) * (dd * zz);
    }
  }
  block_sum<5>(acc, lds5);
  if (threadIdx.x == 0) {
    if (mode == M_REPLACE) {
      part[pidx(cur, kRz) * G + lb] = acc[0];
      part[pidx(cur, kRr) * G + lb] = acc[1];
      part[P_FL * G + lb] = acc[2];
    } else {
      part[pidx(cur, kPq) * G + lb] = acc[0];
      part[pidx(cur, kZu) * G + lb] = acc[1];
      part[pidx(cur, kUu) * G + lb] = acc[2];
      part[pidx(cur, kRz) * G + lb] = acc[3];
      part[pidx(cur, kRr) * G + lb] = acc[4];
    }
    if (lb == 0) put_scalars(&sc[nxt], &sc[cur], s1);
  }
}

// ------------------------------------------------- complex-shifted solves
// Complex arithmetic on (re, im) pairs; every product is written with the
// same fma sequence wherever it is evaluated, so a value formed for a
// gathered neighbour is bitwise the value that row's own lane stores.
template <typename T>
struct Cx {
  T r, i;
};
template <typename T>
__device__ __forceinline__ Cx<T> cfma(Cx<T> a, Cx<T> b, Cx<T> c) {  // a b + c
  return Cx<T>{fma(a.r, b.r, fma(-a.i, b.i, c.r)), fma(a.r, b.i, fma(a.i, b.r, c.i))};
}
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return Cx<T>{fma(a.r, b.r, -a.i * b.i), fma(a.r, b.i, a.i * b.r)};
}
template <typename T>
__device__ __forceinline__ Cx<T> cdiv(Cx<T> a, Cx<T> b) {
  const T den = fma(b.r, b.r, b.i * b.i);
  return Cx<T>{fma(a.r, b.r, a.i * b.i) / den, fma(a.i, b.r, -a.r * b.i) / den};
}
template <typename T>
__device__ __forceinline__ Cx<T> cld(const T* p, int64_t j) {
  const Pack2<T> v = *reinterpret_cast<const Pack2<T>*>(p + 2 * j);
  return Cx<T>{v.a, v.b};
}
template <typename T>
__device__ __forceinline__ void cst(T* p, int64_t j, Cx<T> x) {
  *reinterpret_cast<Pack2<T>*>(p + 2 * j) = Pack2<T>{x.r, x.i};
}
__device__ __forceinline__ Cx<double> cd(Cx<float> a) { return Cx<double>{(double)a.r, (double)a.i}; }
__device__ __forceinline__ Cx<double> cd(Cx<double> a) { return a; }
template <typename T>
__device__ __forceinline__ Cx<T> ct(Cx<double> a) {
  return Cx<T>{(T)a.r, (T)a.i};
}

template <typename T>
struct CVecs {
  T* z[2];
  T* u[2];
  T* p[2];
  T* d;          // diag(M + sigma K), complex
  double* x[2];  // solution, complex FP64
};

// Start of a shifted solve of (M + sigma K) y = M phi from y0 = phi: r0 =
// -sigma K phi with FP64 values, d = m + sigma diag(K), z0 = r0 / d into
// buffer 0, and the sums of (r, z) (complex), ||r||^2 and ||M phi||^2 (as
// parity 1, read by launch 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cinit(Mat m, CVecs<T> v, const double* phi, double* part, CScalars* sc,
                                                   double sr, double si, int G, int spb) {
  __shared__ double lds[4][kWavesPerBlock];
  const int lb = logical_block(G);
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const Cx<double> sig{sr, si};
  const int64_t s_end = min((int64_t)(lb + 1) * spb, m.n_slices);
  for (int64_t s = (int64_t)lb * spb + wid; s < s_end; s += kWavesPerBlock) {
    const int64_t row = s * kWave + lane;
    if (row >= m.n) continue;
    const int64_t base = m.sptr[s];
    const int w = (int)((m.sptr[s + 1] - base) / kWave);
    double a = 0.0;
    for (int k = 0; k < w; ++k) {
      const int64_t e = base + (int64_t)k * kWave + lane;
      a += m.val64[e] * phi[m.col[e]];
    }
    const double ph = phi[row], kd = m.kdiag64[row], mi = m.mass64[row];
    const double kphi = kd * ph + a;
    const Cx<double> r64{-sr * kphi, -si * kphi};
    const Cx<T> dt = ct<T>(Cx<double>{fma(sr, kd, mi), si * kd});
    const Cx<T> rt = ct<T>(r64);
    const Cx<T> zt = cdiv(rt, dt);
    cst(v.x[0], row, Cx<double>{ph, 0.0});
    cst(v.z[0], row, zt);
    cst(v.d, row, dt);
    const Cx<double> rz = cmul(cd(rt), cd(zt));
    acc[0] += rz.r;
    acc[1] += rz.i;
    acc[2] += r64.r * r64.r + r64.i * r64.i;
    acc[3] += (mi * ph) * (mi * ph);
  }
  block_sum<4>(acc, lds);
  if (threadIdx.x == 0) {
    part[cidx(1, kCRzR) * G + lb] = acc[0];
    part[cidx(1, kCRzI) * G + lb] = acc[1];
    part[cidx(1, kCRr) * G + lb] = acc[2];
    part[CP_BB * G + lb] = acc[3];
    part[CP_FL * G + lb] = 0.0;
    if (lb == 0) {
      CScalars s0{};
      s0.sr = sr;
      s0.si = si;
      s0.mode = M_INIT;
      sc[0] = s0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_csetup(double* part, CScalars* sc, double rtol, int G) {
  __shared__ double lw[kWavesPerBlock];
  __shared__ double lo;
  const double bb = reduce_partials(part + CP_BB * G, G, lw, &lo);
  if (threadIdx.x == 0) {
    sc[0].bb = bb;
    sc[0].tol2 = rtol * rtol * bb;
  }
}

// One iteration of Jacobi-preconditioned COCG on the complex-symmetric
// (M + sigma K) y = M phi per launch, or its FP64 residual replacement: the
// complex counterpart of k_cg, with the bilinear form (a, b) = sum a_i b_i
// (no conjugation) in every inner product of the recurrences, so that the
// algebra of k_cg carries over (rho_next = rho - 2 alpha (q, z) + alpha^2
// (q, d^-1 q)); the stopping and replacement tests use the Euclidean norm
// ||r||^2 = sum |r_i|^2. d^-1 (M + sigma K) z' = z' + sigma d^-1 K_off z'.
template <typename T, bool MIXED, int U>
__global__ __launch_bounds__(kBlock) void k_ccg(Mat m, CVecs<T> v, const double* phi, double* part, CScalars* sc,
                                                 int launch, int G, int spb, int max_iter) {
  __shared__ double lds10[10][kWavesPerBlock];
  __shared__ double lds9[9][kWavesPerBlock];
  const int cur = launch & 1, nxt = cur ^ 1;
  const CScalars s0 = sc[cur];
  const int lb = logical_block(G);
  const bool leader = lb == 0 && threadIdx.x == 0;
  if (s0.done) {
    if (leader) {
      CScalars s1 = s0;
      s1.fused_bits &= ~(1u << (launch & 31));
      sc[nxt] = s1;
    }
    return;
  }
  double q[10];
  {
    const double* const src[10] = {
        part + cidx(nxt, kCPqR) * G, part + cidx(nxt, kCPqI) * G, part + cidx(nxt, kCZuR) * G,
        part + cidx(nxt, kCZuI) * G, part + cidx(nxt, kCUuR) * G, part + cidx(nxt, kCUuI) * G,
        part + cidx(nxt, kCRzR) * G, part + cidx(nxt, kCRzI) * G, part + cidx(nxt, kCRr) * G, part + CP_FL * G};
    reduce_many<10>(src, G, q, lds10);
  }
  const Cx<double> pq{q[0], q[1]}, zu{q[2], q[3]}, uu{q[4], q[5]}, rz{q[6], q[7]};
  const double rr = q[8], fl = q[9];
  CScalars s1 = s0;
  s1.fused_bits &= ~(1u << (launch & 31));
  int mode;
  Cx<double> alpha{0.0, 0.0}, beta{0.0, 0.0};
  bool restart = false;
  if (s0.mode != M_ITER) {
    const double floor2 = fl * (kFloorUnits * kUnitRoundoff) * (kFloorUnits * kUnitRoundoff);
    s1.rr_last = rr;
    s1.rr_ref = rr;
    if (rr <= fmax(s0.tol2, floor2)) {
      s1.done = 1;
      mode = M_DONE;
    } else if (s0.iters >= max_iter) {
      s1.done = 3;
      mode = M_DONE;
    } else {
      mode = M_ITER;
      restart = s0.mode == M_INIT;
      beta = restart ? Cx<double>{0.0, 0.0} : cdiv(rz, Cx<double>{s0.rho_r, s0.rho_i});
    }
  } else {
    alpha = cdiv(rz, pq);
    s1.rr_last = rr;
    if (!(pq.r * pq.r + pq.i * pq.i > 0.0) || !isfinite(alpha.r) || !isfinite(alpha.i)) {
      s1.done = 2;
      mode = M_DONE;
    } else if (rr <= s0.tol2 || rr <= kReplaceDelta2 * s0.rr_ref) {
      mode = M_REPLACE;
      s1.rho_r = rz.r;
      s1.rho_i = rz.i;
      s1.updates += 1;
    } else if (s0.iters >= max_iter) {
      s1.done = 3;
      mode = M_DONE;
    } else {
      mode = M_ITER;
      // (rho - 2 alpha zu + alpha^2 uu) / rho
      const Cx<double> t1 = cmul(Cx<double>{-2.0 * alpha.r, -2.0 * alpha.i}, zu);
      const Cx<double> t2 = cmul(cmul(alpha, alpha), uu);
      beta = cdiv(Cx<double>{rz.r + t1.r + t2.r, rz.i + t1.i + t2.i}, rz);
    }
  }
  if (mode == M_DONE) s1.xbuf = cur;
  if (mode == M_ITER) {
    s1.iters += 1;
    if (alpha.r != 0.0 || alpha.i != 0.0) s1.fused_bits |= 1u << (launch & 31);
  }
  s1.mode = mode;
  if (mode == M_DONE) {
    if (leader) sc[nxt] = s1;
    return;
  }
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int64_t s_end = min((int64_t)(lb + 1) * spb, m.n_slices);
  const T* __restrict__ zin = v.z[cur];
  const T* __restrict__ uin = v.u[cur];
  const T* __restrict__ pin = v.p[cur];
  T* __restrict__ zout = v.z[nxt];
  T* __restrict__ uout = v.u[nxt];
  T* __restrict__ pout = v.p[nxt];
  const double* __restrict__ xin = v.x[cur];
  double* __restrict__ xout = v.x[nxt];
  const Cx<double> sig{s0.sr, s0.si};
  double acc[9] = {};
  if (mode == M_REPLACE) {
    const double sabs = sqrt(sig.r * sig.r + sig.i * sig.i);
    for (int64_t s = (int64_t)lb * spb + wid; s < s_end; s += kWavesPerBlock) {
      const int64_t row = s * kWave + lane;
      if (row >= m.n) continue;
      const int64_t base = m.sptr[s];
      const int w = (int)((m.sptr[s + 1] - base) / kWave);
      Cx<double> a{0.0, 0.0};
      double aa = 0.0;
      for (int k0 = 0; k0 < w; k0 += U) {
        int32_t cu[U];
        double vu[U];
        Cx<double> xu[U];
        Cx<T> pu[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t e = base + (int64_t)(k0 + u) * kWave + lane;
          cu[u] = m.col[e];
          const double vv = m.val64[e];
          vu[u] = k0 + u < w ? vv : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          xu[u] = cld(xin, cu[u]);
          pu[u] = cld(pin, cu[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const Cx<double> xn = cfma(alpha, cd(pu[u]), xu[u]);
          a.r = fma(vu[u], xn.r, a.r);
          a.i = fma(vu[u], xn.i, a.i);
          aa = fma(fabs(vu[u]), sqrt(xn.r * xn.r + xn.i * xn.i), aa);
        }
      }
      const Cx<T> pi = cld(pin, row), ui = cld(uin, row);
      const Cx<double> xi = cfma(alpha, cd(pi), cld(xin, row));
      const double mi = m.mass64[row], kd = m.kdiag64[row], ph = phi[row];
      // r = M (phi - x) - sigma (kd x + K_off x)
      const Cx<double> kx{fma(kd, xi.r, a.r), fma(kd, xi.i, a.i)};
      const Cx<double> skx = cmul(sig, kx);
      const Cx<double> r64{mi * (ph - xi.r) - skx.r, -mi * xi.i - skx.i};
      const double xa = sqrt(xi.r * xi.r + xi.i * xi.i);
      const double mag = fabs(mi * ph) + fabs(mi) * xa + sabs * (fabs(kd) * xa + aa);
      const Cx<T> rt = ct<T>(r64);
      const Cx<T> zt = cdiv(rt, cld(v.d, row));
      cst(xout, row, xi);
      cst(zout, row, zt);
      cst(pout, row, pi);
      cst(uout, row, ui);
      const Cx<double> rzv = cmul(cd(rt), cd(zt));
      acc[6] += rzv.r;
      acc[7] += rzv.i;
      acc[8] += r64.r * r64.r + r64.i * r64.i;
      acc[0] += mag * mag;  // the floor norm (stored in its own slot below)
    }
  } else {
    const Cx<T> at = ct<T>(alpha), bt = ct<T>(beta), nat = ct<T>(Cx<double>{-alpha.r, -alpha.i});
    const Cx<T> st = ct<T>(sig);
    const T* __restrict__ val = mval<T>(m);
    const bool step = alpha.r != 0.0 || alpha.i != 0.0;
    for (int64_t s = (int64_t)lb * spb + wid; s < s_end; s += kWavesPerBlock) {
      const int64_t row = s * kWave + lane;
      if (row >= m.n) continue;
      const int64_t base = m.sptr[s];
      const int w = (int)((m.sptr[s + 1] - base) / kWave);
      Cx<T> a{(T)0, (T)0};
      for (int k0 = 0; k0 < w; k0 += U) {
        int32_t cu[U];
        T vu[U];
        Cx<T> zu_[U], uu_[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t e = base + (int64_t)(k0 + u) * kWave + lane;
          cu[u] = m.col[e];
          const T vv = val[e];
          vu[u] = k0 + u < w ? vv : (T)0;
        }
        if (step) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            zu_[u] = cld(zin, cu[u]);
            uu_[u] = cld(uin, cu[u]);
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const Cx<T> zn = cfma(nat, uu_[u], zu_[u]);
            a.r = fma(vu[u], zn.r, a.r);
            a.i = fma(vu[u], zn.i, a.i);
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) zu_[u] = cld(zin, cu[u]);
#pragma unroll
          for (int u = 0; u < U; ++u) {
            a.r = fma(vu[u], zu_[u].r, a.r);
            a.i = fma(vu[u], zu_[u].i, a.i);
          }
        }
      }
      const Cx<T> zi = cld(zin, row), di = cld(v.d, row);
      const Cx<T> ui = restart ? Cx<T>{(T)0, (T)0} : cld(uin, row);
      const Cx<T> pi = restart ? Cx<T>{(T)0, (T)0} : cld(pin, row);
      const Cx<T> zn = step ? cfma(nat, ui, zi) : zi;
      const Cx<double> xi = cld(xin, row);
      cst(xout, row, step ? cfma(alpha, cd(pi), xi) : xi);
      const Cx<T> pn = cfma(bt, pi, zn);
      const Cx<T> sa = cdiv(cmul(st, a), di);  // sigma d^-1 K_off z'
      const Cx<T> un = cfma(bt, ui, Cx<T>{zn.r + sa.r, zn.i + sa.i});
      cst(zout, row, zn);
      cst(pout, row, pn);
      cst(uout, row, un);
      const Cx<double> dd = cd(di), zz = cd(zn), uv = cd(un);
      const Cx<double> du = cmul(dd, uv);
      const Cx<double> pqv = cmul(cd(pn), du), zuv = cmul(zz, du), uuv = cmul(uv, du);
      const Cx<double> dz = cmul(dd, zz);
      const Cx<double> rzv = cmul(zz, dz);
      acc[0] += pqv.r;
      acc[1] += pqv.i;
      acc[2] += zuv.r;
      acc[3] += zuv.i;
      acc[4] += uuv.r;
      acc[5] += uuv.i;
      acc[6] += rzv.r;
      acc[7] += rzv.i;
      acc[8] += dz.r * dz.r + dz.i * dz.i;
    }
    (void)at;
  }
  block_sum<9>(acc, lds9);
  if (threadIdx.x == 0) {
    if (mode == M_REPLACE) {
      part[cidx(cur, kCRzR) * G + lb] = acc[6];
      part[cidx(cur, kCRzI) * G + lb] = acc[7];
      part[cidx(cur, kCRr) * G + lb] = acc[8];
      part[CP_FL * G + lb] = acc[0];
    } else {
#pragma unroll
      for (int q2 = 0; q2 < kCPerParity; ++q2) part[cidx(cur, q2) * G + lb] = acc[q2];
    }
    if (lb == 0) sc[nxt] = s1;
  }
}

// acc += w x[stride i] over the rows (the real part of a complex solution:
// stride 2)
__global__ void k_accumulate(double* __restrict__ acc, const double* __restrict__ x, int stride, double w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) acc[i] = fma(w, x[(int64_t)stride * i], acc[i]);
}

// End of a shifted solve: the summed solution to the caller's numbering,
// with the partials of the FP64 true residual of S = M + c K_n itself (K_n
// in m) and of sum M x^2.
__global__ __launch_bounds__(kBlock) void k_sfinish(Mat m, const double* x, const double* phi, double c,
                                                    const int64_t* entity, double* out, double* part, int G, int spb) {
  __shared__ double lds[2][kWavesPerBlock];
  const int lb = logical_block(G);
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  double acc[2] = {0.0, 0.0};
  const int64_t s_end = min((int64_t)(lb + 1) * spb, m.n_slices);
  for (int64_t s = (int64_t)lb * spb + wid; s < s_end; s += kWavesPerBlock) {
    const int64_t row = s * kWave + lane;
    if (row >= m.n) continue;
    const int64_t base = m.sptr[s];
    const int w = (int)((m.sptr[s + 1] - base) / kWave);
    double a = 0.0;
    for (int k = 0; k < w; ++k) {
      const int64_t e = base + (int64_t)k * kWave + lane;
      a += m.val64[e] * x[m.col[e]];
    }
    const double xi = x[row];
    const double r64 = m.mass64[row] * (phi[row] - xi) - c * (m.kdiag64[row] * xi + a);
    if (out) out[entity[row]] = xi;
    acc[0] += r64 * r64;
    acc[1] += m.mass64[row] * xi * xi;
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x == 0) {
    part[CP_RES * G + lb] = acc[0];
    part[CP_EN * G + lb] = acc[1];
  }
}

// End of a solve: x (the buffer the stopping launch recorded, else the last
// one written) scattered to the caller's numbering; partials of the true
// FP64 residual and of sum M x^2.
__global__ __launch_bounds__(kBlock) void k_finish(Mat m, const double* x0, const double* x1, const double* phi,
                                                   const int64_t* entity, double* out, double* part,
                                                   const Scalars* sc, int last_buf, int G, int spb) {
  __shared__ double lds[2][kWavesPerBlock];
  const int lb = logical_block(G);
  const double c = sc->c;
  const double* __restrict__ x = (sc->done ? sc->xbuf : last_buf) ? x1 : x0;
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  double acc[2] = {0.0, 0.0};
  const int64_t s_end = min((int64_t)(lb + 1) * spb, m.n_slices);
  for (int64_t s = (int64_t)lb * spb + wid; s < s_end; s += kWavesPerBlock) {
    const int64_t row = s * kWave + lane;
    if (row >= m.n) continue;
    const int64_t base = m.sptr[s];
    const int w = (int)((m.sptr[s + 1] - base) / kWave);
    double a = 0.0;
    for (int k = 0; k < w; ++k) {
      const int64_t e = base + (int64_t)k * kWave + lane;
      a += m.val64[e] * x[m.col[e]];
    }
    const double xi = x[row];
    const double r64 = m.mass64[row] * (phi[row] - xi) - c * (m.kdiag64[row] * xi + a);
    if (out) out[entity[row]] = xi;
    acc[0] += r64 * r64;
    acc[1] += m.mass64[row] * xi * xi;
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x == 0) {
    part[P_RES * G + lb] = acc[0];
    part[P_EN * G + lb] = acc[1];
  }
}

__global__ __launch_bounds__(kBlock) void k_finish_scalars(double* part, Scalars* sc, int G) {
  __shared__ double lw[kWavesPerBlock];
  __shared__ double lo;
  const double res = reduce_partials(part + P_RES * G, G, lw, &lo);
  const double en = reduce_partials(part + P_EN * G, G, lw, &lo);
  if (threadIdx.x == 0) {
    sc->res2 = res;
    sc->energy2 = en;
  }
}

// Caller numbering -> internal order; flags non-finite wet entries.
__global__ void k_gather_field(const double* __restrict__ src, const int64_t* __restrict__ entity, int64_t n,
                               double* __restrict__ dst, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = src[entity[i]];
  if (!isfinite(v)) atomicOr(flag, 1);
  dst[i] = v;
}

// Cell -> vertex projection (Sect. 2.1.2): one thread per dof d (rows 2d,
// 2d+1) sums w_e u_c over its incident active triangles, w_e = (A_c / 3) /
// M_d, and writes (east, north) to the dof's vertex in the caller numbering.
__global__ __launch_bounds__(kBlock) void k_project_cells(int64_t nd, const int64_t* ptr, const int32_t* tri,
                                                           const double* w, const int64_t* entity,
                                                           const double* cells, double* out) {
  const int64_t d = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (d >= nd) return;
  double ue = 0.0, un = 0.0;
  for (int64_t e = ptr[d]; e < ptr[d + 1]; ++e) {
    const int64_t t = tri[e];
    ue += w[e] * cells[2 * t];
    un += w[e] * cells[2 * t + 1];
  }
  const int64_t v2 = entity[2 * d];
  out[v2] = ue;
  out[v2 + 1] = un;
}

// y = S x with FP64 values (internal order), scattered to the caller numbering.
__global__ __launch_bounds__(kBlock) void k_apply(Mat m, const double* x, double c, const int64_t* entity,
                                                  double* out) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int64_t s = (int64_t)blockIdx.x * kWavesPerBlock + wid;
  if (s >= m.n_slices) return;
  const int64_t row = s * kWave + lane;
  if (row >= m.n) return;
  const int64_t base = m.sptr[s];
  const int w = (int)((m.sptr[s + 1] - base) / kWave);
  double a = 0.0;
  for (int k = 0; k < w; ++k) {
    const int64_t e = base + (int64_t)k * kWave + lane;
    a += m.val64[e] * x[m.col[e]];
  }
  out[entity[row]] = (m.mass64[row] + c * m.kdiag64[row]) * x[row] + c * a;
}

// ------------------------------------------------------------- host driver
namespace {

template <typename T>
ifl_status dalloc(T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(IFL_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  return IFL_OK;
}

template <typename T>
ifl_status upload(T** p, const std::vector<T>& v) {
  ifl_status st = dalloc(p, v.size());
  if (st != IFL_OK) return st;
  if (!v.empty()) IFL_HIP(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return IFL_OK;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

Mat mat_view(const DevMatrix& m) {
  return Mat{m.n, m.n_slices, m.sptr, m.col, m.val64, m.val32, m.kdiag64, m.kdiag32, m.mass64};
}

hipStream_t stream_of(Handle* h) {
  return h->opt.stream ? (hipStream_t)h->opt.stream : h->dev->own_stream;
}

}  // namespace

// Address of 'scratch' on each device, looked up once per device (with that
// device current) when the first handle on it is made.
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

static ifl_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(IFL_EDEVICE, "device ordinal beyond the library's table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[device]) return IFL_OK;
  void* p = nullptr;
  IFL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return fail(IFL_EDEVICE, "hipGetSymbolAddress returned NULL for the no-allocation work space");
  g_scratch_addr[device] = p;
  return IFL_OK;
}

static void* noalloc_scratch_addr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_addr[device];
}

// Entries per row the gathering kernels load together: the smallest class
// (6, 12, 20) that covers 90% of the slices.
static int head_class(const SellPack& sp) {
  std::vector<int64_t> widths((size_t)sp.n_slices);
  for (int64_t s = 0; s < sp.n_slices; ++s) widths[(size_t)s] = (sp.slice_ptr[s + 1] - sp.slice_ptr[s]) / kWave;
  int64_t w90 = 0;
  if (!widths.empty()) {
    const size_t at = (widths.size() * 9) / 10;
    std::nth_element(widths.begin(), widths.begin() + at, widths.end());
    w90 = widths[at];
  }
  return w90 <= 6 ? 6 : (w90 <= 12 ? 12 : 20);
}

ifl_status device_create(Handle* h) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(IFL_EDEVICE, "no HIP device available");
  }
  if (h->opt.device < 0 || h->opt.device >= ndev) return fail(IFL_EDEVICE, "device ordinal out of range");
  IFL_HIP(hipSetDevice(h->opt.device));
  hipDeviceProp_t prop;
  IFL_HIP(hipGetDeviceProperties(&prop, h->opt.device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(IFL_EDEVICE, std::string("library is built for gfx950, device is ") + prop.gcnArchName);
  DeviceState* d = new DeviceState();
  h->dev = d;
  d->device = h->opt.device;
  d->order = h->op.order;
  IFL_HIP(hipStreamCreateWithFlags(&d->own_stream, hipStreamNonBlocking));
  IFL_HIP(hipEventCreateWithFlags(&d->done_ev[0], hipEventDisableTiming));
  IFL_HIP(hipEventCreateWithFlags(&d->done_ev[1], hipEventDisableTiming));
  if (ifl_status e = noalloc_scratch_init(d->device); e != IFL_OK) return e;

  SellPack sp;
  pack_sell(h->op, &sp);
  DevMatrix& m = d->m;
  m.n = sp.n;
  m.n_slices = sp.n_slices;
  m.n_pad = sp.n_slices * kWave;
  m.nnz_stored = sp.slice_ptr.back();  // without the zero tail
  m.offdiag = sp.stored_offdiag;
  std::vector<float> v32(sp.val.begin(), sp.val.end());
  std::vector<float> kd32(sp.diag.begin(), sp.diag.end());
  ifl_status st;
  if ((st = upload(&m.sptr, sp.slice_ptr)) || (st = upload(&m.col, sp.col)) || (st = upload(&m.val64, sp.val)) ||
      (st = upload(&m.val32, v32)) || (st = upload(&m.kdiag64, sp.diag)) || (st = upload(&m.kdiag32, kd32)) ||
      (st = upload(&m.mass64, sp.mass)) || (st = upload(&m.entity, h->op.entity)))
    return st;
  {
    std::vector<int32_t> row_of((size_t)h->op.field_len, -1);
    for (int64_t i = 0; i < (int64_t)h->op.entity.size(); ++i) row_of[(size_t)h->op.entity[i]] = (int32_t)i;
    m.field_len = h->op.field_len;
    if ((st = upload(&m.row_of, row_of))) return st;
  }
  m.mass_sum = 0.0;
  for (double a : h->op.mass) m.mass_sum += a;
  // the batched kernels' pipelined head: the smallest class (6, 12, 20
  // entries) that covers 90% of the slices; wider slices finish their rows
  // unpipelined
  m.head = head_class(sp);
  if (const char* e = std::getenv("IFL_HEAD")) {
    const int v = std::atoi(e);
    if (v == 6 || v == 12 || v == 20) m.head = v;
  }
  // two-component operators with wide rows: 2 x 2 blocks for the batched
  // gathering kernels, a head of 6 blocks (wider rows finish in unpipelined
  // steps of 6; a head of 12 blocks would spill registers). Measured on the
  // level-8 sphere: the vertex vectors (6 neighbour blocks a block row)
  // iterate 3-4% faster in blocks than in rows; the cell vectors (3
  // neighbour blocks) 2-5% slower, so operators whose rows hold at most 3
  // blocks in 90% of the slices keep the row kernels.
  {
    PairPack pp;
    if (pack_pairs(h->op, &pp)) {
      std::vector<int64_t> widths((size_t)pp.n_slices);
      for (int64_t q = 0; q < pp.n_slices; ++q) widths[(size_t)q] = (pp.slice_ptr[q + 1] - pp.slice_ptr[q]) / kWave;
      int64_t w90 = 0;
      if (!widths.empty()) {
        const size_t at = (widths.size() * 9) / 10;
        std::nth_element(widths.begin(), widths.begin() + at, widths.end());
        w90 = widths[at];
      }
      if (w90 > 3) {
        m.nb = pp.nb;
        m.nb_slices = pp.n_slices;
        m.pnnz = pp.slice_ptr.back();
        m.phead = 6;
        std::vector<float> p32(pp.val.begin(), pp.val.end());
        if ((st = upload(&m.psptr, pp.slice_ptr)) || (st = upload(&m.pcol, pp.col)) ||
            (st = upload(&m.pval64, pp.val)) || (st = upload(&m.pval32, p32)))
          return st;
      }
    }
  }
  // orders >= 2: the first-order operator for the shifted solves
  if (h->op.order >= 2 && !h->op.k1_col.empty()) {
    SellPack s1;
    pack_sell_csr(h->op.n, h->op.k1_row_ptr, h->op.k1_col, h->op.k1_val, h->op.mass, &s1);
    DevK1& k1 = d->k1;
    k1.nnz_stored = s1.slice_ptr.back();
    k1.head = head_class(s1);
    std::vector<float> w32(s1.val.begin(), s1.val.end());
    std::vector<float> kd1(s1.diag.begin(), s1.diag.end());
    if ((st = upload(&k1.sptr, s1.slice_ptr)) || (st = upload(&k1.col, s1.col)) || (st = upload(&k1.val64, s1.val)) ||
        (st = upload(&k1.val32, w32)) || (st = upload(&k1.kdiag64, s1.diag)) || (st = upload(&k1.kdiag32, kd1)))
      return st;
    // ||K M^-1||_2 <= ||K||_2 / min M, ||K||_2 <= the largest absolute row sum (K symmetric)
    double rowmax = 0.0, mmin = INFINITY;
    for (int64_t r = 0; r < h->op.n; ++r) {
      double a = 0.0;
      for (int64_t e = h->op.k1_row_ptr[r]; e < h->op.k1_row_ptr[r + 1]; ++e) a += std::fabs(h->op.k1_val[e]);
      rowmax = std::max(rowmax, a);
      if (h->op.mass[r] > 0.0) mmin = std::min(mmin, h->op.mass[r]);
    }
    d->k1_gnorm = std::isfinite(mmin) ? rowmax / mmin : 0.0;
  }

  // launch geometry: logical blocks own contiguous slice ranges
  const int64_t ns = m.n_slices;
  int max_blocks = kMaxBlocks;
  if (const char* e = std::getenv("IFL_MAX_BLOCKS")) max_blocks = std::max(8, std::min(4096, std::atoi(e)));
  int G = (int)std::min<int64_t>(max_blocks, (ns + kWavesPerBlock - 1) / kWavesPerBlock);
  if (G >= kXcd) G = (G / kXcd) * kXcd;
  d->G = std::max(1, G);
  d->spb = (int)((ns + d->G - 1) / d->G);

  ColWork& w = d->w;
  const size_t np = (size_t)m.n_pad;
  for (double** v : {&w.x[0], &w.x[1], &w.z[0], &w.z[1], &w.u[0], &w.u[1], &w.p[0], &w.p[1], &w.d, &w.phi})
    if ((st = dalloc(v, np))) return st;
  for (float** v : {&w.z32[0], &w.z32[1], &w.u32[0], &w.u32[1], &w.p32[0], &w.p32[1], &w.d32})
    if ((st = dalloc(v, np))) return st;
  if ((st = dalloc(&w.part, (size_t)P_COUNT * d->G)) || (st = dalloc(&w.sc, 2)) || (st = dalloc(&w.flag, 1)))
    return st;
  IFL_HIP(hipHostMalloc((void**)&w.sc_host, 2 * sizeof(Scalars), hipHostMallocDefault));
  IFL_HIP(hipMemset(w.part, 0, sizeof(double) * P_COUNT * d->G));
  IFL_HIP(hipMemset(w.sc, 0, 2 * sizeof(Scalars)));
  // hipMemset of device memory may return before it completes, and the
  // solves run on streams that do not wait for the null stream
  IFL_HIP(hipDeviceSynchronize());
  return IFL_OK;
}

void device_destroy(Handle* h) {
  DeviceState* d = h->dev;
  if (!d) return;
  (void)hipSetDevice(d->device);
  if (d->own_stream) (void)hipStreamSynchronize(d->own_stream);
  DevMatrix& m = d->m;
  const ColWork& w = d->w;
  void* pptrs[] = {m.psptr, m.pcol, m.pval64, m.pval32};
  for (void* p : pptrs)
    if (p) (void)hipFree(p);
  void* ptrs[] = {m.sptr,   m.col,    m.val64,  m.val32,  m.kdiag64, m.kdiag32, m.mass64,   m.entity,
                  m.row_of, w.x[0],   w.x[1],   w.z[0],   w.z[1],    w.u[0],    w.u[1],     w.p[0],
                  w.p[1],   w.d,      w.z32[0], w.z32[1], w.u32[0],  w.u32[1],  w.p32[0],   w.p32[1],
                  w.d32,    w.phi,    w.part,   w.sc,     w.flag,    w.stage_in, w.stage_out};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (d->w.sc_host) (void)hipHostFree(d->w.sc_host);
  const DevK1& k1 = d->k1;
  const ShiftWork& sw = d->sw;
  void* sptrs[] = {k1.sptr,    k1.col,     k1.val64,   k1.val32,   k1.kdiag64, k1.kdiag32, sw.x[0],  sw.x[1],
                   sw.z64[0],  sw.z64[1],  sw.u64[0],  sw.u64[1],  sw.p64[0],  sw.p64[1],  sw.d64,   sw.z32[0],
                   sw.z32[1],  sw.u32[0],  sw.u32[1],  sw.p32[0],  sw.p32[1],  sw.d32,     sw.acc,   sw.part,
                   sw.sc};
  for (void* p : sptrs)
    if (p) (void)hipFree(p);
  if (sw.sc_host) (void)hipHostFree(sw.sc_host);
  batch_free(&d->bw);
  batch_free(&d->bwc);
  if (d->zero_rows) (void)hipFree(d->zero_rows);
  for (BatchWork& t : d->spare) batch_free(&t);
  if (d->field_stage) (void)hipFree(d->field_stage);
  if (d->field_rows) (void)hipFree(d->field_rows);
  if (d->col_stage) (void)hipFree(d->col_stage);
  void* proj[] = {d->proj_ptr, d->proj_tri, d->proj_w, d->proj_in};
  for (void* p : proj)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : d->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : d->done_ev)
    if (e) (void)hipEventDestroy(e);
  if (d->own_stream) (void)hipStreamDestroy(d->own_stream);
  delete d;
  h->dev = nullptr;
}

namespace {

ifl_status ensure_stage(DeviceState* d, int64_t len) {
  if (d->w.stage_len >= len) return IFL_OK;
  if (d->w.stage_in) (void)hipFree(d->w.stage_in);
  if (d->w.stage_out) (void)hipFree(d->w.stage_out);
  d->w.stage_in = d->w.stage_out = nullptr;
  d->w.stage_len = 0;
  ifl_status st;
  if ((st = dalloc(&d->w.stage_in, (size_t)len)) || (st = dalloc(&d->w.stage_out, (size_t)len))) return st;
  d->w.stage_len = len;
  return IFL_OK;
}

ifl_status ensure_events(DeviceState* d, size_t count) {
  while (d->ev.size() < count) {
    hipEvent_t e;
    IFL_HIP(hipEventCreate(&e));
    d->ev.push_back(e);
  }
  return IFL_OK;
}

// Bring one field (caller numbering, host or device) into w.phi (internal
// order); IFL_EINVAL on a non-finite wet entry.
ifl_status load_field(Handle* h, const double* field, bool dev_ptr, hipStream_t s) {
  DeviceState* d = h->dev;
  const int64_t L = h->op.field_len;
  const double* src = field;
  if (!dev_ptr) {
    IFL_HIP(hipMemcpyAsync(d->w.stage_in, field, sizeof(double) * L, hipMemcpyHostToDevice, s));
    src = d->w.stage_in;
  }
  IFL_HIP(hipMemsetAsync(d->w.flag, 0, sizeof(int), s));
  const int64_t n = d->m.n;
  k_gather_field<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, d->m.entity, n, d->w.phi, d->w.flag);
  IFL_HIP(hipGetLastError());
  int flag = 0;
  IFL_HIP(hipMemcpyAsync(&flag, d->w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  IFL_HIP(hipStreamSynchronize(s));
  if (flag) return fail(IFL_EINVAL, "field has a NaN or Inf at a wet entry");
  return IFL_OK;
}

// Algorithmic bytes of one iterating k_cg launch: the sliced-ELL stream
// (index + value per stored entry, slice pointers), the reads of z, u, p
// and d and the writes of z, u and p (each vector once), and the FP64
// solution read and written.
double spmv_bytes(const DevMatrix& m, size_t vb) {
  return (double)m.nnz_stored * (4.0 + vb) + 8.0 * (m.n_slices + 1) + (double)m.n * (vb * 7.0 + 16.0);
}

// Partials and scalars of a one-column solve: the handle's own, or the
// no-allocation work space.
struct ColScratch {
  double* part;
  Scalars* sc;  // two copies
  bool allow_profile;  // the handle's profiling events may be made and used
  bool allow_shifted;  // the shifted solves (their own work space) may run
};

template <typename T, bool MIXED, int U>
void launch_cg(const Mat& m, const CgVecs<T>& v, const double* phi, const ColScratch& cs, int launch, int G, int spb,
               int max_iter, hipStream_t s) {
  k_cg<T, MIXED, U><<<G, kBlock, 0, s>>>(m, v, phi, cs.part, cs.sc, launch, G, spb, max_iter);
}

// Zero n doubles (a fill kernel rather than a memset node, so that the calls
// that use it can also be captured)
__global__ void k_fill_zero(double* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Result of the CG loop of one column.
struct ColRun {
  Scalars last;          // host copy of the final state
  int64_t launched = 0;  // launches made
  double secs = 0.0;
};

// Jacobi-PCG on (M + c K) x = M phi (w.phi) from x0 = phi, K in m (K_n, or
// the first-order operator of a shifted solve): start, then launches in
// chunks of 8 until a launch stops; the solution is left in w.x[buffer of
// the final state] (see k_finish).
template <typename T, bool MIXED>
ifl_status run_column(Handle* h, const Mat& m, int head, double c, const ColScratch& cs, bool prof_ok,
                      ColRun* res) {
  DeviceState* d = h->dev;
  ColWork& w = d->w;
  const DevMatrix& M = d->m;
  hipStream_t s = stream_of(h);
  CgVecs<T> v;
  if constexpr (MIXED) {
    v = CgVecs<T>{{w.z32[0], w.z32[1]}, {w.u32[0], w.u32[1]}, {w.p32[0], w.p32[1]}, w.d32, {w.x[0], w.x[1]}};
  } else {
    v = CgVecs<T>{{w.z[0], w.z[1]}, {w.u[0], w.u[1]}, {w.p[0], w.p[1]}, w.d, {w.x[0], w.x[1]}};
  }
  const int G = d->G, spb = d->spb;
  const auto t0 = std::chrono::steady_clock::now();
  k_init<T><<<G, kBlock, 0, s>>>(m, v, w.phi, cs.part, cs.sc, c, G, spb);
  k_setup<<<1, kBlock, 0, s>>>(cs.part, cs.sc, h->opt.rtol, G);
  IFL_HIP(hipGetLastError());

  const int chunk = 8;  // launches between host checks
  const bool prof = h->opt.profile != 0 && cs.allow_profile && prof_ok;
  const int max_iter = h->opt.max_iter;
  // at most max_iter iterating launches, each followed by at most one
  // replacement, and the stopping launch: the cap ends the loop in any case
  const int64_t max_launch = 2 * (int64_t)max_iter + 16;
  void (*cg)(const Mat&, const CgVecs<T>&, const double*, const ColScratch&, int, int, int, int, hipStream_t) =
      head <= 6 ? launch_cg<T, MIXED, 6> : (head <= 12 ? launch_cg<T, MIXED, 12> : launch_cg<T, MIXED, 20>);
  int64_t launched = 0;
  int chunk_id = 0;
  bool finished = false;
  int pending = -1;  // chunk whose scalars are in flight
  int64_t prof_launch[2] = {-1, -1};
  if (prof) {
    ifl_status e = ensure_events(d, 4);
    if (e != IFL_OK) return e;
  }
  hipEvent_t* done_ev = d->done_ev;
  while (!finished) {
    const int slot = chunk_id & 1;
    // profiling samples one launch per chunk (bracketing every launch with
    // events would itself slow the loop down)
    const int pos = chunk_id % chunk;
    prof_launch[slot] = -1;
    for (int j = 0; j < chunk && launched < max_launch; ++j) {
      const bool sample = prof && j == pos;
      if (sample) IFL_HIP(hipEventRecord(d->ev[2 * slot], s));
      cg(m, v, w.phi, cs, (int)launched, G, spb, max_iter, s);
      if (sample) {
        IFL_HIP(hipEventRecord(d->ev[2 * slot + 1], s));
        prof_launch[slot] = launched;
      }
      ++launched;
    }
    IFL_HIP(hipGetLastError());
    // the state copy the next launch would read
    IFL_HIP(hipMemcpyAsync(&w.sc_host[slot], cs.sc + (launched & 1), sizeof(Scalars), hipMemcpyDeviceToHost, s));
    IFL_HIP(hipEventRecord(done_ev[slot], s));
    const bool capped = launched >= max_launch;
    // wait for the previous chunk (the current one keeps the GPU busy)
    int wait_chunk = capped ? chunk_id : pending;
    if (wait_chunk >= 0) {
      const int ws = wait_chunk & 1;
      IFL_HIP(hipEventSynchronize(done_ev[ws]));
      const Scalars& sh = w.sc_host[ws];
      // count the sample only if that launch iterated with a step (the
      // fused form the byte count describes)
      if (prof && prof_launch[ws] >= 0 && ((sh.fused_bits >> (prof_launch[ws] & 31)) & 1u)) {
        float ms = 0.f;
        IFL_HIP(hipEventElapsedTime(&ms, d->ev[2 * ws], d->ev[2 * ws + 1]));
        d->prof_ms += ms;
        d->prof_launches += 1;
        d->prof_bytes += spmv_bytes(M, sizeof(T));
        d->prof_kernel = std::string("k_cg<") + (MIXED ? "float, true, " : "double, false, ") +
                         std::to_string(head <= 6 ? 6 : (head <= 12 ? 12 : 20)) + ">";
      }
      if (sh.done) finished = true;
    }
    if (capped) finished = true;
    pending = chunk_id;
    ++chunk_id;
  }
  IFL_HIP(hipMemcpyAsync(&w.sc_host[0], cs.sc + (launched & 1), sizeof(Scalars), hipMemcpyDeviceToHost, s));
  IFL_HIP(hipStreamSynchronize(s));
  res->last = w.sc_host[0];
  res->launched = launched;
  res->secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return IFL_OK;
}

template <typename T, bool MIXED>
ifl_status solve_column(Handle* h, double k, ifl_solve_stats* st_out, double* out_dev, double* energy,
                        const ColScratch& cs) {
  DeviceState* d = h->dev;
  ColWork& w = d->w;
  const DevMatrix& M = d->m;
  hipStream_t s = stream_of(h);
  const Mat m = mat_view(M);
  const int G = d->G, spb = d->spb;
  const double c = h->opt.gamma / std::pow(k, 2.0 * h->op.order);
  ColRun run;
  ifl_status st = run_column<T, MIXED>(h, m, M.head, c, cs, true, &run);
  if (st != IFL_OK) return st;
  const int64_t launched = run.launched;
  // finish: x to caller numbering, true residual, energy (from the final
  // state copy; a solve cut off by the launch cap uses the last x written)
  Scalars* fin = cs.sc + (launched & 1);
  k_finish<<<G, kBlock, 0, s>>>(m, w.x[0], w.x[1], w.phi, M.entity, out_dev, cs.part, fin, (int)(launched & 1), G,
                                spb);
  k_finish_scalars<<<1, kBlock, 0, s>>>(cs.part, fin, G);
  IFL_HIP(hipGetLastError());
  IFL_HIP(hipMemcpyAsync(&w.sc_host[0], fin, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  IFL_HIP(hipStreamSynchronize(s));
  const Scalars& sh = w.sc_host[0];
  const double rel = sh.bb > 0 ? std::sqrt(sh.res2 / sh.bb) : std::sqrt(sh.res2);
  const bool ok = sh.done == 1;
  if (st_out) {
    st_out->iterations = sh.iters;
    st_out->refinements = sh.updates;
    st_out->status = ok ? IFL_OK : IFL_ENOTCONV;
    st_out->reserved = 0;
    st_out->rel_residual = rel;
    st_out->seconds = run.secs;
    st_out->energy = 0.5 * sh.energy2 / M.mass_sum;
  }
  if (energy) *energy = 0.5 * sh.energy2 / M.mass_sum;
  if (!ok)
    return fail(IFL_ENOTCONV, sh.done == 2 ? "CG breakdown ((p, Sp) <= 0 or non-finite)"
                                           : "CG reached max_iter before the tolerance");
  return IFL_OK;
}

// The shifted solves' work space, made on first use.
ifl_status ensure_shift_work(DeviceState* d) {
  ShiftWork& sw = d->sw;
  if (sw.acc) return IFL_OK;
  const size_t np = (size_t)d->m.n_pad;
  ifl_status st;
  for (double** v : {&sw.x[0], &sw.x[1], &sw.z64[0], &sw.z64[1], &sw.u64[0], &sw.u64[1], &sw.p64[0], &sw.p64[1],
                     &sw.d64})
    if ((st = dalloc(v, 2 * np))) return st;
  for (float** v : {&sw.z32[0], &sw.z32[1], &sw.u32[0], &sw.u32[1], &sw.p32[0], &sw.p32[1], &sw.d32})
    if ((st = dalloc(v, 2 * np))) return st;
  if ((st = dalloc(&sw.part, (size_t)CP_COUNT * d->G)) || (st = dalloc(&sw.sc, 2)) || (st = dalloc(&sw.acc, np)))
    return st;
  IFL_HIP(hipHostMalloc((void**)&sw.sc_host, 2 * sizeof(CScalars), hipHostMallocDefault));
  IFL_HIP(hipMemset(sw.part, 0, sizeof(double) * CP_COUNT * d->G));
  IFL_HIP(hipMemset(sw.sc, 0, 2 * sizeof(CScalars)));
  IFL_HIP(hipDeviceSynchronize());
  return IFL_OK;
}

template <typename T, bool MIXED, int U>
void launch_ccg(const Mat& m, const CVecs<T>& v, const double* phi, double* part, CScalars* sc, int launch, int G,
                int spb, int max_iter, hipStream_t s) {
  k_ccg<T, MIXED, U><<<G, kBlock, 0, s>>>(m, v, phi, part, sc, launch, G, spb, max_iter);
}

// Jacobi-COCG on (M + sigma K) y = M phi (w.phi) from y0 = phi, K the
// first-order operator; the solution is left in sw.x[buffer of the final
// state].
template <typename T, bool MIXED>
ifl_status run_ccolumn(Handle* h, const Mat& m, int head, double sr, double si, CScalars* last, int64_t* launched_out) {
  DeviceState* d = h->dev;
  ColWork& w = d->w;
  ShiftWork& sw = d->sw;
  hipStream_t s = stream_of(h);
  CVecs<T> v;
  if constexpr (MIXED) {
    v = CVecs<T>{{sw.z32[0], sw.z32[1]}, {sw.u32[0], sw.u32[1]}, {sw.p32[0], sw.p32[1]}, sw.d32, {sw.x[0], sw.x[1]}};
  } else {
    v = CVecs<T>{{sw.z64[0], sw.z64[1]}, {sw.u64[0], sw.u64[1]}, {sw.p64[0], sw.p64[1]}, sw.d64, {sw.x[0], sw.x[1]}};
  }
  const int G = d->G, spb = d->spb;
  k_cinit<T><<<G, kBlock, 0, s>>>(m, v, w.phi, sw.part, sw.sc, sr, si, G, spb);
  // each shifted system stops at rtol on its own FP64 true residual (the
  // complex tiles use a tighter target with a stall rule; here COCG pushed
  // to that target wandered off at C2's 6.4h scale)
  k_csetup<<<1, kBlock, 0, s>>>(sw.part, sw.sc, h->opt.rtol, G);
  IFL_HIP(hipGetLastError());
  const int chunk = 8;
  const int max_iter = h->opt.max_iter;
  const int64_t max_launch = 2 * (int64_t)max_iter + 16;
  void (*cg)(const Mat&, const CVecs<T>&, const double*, double*, CScalars*, int, int, int, int, hipStream_t) =
      head <= 6 ? launch_ccg<T, MIXED, 6> : (head <= 12 ? launch_ccg<T, MIXED, 12> : launch_ccg<T, MIXED, 20>);
  int64_t launched = 0;
  int chunk_id = 0, pending = -1;
  bool finished = false;
  hipEvent_t* done_ev = d->done_ev;
  while (!finished) {
    const int slot = chunk_id & 1;
    for (int j = 0; j < chunk && launched < max_launch; ++j) {
      cg(m, v, w.phi, sw.part, sw.sc, (int)launched, G, spb, max_iter, s);
      ++launched;
    }
    IFL_HIP(hipGetLastError());
    IFL_HIP(hipMemcpyAsync(&sw.sc_host[slot], sw.sc + (launched & 1), sizeof(CScalars), hipMemcpyDeviceToHost, s));
    IFL_HIP(hipEventRecord(done_ev[slot], s));
    const bool capped = launched >= max_launch;
    const int wait_chunk = capped ? chunk_id : pending;
    if (wait_chunk >= 0) {
      IFL_HIP(hipEventSynchronize(done_ev[wait_chunk & 1]));
      if (sw.sc_host[wait_chunk & 1].done) finished = true;
    }
    if (capped) finished = true;
    pending = chunk_id;
    ++chunk_id;
  }
  IFL_HIP(hipMemcpyAsync(&sw.sc_host[0], sw.sc + (launched & 1), sizeof(CScalars), hipMemcpyDeviceToHost, s));
  IFL_HIP(hipStreamSynchronize(s));
  *last = sw.sc_host[0];
  *launched_out = launched;
  return IFL_OK;
}

// S^-1 M phi for an order n >= 2 through first-order systems only (the
// partial fractions of 1 / (1 + y^n), y the eigenvalues of c^(1/n) M^-1 K):
// x = (1/n) sum_j (M + s_j b K)^-1 M phi, b = c^(1/n), s_j = -1 / w_j over
// the roots of w^n = -1. A real shift (s = 1, odd n) is solved by the real
// CG on K, each conjugate pair of complex shifts by one COCG solve whose
// real part counts twice. Every shifted solve stops on its own FP64 true
// residual; the stats report the FP64 true residual of S itself.
template <typename T, bool MIXED>
ifl_status solve_shifted(Handle* h, double k, ifl_solve_stats* st_out, double* out_dev, double* energy) {
  DeviceState* d = h->dev;
  ColWork& w = d->w;
  const DevMatrix& M = d->m;
  const DevK1& K1 = d->k1;
  hipStream_t s = stream_of(h);
  if (!K1.sptr) return fail(IFL_EINVAL, "handle has no first-order operator (order 1, or an old saved file)");
  ifl_status st = ensure_shift_work(d);
  if (st != IFL_OK) return st;
  const int n = h->op.order;
  const int G = d->G, spb = d->spb;
  const double c = h->opt.gamma / std::pow(k, 2.0 * n);
  const double b = std::pow(c, 1.0 / n);
  const Mat m1{M.n, M.n_slices, K1.sptr, K1.col, K1.val64, K1.val32, K1.kdiag64, K1.kdiag32, M.mass64};
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t nz = M.n_pad;
  k_fill_zero<<<(unsigned)((nz + 255) / 256), 256, 0, s>>>(d->sw.acc, nz);
  int iters = 0, updates = 0;
  int bad = 0;  // 0 ok, else the done code of a failed shifted solve
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < n; ++j) {
    // s_j = -1 / w_j, w_j = exp(i pi (2j + 1) / n); the conjugate of
    // s_{n-1-j}: solve the shifts with Im s >= 0 (j >= n/2 ... by symmetry)
    const double th = pi * (2 * j + 1) / n;
    const double sr = -std::cos(th), si = std::sin(th);  // -1/w = -conj(w) for |w| = 1
    if (si < -1e-12) continue;
    if (std::fabs(si) <= 1e-12) {
      ColRun run;
      const ColScratch cs{w.part, w.sc, false, false};
      if ((st = run_column<T, MIXED>(h, m1, K1.head, sr * b, cs, false, &run)) != IFL_OK) return st;
      iters += run.last.iters;
      updates += run.last.updates;
      if (run.last.done != 1) bad = run.last.done ? run.last.done : 3;
      const int xb = run.last.done ? run.last.xbuf : (int)(run.launched & 1);
      k_accumulate<<<(unsigned)((M.n + 255) / 256), 256, 0, s>>>(d->sw.acc, w.x[xb], 1, 1.0 / n, M.n);
    } else {
      CScalars last;
      int64_t launched = 0;
      if ((st = run_ccolumn<T, MIXED>(h, m1, K1.head, sr * b, si * b, &last, &launched)) != IFL_OK) return st;
      iters += last.iters;
      updates += last.updates;
      if (last.done != 1) bad = last.done ? last.done : 3;
      const int xb = last.done ? last.xbuf : (int)(launched & 1);
      k_accumulate<<<(unsigned)((M.n + 255) / 256), 256, 0, s>>>(d->sw.acc, d->sw.x[xb], 2, 2.0 / n, M.n);
    }
    IFL_HIP(hipGetLastError());
  }
  // the summed solution to the caller, the true residual of S itself
  const Mat mn = mat_view(M);
  k_sfinish<<<G, kBlock, 0, s>>>(mn, d->sw.acc, w.phi, c, M.entity, out_dev, d->sw.part, G, spb);
  IFL_HIP(hipGetLastError());
  // the finish sums and ||M phi||^2 of the complex starts (every order >= 2
  // has a complex shift; all shifts share the right-hand side), summed on
  // the host in a fixed order
  std::vector<double> part(4 * (size_t)G);
  IFL_HIP(hipMemcpyAsync(part.data(), d->sw.part + (size_t)CP_BB * G, sizeof(double) * 3 * G,
                         hipMemcpyDeviceToHost, s));
  IFL_HIP(hipStreamSynchronize(s));
  static_assert(CP_RES == CP_BB + 1 && CP_EN == CP_BB + 2, "finish sums follow ||M phi||^2");
  double bb = 0.0, res2 = 0.0, en = 0.0;
  for (int i = 0; i < G; ++i) bb += part[i];
  for (int i = 0; i < G; ++i) res2 += part[G + i];
  for (int i = 0; i < G; ++i) en += part[2 * G + i];
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st_out) {
    st_out->iterations = iters;
    st_out->refinements = updates;
    st_out->status = bad ? IFL_ENOTCONV : IFL_OK;
    st_out->reserved = 0;
    st_out->rel_residual = bb > 0 ? std::sqrt(res2 / bb) : std::sqrt(res2);
    st_out->seconds = secs;
    st_out->energy = 0.5 * en / M.mass_sum;
  }
  if (energy) *energy = 0.5 * en / M.mass_sum;
  if (bad)
    return fail(IFL_ENOTCONV, bad == 2 ? "shifted CG breakdown ((p, A p) = 0 or non-finite)"
                                       : "a shifted solve reached max_iter before the tolerance");
  return IFL_OK;
}

}  // namespace

namespace {

// One column at a time (the plain path, and single solves).
ifl_status filter_single(Handle* h, int32_t n_fields, const double* fields, int32_t n_scales, const double* k,
                         double* out, ifl_solve_stats* stats, double* energy, const ColScratch& cs) {
  DeviceState* d = h->dev;
  hipStream_t s = stream_of(h);
  const int64_t L = h->op.field_len;
  const bool fdev = is_device_ptr(fields);
  const bool odev = out ? is_device_ptr(out) : false;
  ifl_status st = IFL_OK;
  if (!fdev || (out && !odev)) {
    if ((st = ensure_stage(d, L)) != IFL_OK) return st;
  }
  ifl_status agg = IFL_OK;
  for (int32_t f = 0; f < n_fields; ++f) {
    st = load_field(h, fields + (int64_t)f * L, fdev, s);
    if (st != IFL_OK) return st;
    for (int32_t j = 0; j < n_scales; ++j) {
      double* dst = nullptr;
      if (out) {
        dst = odev ? out + ((int64_t)f * n_scales + j) * L : d->w.stage_out;
        IFL_HIP(hipMemsetAsync(dst, 0, sizeof(double) * L, s));
      }
      ifl_solve_stats* so = stats ? &stats[(int64_t)f * n_scales + j] : nullptr;
      double* eo = energy ? &energy[(int64_t)f * n_scales + j] : nullptr;
      const bool shifted = h->opt.solver == IFL_SOLVER_SHIFTED && h->op.order >= 2 && cs.allow_shifted;
      if (shifted && h->opt.precision == IFL_MIXED) st = solve_shifted<float, true>(h, k[j], so, dst, eo);
      else if (shifted) st = solve_shifted<double, false>(h, k[j], so, dst, eo);
      else if (h->opt.precision == IFL_MIXED) st = solve_column<float, true>(h, k[j], so, dst, eo, cs);
      else st = solve_column<double, false>(h, k[j], so, dst, eo, cs);
      if (st == IFL_ENOTCONV) agg = st;
      else if (st != IFL_OK) return st;
      if (out && !odev) {
        IFL_HIP(hipMemcpyAsync(out + ((int64_t)f * n_scales + j) * L, d->w.stage_out, sizeof(double) * L,
                               hipMemcpyDeviceToHost, s));
        IFL_HIP(hipStreamSynchronize(s));
      }
    }
  }
  if (agg != IFL_OK) return fail(agg, "at least one column did not converge (see stats)");
  return IFL_OK;
}

}  // namespace

// Clamp a grid size to the tile's task count and round it to the XCDs.
static int fit_grid(const DeviceState* d, int R, bool mixed, int g) {
  const int64_t tasks = d->m.n_slices * batch_lanes_per_row(R, mixed);
  const int64_t most = (tasks + kWavesPerBlock - 1) / kWavesPerBlock;
  g = (int)std::min<int64_t>(g, most);
  if (g >= kXcd) g = (g / kXcd) * kXcd;
  return std::max(1, g);
}

static int device_cus(int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) cus = 256;
  return cus;
}

BatchMatrix batch_matrix(DeviceState* d, int R, bool mixed) {
  BatchMatrix bm;
  const DevMatrix& m = d->m;
  bm.n = m.n;
  bm.n_slices = m.n_slices;
  bm.n_pad = m.n_pad;
  bm.sptr = m.sptr;
  bm.col = m.col;
  bm.val64 = m.val64;
  bm.val32 = m.val32;
  bm.kdiag = m.kdiag64;
  bm.mass = m.mass64;
  bm.entity = m.entity;
  bm.row_of = m.row_of;
  bm.field_len = m.field_len;
  bm.head = m.head;
  bm.chunk = chunk_for_order(d->order);
  if (m.psptr) {
    bm.pairs = true;
    bm.nb = m.nb;
    bm.nb_slices = m.nb_slices;
    bm.pnnz = m.pnnz;
    bm.psptr = m.psptr;
    bm.pcol = m.pcol;
    bm.pval64 = m.pval64;
    bm.pval32 = m.pval32;
    bm.head = m.phead;
  }
  // a task is one wavefront's rows: 64 / lanes-per-row consecutive rows.
  // Defaults: the gathering kernels run one block per CU, so that the rows
  // in flight on an XCD form a band narrow enough for its L2 to keep the
  // gathered neighbours; the complex tiles' x update runs all resident
  // blocks (the real tiles' x update is a one-pass launch). The autotuner
  // may have picked others for this tile size.
  int G = device_cus(d->device), Gu = batch_resident_blocks(R, mixed, d->device);
  for (const auto& t : d->tuned)
    if (t.R == R && t.mixed == mixed) {
      G = t.G;
      Gu = t.Gu;
    }
  G = fit_grid(d, R, mixed, G);
  bm.Gu = fit_grid(d, R, mixed, Gu);
  bm.G = std::max(1, G);
  return bm;
}

// The first-order operator K of an order >= 2 handle (same rows, mass and
// numbering as K_n) for the complex tiles of the shifted solves.
static BatchMatrix batch_matrix_k1(DeviceState* d, int R, bool mixed) {
  BatchMatrix bm = batch_matrix(d, R, mixed);
  const DevK1& k1 = d->k1;
  bm.sptr = k1.sptr;
  bm.col = k1.col;
  bm.val64 = k1.val64;
  bm.val32 = k1.val32;
  bm.kdiag = k1.kdiag64;
  bm.head = k1.head;
  bm.pairs = false;
  bm.psptr = nullptr;
  bm.pcol = nullptr;
  bm.pval64 = nullptr;
  bm.pval32 = nullptr;
  return bm;
}

BatchMatrix handle_batch_matrix(Handle* h, int R, bool mixed) { return batch_matrix(h->dev, R, mixed); }
BatchMatrix handle_batch_matrix_k1(Handle* h, int R, bool mixed) { return batch_matrix_k1(h->dev, R, mixed); }

double handle_cx_gnorm(const Handle* h) { return h->dev ? h->dev->k1_gnorm : 0.0; }

bool handle_cx_tiles(const Handle* h) {
  return h->opt.solver == IFL_SOLVER_SHIFTED && h->op.order == 2 && h->dev && h->dev->k1.sptr &&
         h->dev->k1.head <= 6;
}

// sigma = -b / w_0 for the shift pair with Im >= 0 (w_0 = exp(i pi / 2),
// b = c^(1/2), c = gamma / k^4), as the one-column shifted solves take it
void cx_shift(const Handle* h, double k, double* sigma_re, double* sigma_im) {
  const double pi = 3.14159265358979323846, th = pi / 2;
  const double b = std::sqrt(h->opt.gamma / std::pow(k, 4.0));
  *sigma_re = -std::cos(th) * b;
  *sigma_im = std::sin(th) * b;
}
double handle_mass_sum(const Handle* h) { return h->dev->m.mass_sum; }

namespace {

ifl_status ensure_batch(DeviceState* d, int R, bool mixed) {
  const BatchMatrix bm = batch_matrix(d, R, mixed);
  if (d->bw.R == R && d->bw.mixed == mixed && d->bw.G == bm.G && d->bw.Gu == bm.Gu && d->bw.slots) return IFL_OK;
  batch_free(&d->bw);
  return batch_alloc(&d->bw, bm, R, mixed);
}

// A cached narrower tile of width R (its slots all idle).
ifl_status spare_tile(DeviceState* d, int R, bool mixed, hipStream_t s, BatchWork** out) {
  const BatchMatrix bm = batch_matrix(d, R, mixed);
  for (BatchWork& t : d->spare)
    if (t.R == R && t.mixed == mixed) {
      if (t.G != bm.G || t.Gu != bm.Gu) {
        batch_free(&t);
        ifl_status st = batch_alloc(&t, bm, R, mixed);
        if (st != IFL_OK) return st;
      }
      *out = &t;
      return batch_release(t, ~0ull, s);
    }
  d->spare.emplace_back();
  BatchWork& t = d->spare.back();
  ifl_status st = batch_alloc(&t, bm, R, mixed);
  if (st != IFL_OK) {
    d->spare.pop_back();
    return st;
  }
  *out = &t;
  return batch_release(t, ~0ull, s);
}

// Many columns at once: slots of a tile of R columns are filled from the
// (field, scale) list, iterated together, and refilled as columns finish.
// A batched call's staging: the fields on the device, then in row order in
// d->field_rows (once per call; each is loaded once per scale) with the
// non-finite check of every wet entry (through w's flag), and host-output
// staging for out_cols columns.
ifl_status stage_call(Handle* h, const BatchMatrix& bm, BatchWork& w, int32_t n_fields, const double* fields,
                      int out_cols, hipStream_t s) {
  DeviceState* d = h->dev;
  const int64_t L = h->op.field_len;
  ifl_status st;
  const double* fdev = fields;
  if (!is_device_ptr(fields)) {
    const int64_t need = (int64_t)n_fields * L;
    if (d->field_stage_len < need) {
      if (d->field_stage) (void)hipFree(d->field_stage);
      d->field_stage = nullptr;
      d->field_stage_len = 0;
      if ((st = dalloc(&d->field_stage, (size_t)need)) != IFL_OK) return st;
      d->field_stage_len = need;
    }
    IFL_HIP(hipMemcpyAsync(d->field_stage, fields, sizeof(double) * need, hipMemcpyHostToDevice, s));
    fdev = d->field_stage;
  }
  if (out_cols > 0 && d->col_stage_len < (int64_t)out_cols * L) {
    if (d->col_stage) (void)hipFree(d->col_stage);
    d->col_stage = nullptr;
    d->col_stage_len = 0;
    if ((st = dalloc(&d->col_stage, (size_t)out_cols * L)) != IFL_OK) return st;
    d->col_stage_len = (int64_t)out_cols * L;
  }
  const int64_t need = (int64_t)n_fields * bm.n_pad;
  if (d->field_rows_len < need) {
    if (d->field_rows) (void)hipFree(d->field_rows);
    d->field_rows = nullptr;
    d->field_rows_len = 0;
    if ((st = dalloc(&d->field_rows, (size_t)need)) != IFL_OK) return st;
    d->field_rows_len = need;
  }
  bool bad = false;
  if ((st = batch_clear_flag(w, s)) != IFL_OK) return st;
  if ((st = batch_permute_fields(bm, fdev, L, n_fields, d->field_rows, w.flag, s)) != IFL_OK) return st;
  if ((st = batch_check_flag(w, s, &bad)) != IFL_OK) return st;
  if (bad) return fail(IFL_EINVAL, "field has a NaN or Inf at a wet entry");
  return IFL_OK;
}

ifl_status filter_batched(Handle* h, int R, int32_t n_fields, const double* fields, int32_t n_scales,
                          const double* k, double* out, ifl_solve_stats* stats, double* energy) {
  DeviceState* d = h->dev;
  hipStream_t s = stream_of(h);
  const int64_t L = h->op.field_len;
  const bool mixed = h->opt.precision == IFL_MIXED;
  ifl_status st = ensure_batch(d, R, mixed);
  if (st != IFL_OK) return st;
  BatchWork* wp = &d->bw;
  BatchMatrix bm = batch_matrix(d, R, mixed);
  const int R0 = R;
  // slots left active by an earlier call that stopped on an error
  if ((st = batch_release(*wp, ~0ull, s)) != IFL_OK) return st;
  const bool odev = out ? is_device_ptr(out) : false;
  if ((st = stage_call(h, bm, *wp, n_fields, fields, out && !odev ? R : 0, s)) != IFL_OK) return st;
  // columns: larger scales (more iterations) first, fields in order
  const int64_t ncols = (int64_t)n_fields * n_scales;
  std::vector<int64_t> order(ncols);
  for (int64_t i = 0; i < ncols; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return k[a % n_scales] < k[b % n_scales]; });
  BatchParams prm;
  prm.max_iter = h->opt.max_iter;
  prm.graphs = h->opt.graphs != 0;
  std::vector<int64_t> slot_col(R, -1);
  std::vector<std::chrono::steady_clock::time_point> t_in(R);
  int64_t next = 0, finished = 0;
  bool any_notconv = false;
  const int chunk = chunk_for_order(h->op.order);
  // with the tile width left to the library, the last columns of the call
  // move to narrower tiles as the others finish: a tile pays for all of its
  // slots every iteration
  const bool shrink = h->opt.batch == 0;
  while (finished < ncols) {
    BatchWork& w = *wp;
    // fill free slots
    uint64_t mask = 0;
    SlotScales cs{};
    const double* src[64] = {};
    for (int j = 0; j < R && next < ncols; ++j) {
      if (slot_col[j] >= 0) continue;
      const int64_t col = order[next++];
      const int64_t f = col / n_scales, sc = col % n_scales;
      src[j] = d->field_rows + f * bm.n_pad;
      cs.c[j] = h->opt.gamma / std::pow(k[sc], 2.0 * h->op.order);
      slot_col[j] = col;
      t_in[j] = std::chrono::steady_clock::now();
      mask |= 1ull << j;
    }
    if (mask) {
      if ((st = batch_load_columns(bm, w, mask, src, true, s)) != IFL_OK) return st;
      if ((st = batch_init(bm, w, mask, cs, h->opt.rtol, s)) != IFL_OK) return st;
    }
    BatchParams p = prm;
    int live = 0;
    if (h->opt.profile && R == R0) {  // the timed launches are those of the call's full-width tile
      if ((st = ensure_events(d, 2)) != IFL_OK) return st;
      p.ev_begin = d->ev[0];
      p.ev_end = d->ev[1];
      for (int j = 0; j < R; ++j)
        live += slot_col[j] >= 0 && (((mask >> j) & 1ull) || w.slots_host[j].done == 0);
    }
    if ((st = batch_iterate(bm, w, chunk, p, s)) != IFL_OK) return st;
    if ((st = batch_read_slots(w, s)) != IFL_OK) return st;
    if (h->opt.profile && R == R0 && live > 0) {
      float ms = 0.f;
      IFL_HIP(hipEventElapsedTime(&ms, d->ev[0], d->ev[1]));
      d->prof_ms += ms;
      d->prof_launches += 1;
      d->prof_bytes += batch_spmv_bytes(bm, d->m.nnz_stored, mixed, live);
      d->prof_kernel = std::string(bm.pairs ? "kb_iter2<" : "kb_iter<") + (mixed ? "float, " : "double, ") +
                       std::to_string(R) + ", true, " +
                       std::to_string(bm.head) + ">";
    }
    uint64_t fin = 0;
    std::vector<double*> dst(R, nullptr);
    for (int j = 0; j < R; ++j) {
      if (slot_col[j] < 0 || w.slots_host[j].done == 0) continue;
      fin |= 1ull << j;
      if (out) dst[j] = odev ? out + slot_col[j] * L : d->col_stage + (int64_t)j * L;
    }
    if (!fin) continue;
    if ((st = batch_finish(bm, w, fin, dst.data(), s)) != IFL_OK) return st;
    if ((st = batch_read_slots(w, s)) != IFL_OK) return st;
    const auto now = std::chrono::steady_clock::now();
    for (int j = 0; j < R; ++j) {
      if (!((fin >> j) & 1ull)) continue;
      const BSlot& sl = w.slots_host[j];
      const int64_t col = slot_col[j];
      const bool ok = sl.done == 1;
      any_notconv |= !ok;
      if (stats) {
        ifl_solve_stats& so = stats[col];
        so.iterations = sl.iters;
        so.refinements = sl.updates;
        so.status = ok ? IFL_OK : IFL_ENOTCONV;
        so.reserved = 0;
        so.rel_residual = sl.bb > 0 ? std::sqrt(sl.res2 / sl.bb) : std::sqrt(sl.res2);
        so.seconds = std::chrono::duration<double>(now - t_in[j]).count();
        so.energy = 0.5 * sl.energy2 / d->m.mass_sum;
      }
      if (energy) energy[col] = 0.5 * sl.energy2 / d->m.mass_sum;
      if (out && !odev)
        IFL_HIP(hipMemcpyAsync(out + col * L, dst[j], sizeof(double) * L, hipMemcpyDeviceToHost, s));
      slot_col[j] = -1;
      ++finished;
    }
    if ((st = batch_release(w, fin, s)) != IFL_OK) return st;
    // no column left to enter and at most a quarter of the slots running:
    // move the running columns to a tile of the next power of two >= their
    // count (at least 2); iteration state moves as it is at the boundary
    int running = 0;
    for (int j = 0; j < R; ++j) running += slot_col[j] >= 0;
    if (shrink && next >= ncols && running > 0 && R >= 4 && running * 4 <= R) {
      int R2 = 2;
      while (R2 < running) R2 *= 2;
      BatchWork* nw = nullptr;
      if ((st = spare_tile(d, R2, mixed, s, &nw)) != IFL_OK) return st;
      std::vector<int> from, to;
      std::vector<int64_t> col2(R2, -1);
      std::vector<std::chrono::steady_clock::time_point> t2(R2);
      for (int j = 0; j < R; ++j)
        if (slot_col[j] >= 0) {
          const int c = (int)from.size();
          from.push_back(j);
          to.push_back(c);
          col2[c] = slot_col[j];
          t2[c] = t_in[j];
        }
      const BatchMatrix bm2 = batch_matrix(d, R2, mixed);
      if ((st = batch_move_columns(bm2, w, *nw, from.data(), to.data(), running, s)) != IFL_OK) return st;
      if ((st = batch_release(w, ~0ull, s)) != IFL_OK) return st;
      if ((st = batch_read_slots(*nw, s)) != IFL_OK) return st;
      wp = nw;
      bm = bm2;
      R = R2;
      slot_col = col2;
      t_in = t2;
    }
  }
  IFL_HIP(hipStreamSynchronize(s));
  if (any_notconv) return fail(IFL_ENOTCONV, "at least one column did not converge (see stats)");
  return IFL_OK;
}

// Tile width: opt.batch >= 2 fixes R (rounded down to a power of two);
// auto (0) uses the autotuner's width (else 32), but at most a quarter of
// the columns (at least 2), and the single-column path for one column. A
// tile iterates until its slowest column is done, at the cost of a full
// tile per iteration; with few columns of very different iteration counts
// (many scales, n = 2) a narrower tile spends less on slots left idle.
int pick_tile(const Handle* h, int64_t ncols) {
  const int want = h->opt.batch;
  if (want == 1) return 1;
  int R = 1;
  if (want >= 2) {
    while (R * 2 <= want && R < 64) R *= 2;
    return R;
  }
  if (ncols <= 1) return 1;
  const int tuned = h->dev->tuned_R[h->opt.precision == IFL_MIXED ? 1 : 0];
  R = tuned > 0 ? tuned : 32;
  while (R > 2 && (int64_t)R * 4 > ncols) R /= 2;
  return R;
}

}  // namespace

// Order 2 with IFL_SOLVER_SHIFTED in tiles: S_2^-1 M phi is the real part of
// (M + sigma K)^-1 M phi, sigma = -b / w_0 (w_0 = exp(i pi / 2), b = c^(1/2)),
// one complex column per (field, scale) in a complex tile of 2 Rc real
// columns over the first-order operator (Jacobi-COCG, FP64 replacements at
// every chunk end, stop on the shifted system's FP64 true residual, as the
// one-column shifted solves). Columns enter at chunk boundaries, larger
// scales first; the tile keeps its width.
ifl_status filter_batched_cx(Handle* h, int Rc, int32_t n_fields, const double* fields, int32_t n_scales,
                             const double* k, double* out, ifl_solve_stats* stats, double* energy) {
  DeviceState* d = h->dev;
  hipStream_t s = stream_of(h);
  const int64_t L = h->op.field_len;
  const bool mixed = h->opt.precision == IFL_MIXED;
  const int R = 2 * Rc;
  ifl_status st;
  if (!d->k1.sptr) return fail(IFL_EINVAL, "handle has no first-order operator (an old saved file)");
  BatchMatrix bm = batch_matrix_k1(d, R, mixed);
  BatchWork& w = d->bwc;
  if (!w.slots || w.R != R || w.mixed != mixed || w.G != bm.G || w.Gu != bm.Gu) {
    batch_free(&w);
    w = BatchWork();
    if ((st = batch_alloc(&w, bm, R, mixed, true)) != IFL_OK) return st;
  }
  w.cx_g = d->k1_gnorm;
  if (!d->zero_rows) {
    if ((st = dalloc(&d->zero_rows, (size_t)bm.n_pad)) != IFL_OK) return st;
    k_fill_zero<<<(unsigned)((bm.n_pad + 255) / 256), 256, 0, s>>>(d->zero_rows, bm.n_pad);
    IFL_HIP(hipGetLastError());
  }
  if ((st = batch_release(w, ~0ull, s)) != IFL_OK) return st;
  const bool odev = out ? is_device_ptr(out) : false;
  if ((st = stage_call(h, bm, w, n_fields, fields, out && !odev ? R : 0, s)) != IFL_OK) return st;
  const int64_t ncols = (int64_t)n_fields * n_scales;
  std::vector<int64_t> order(ncols);
  for (int64_t i = 0; i < ncols; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return k[a % n_scales] < k[b % n_scales]; });
  BatchParams prm;
  prm.max_iter = h->opt.max_iter;
  prm.graphs = h->opt.graphs != 0;
  std::vector<int64_t> slot_col(Rc, -1);
  std::vector<std::chrono::steady_clock::time_point> t_in(Rc);
  int64_t next = 0, finished = 0;
  bool any_notconv = false;
  while (finished < ncols) {
    uint64_t mask = 0;
    SlotScales cs{};
    const double* src[64] = {};
    for (int q = 0; q < Rc && next < ncols; ++q) {
      if (slot_col[q] >= 0) continue;
      const int64_t col = order[next++];
      const int64_t f = col / n_scales, sc = col % n_scales;
      src[2 * q] = d->field_rows + f * bm.n_pad;
      src[2 * q + 1] = d->zero_rows;
      cx_shift(h, k[sc], &cs.c[2 * q], &cs.c[2 * q + 1]);
      slot_col[q] = col;
      t_in[q] = std::chrono::steady_clock::now();
      mask |= 3ull << (2 * q);
    }
    if (mask) {
      if ((st = batch_load_columns(bm, w, mask, src, true, s)) != IFL_OK) return st;
      if ((st = batch_init(bm, w, mask, cs, h->opt.rtol, s)) != IFL_OK) return st;
    }
    if ((st = batch_iterate(bm, w, w.chunk, prm, s)) != IFL_OK) return st;
    if ((st = batch_read_slots(w, s)) != IFL_OK) return st;
    uint64_t fin = 0;
    std::vector<double*> dst(R, nullptr);
    for (int q = 0; q < Rc; ++q) {
      if (slot_col[q] < 0 || w.slots_host[2 * q].done == 0) continue;
      fin |= 3ull << (2 * q);
      if (out) dst[2 * q] = odev ? out + slot_col[q] * L : d->col_stage + (int64_t)(2 * q) * L;
    }
    if (!fin) continue;
    if ((st = batch_finish(bm, w, fin, dst.data(), s)) != IFL_OK) return st;
    if ((st = batch_read_slots(w, s)) != IFL_OK) return st;
    const auto now = std::chrono::steady_clock::now();
    for (int q = 0; q < Rc; ++q) {
      if (!((fin >> (2 * q)) & 1ull)) continue;
      const BSlot& sl = w.slots_host[2 * q];
      const int64_t col = slot_col[q];
      const bool ok = sl.done == 1;
      any_notconv |= !ok;
      if (stats) {
        ifl_solve_stats& so = stats[col];
        so.iterations = sl.iters;
        so.refinements = sl.updates;
        so.status = ok ? IFL_OK : IFL_ENOTCONV;
        so.reserved = 0;
        so.rel_residual = sl.bb > 0 ? std::sqrt(sl.res2 / sl.bb) : std::sqrt(sl.res2);
        so.seconds = std::chrono::duration<double>(now - t_in[q]).count();
        so.energy = 0.5 * sl.energy2 / d->m.mass_sum;
      }
      if (energy) energy[col] = 0.5 * sl.energy2 / d->m.mass_sum;
      if (out && !odev)
        IFL_HIP(hipMemcpyAsync(out + col * L, dst[2 * q], sizeof(double) * L, hipMemcpyDeviceToHost, s));
      slot_col[q] = -1;
      ++finished;
    }
    if ((st = batch_release(w, fin, s)) != IFL_OK) return st;
  }
  IFL_HIP(hipStreamSynchronize(s));
  if (any_notconv) return fail(IFL_ENOTCONV, "a shifted solve did not converge within max_iter");
  return IFL_OK;
}

ifl_status device_filter(Handle* h, int32_t n_fields, const double* fields, int32_t n_scales, const double* k,
                         double* out, ifl_solve_stats* stats, double* energy) {
  DeviceState* d = h->dev;
  IFL_HIP(hipSetDevice(d->device));
  const bool shifted = h->opt.solver == IFL_SOLVER_SHIFTED && h->op.order >= 2;
  // order 2 (one complex shift) in complex tiles of first-order operators
  // with narrow rows; other orders, and batch = 1, one column at a time
  if (handle_cx_tiles(h) && h->opt.batch != 1) {
    const int64_t ncols = (int64_t)n_fields * n_scales;
    int Rc = 1;
    if (h->opt.batch >= 2) {
      Rc = std::min(32, std::max(1, h->opt.batch / 2));
    } else {
      while (Rc * 2 <= std::min<int64_t>(16, std::max<int64_t>(1, ncols / 2))) Rc *= 2;
    }
    int Rp = 1;  // tiles come in powers of two
    while (Rp * 2 <= Rc) Rp *= 2;
    return filter_batched_cx(h, Rp, n_fields, fields, n_scales, k, out, stats, energy);
  }
  const int R = shifted ? 1 : pick_tile(h, (int64_t)n_fields * n_scales);
  if (R <= 1) return filter_single(h, n_fields, fields, n_scales, k, out, stats, energy, ColScratch{d->w.part, d->w.sc, true, true});
  return filter_batched(h, R, n_fields, fields, n_scales, k, out, stats, energy);
}

// Streaming probe: dst = src in 16-byte units, one unit per thread and one
// pass (as many 256-thread workgroups as the copy needs). Measured on
// MI355X with 4 GiB buffers this moves 6.2 TB/s, where grid-stride loops
// over the resident workgroups (1, 2, 4 or 8 per CU, with or without four
// loads in flight per thread or non-temporal hints) move 4.6-5.3 TB/s.
constexpr int kCopyBlock = 256;
__global__ __launch_bounds__(kCopyBlock) void k_stream_copy(const int4* __restrict__ src, int4* __restrict__ dst,
                                                            int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kCopyBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

ifl_status device_stream_probe(int device, int64_t bytes, int reps, double* best_gbs, double* median_gbs) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return fail(IFL_EDEVICE, "no such HIP device");
  }
  IFL_HIP(hipSetDevice(device));
  const int64_t n = bytes / 16;
  int4 *a = nullptr, *b = nullptr;
  if (hipMalloc((void**)&a, n * 16) != hipSuccess || hipMalloc((void**)&b, n * 16) != hipSuccess) {
    if (a) (void)hipFree(a);
    (void)hipGetLastError();
    return fail(IFL_ENOMEM, "hipMalloc of the probe buffers failed");
  }
  const int64_t blocks = (n + kCopyBlock - 1) / kCopyBlock;
  if (blocks > INT32_MAX) {
    (void)hipFree(a);
    (void)hipFree(b);
    return fail(IFL_EINVAL, "copy probe larger than one launch covers");
  }
  const unsigned grid = (unsigned)blocks;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ifl_status st = IFL_OK;
  std::vector<double> rates;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(a, 0, n * 16, s) != hipSuccess) {
    st = fail(IFL_EDEVICE, "probe set-up failed");
  } else {
    k_stream_copy<<<grid, kCopyBlock, 0, s>>>(a, b, n);  // untimed
    for (int r = 0; r < reps && st == IFL_OK; ++r) {
      float ms = 0.f;
      if (hipEventRecord(e0, s) != hipSuccess) st = fail(IFL_EDEVICE, "hipEventRecord failed");
      k_stream_copy<<<grid, kCopyBlock, 0, s>>>(a, b, n);
      if (st == IFL_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(IFL_EDEVICE, "timing the probe failed");
      if (st == IFL_OK) rates.push_back(2.0 * 16.0 * (double)n / (ms * 1e-3) / 1e9);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  (void)hipFree(a);
  (void)hipFree(b);
  if (st != IFL_OK) return st;
  std::sort(rates.begin(), rates.end());
  *best_gbs = rates.back();
  *median_gbs = rates[rates.size() / 2];
  return IFL_OK;
}


ifl_status device_shift_work(Handle* h, size_t* bytes) {
  DeviceState* d = h->dev;
  IFL_HIP(hipSetDevice(d->device));
  const size_t np = (size_t)d->m.n_pad;
  // nine FP64 and seven FP32 complex vectors (two parts each), the weighted
  // sum, the partials and the scalars (ensure_shift_work)
  *bytes = 2 * np * (9 * sizeof(double) + 7 * sizeof(float)) + np * sizeof(double) +
           sizeof(double) * CP_COUNT * (size_t)d->G + 2 * sizeof(CScalars);
  return ensure_shift_work(d);
}

ifl_status device_solve_shifted_rows(Handle* h, const double* phi_rows, double k, double* out_dev,
                                     ifl_solve_stats* st) {
  DeviceState* d = h->dev;
  IFL_HIP(hipSetDevice(d->device));
  if (h->op.order < 2) return fail(IFL_EINVAL, "the shifted solves need an order n >= 2");
  hipStream_t s = stream_of(h);
  IFL_HIP(hipMemcpyAsync(d->w.phi, phi_rows, sizeof(double) * (size_t)d->m.n, hipMemcpyDeviceToDevice, s));
  // entries without a dof are 0 in the output (only the dofs are scattered)
  if (out_dev) k_fill_zero<<<(unsigned)((d->m.field_len + 255) / 256), 256, 0, s>>>(out_dev, d->m.field_len);
  if (h->opt.precision == IFL_MIXED) return solve_shifted<float, true>(h, k, st, out_dev, nullptr);
  return solve_shifted<double, false>(h, k, st, out_dev, nullptr);
}

ifl_status device_filter_noalloc(Handle* h, int32_t n_fields, const double* fields, int32_t n_scales,
                                 const double* k, double* out, ifl_solve_stats* stats) {
  DeviceState* d = h->dev;
  IFL_HIP(hipSetDevice(d->device));
  if (!is_device_ptr(fields) || !is_device_ptr(out))
    return fail(IFL_EINVAL, "ifl_filter_noalloc takes device fields and outputs only");
  const size_t need = sizeof(double) * (size_t)P_COUNT * (size_t)d->G;
  if (need > kNoallocScalarsOffset)
    return fail(IFL_EINVAL, "the handle's " + std::to_string(d->G) + " logical blocks need " + std::to_string(need) +
                                " bytes of partials; the no-allocation work space holds " +
                                std::to_string(kNoallocScalarsOffset));
  unsigned char* base = static_cast<unsigned char*>(noalloc_scratch_addr(d->device));
  if (!base) return fail(IFL_EDEVICE, "no-allocation work space not set up on this device");
  // the plain path only: the shifted solves allocate their work space
  const ColScratch cs{reinterpret_cast<double*>(base), reinterpret_cast<Scalars*>(base + kNoallocScalarsOffset),
                      false, false};
  hipStream_t s = stream_of(h);
  const int64_t nz = (int64_t)(kNoallocScratchBytes / sizeof(double));
  k_fill_zero<<<(unsigned)((nz + 255) / 256), 256, 0, s>>>(cs.part, nz);
  IFL_HIP(hipGetLastError());
  return filter_single(h, n_fields, fields, n_scales, k, out, stats, nullptr, cs);
}

// Autotuner of the batched engine: times 8 iterations (two replacement
// periods) of full tiles of pseudo-random columns for every tile size in
// {16, 32, 64} and grid sizes of the gathering kernels in {1/2, 1, 2} blocks
// per CU and of the update in {1, 2} blocks per CU, at a scale where the
// stiffness term dominates (the columns keep iterating), and keeps the
// fastest per column-iteration: per tile size for its grid sizes, overall
// for the default tile size of ifl_filter.
ifl_status device_autotune(Handle* h, ifl_tune* out) {
  DeviceState* d = h->dev;
  IFL_HIP(hipSetDevice(d->device));
  hipStream_t s = stream_of(h);
  const bool mixed = h->opt.precision == IFL_MIXED;
  ifl_status st = ensure_events(d, 2);
  if (st != IFL_OK) return st;
  double kd_sum = 0.0;
  for (int64_t r = 0; r < h->op.n; ++r)
    for (int64_t e = h->op.row_ptr[r]; e < h->op.row_ptr[r + 1]; ++e)
      if (h->op.col[e] == r) kd_sum += std::fabs(h->op.val[e]);
  const double c = 1e4 * d->m.mass_sum / std::max(kd_sum, 1e-300);
  const int cus = device_cus(d->device);
  batch_free(&d->bw);  // room for the trial tiles; the cached tiles are rebuilt on demand
  for (BatchWork& t : d->spare) batch_free(&t);
  d->spare.clear();
  struct Best {
    int R = 0, G = 0, Gu = 0;
    double us = 1e300;
  };
  Best overall;
  std::vector<Best> per_R;
  int tried = 0;
  for (int R : {16, 32, 64}) {
    Best b;
    std::vector<std::pair<int, int>> seen;
    // the update grid only sizes the complex tiles' x update (the real
    // tiles' x update is a one-pass launch): one value
    for (int gm : {1, 2, 4})
      for (int gu : {2}) {
        const int G = fit_grid(d, R, mixed, cus * gm / 2), Gu = fit_grid(d, R, mixed, cus * gu / 2);
        if (std::find(seen.begin(), seen.end(), std::make_pair(G, Gu)) != seen.end()) continue;
        seen.emplace_back(G, Gu);
        BatchMatrix bm = batch_matrix(d, R, mixed);
        bm.G = G;
        bm.Gu = Gu;
        BatchWork w;
        st = batch_alloc(&w, bm, R, mixed);
        SlotScales cs{};
        uint64_t mask = 0;
        for (int j = 0; j < R && st == IFL_OK; ++j) {
          st = batch_load_synthetic(bm, w, j, 0x5eed0000ull + (uint64_t)j, s);
          cs.c[j] = c;
          mask |= 1ull << j;
        }
        BatchParams prm;
        prm.max_iter = 1 << 30;
        prm.graphs = h->opt.graphs != 0;
        if (st == IFL_OK) st = batch_init(bm, w, mask, cs, 1e-300, s);
        if (st == IFL_OK) st = batch_iterate(bm, w, w.chunk, prm, s);  // warm-up
        float ms = 0.f;
        if (st == IFL_OK) {
          (void)hipEventRecord(d->ev[0], s);
          st = batch_iterate(bm, w, 2 * w.chunk, prm, s);
          (void)hipEventRecord(d->ev[1], s);
          if (hipEventSynchronize(d->ev[1]) != hipSuccess || hipEventElapsedTime(&ms, d->ev[0], d->ev[1]) != hipSuccess)
            st = fail(IFL_EDEVICE, "timing the autotuner trial failed");
        }
        batch_free(&w);
        if (st != IFL_OK) return st;
        ++tried;
        const double us = ms * 1e3 / (2.0 * w.chunk * R);
        if (us < b.us) b = Best{R, G, Gu, us};
      }
    per_R.push_back(b);
  }
  // the fastest tile size, preferring the smaller one within 5%: a smaller
  // tile wastes fewer slots when a call's columns run out (the trial tiles
  // are always full) and needs less memory
  for (const Best& b : per_R)
    if (b.us < overall.us * 0.95 || overall.R == 0) overall = b;
  for (const Best& b : per_R) {
    bool found = false;
    for (auto& t : d->tuned)
      if (t.R == b.R && t.mixed == mixed) {
        t.G = b.G;
        t.Gu = b.Gu;
        found = true;
      }
    if (!found) d->tuned.push_back(DeviceState::TunedGrid{b.R, mixed, b.G, b.Gu});
  }
  d->tuned_R[mixed ? 1 : 0] = overall.R;
  if (out) {
    out->batch = overall.R;
    out->blocks_gather = overall.G;
    out->blocks_update = overall.Gu;
    out->candidates = tried;
    out->us_per_column_iteration = overall.us;
  }
  return IFL_OK;
}

ifl_status device_apply(Handle* h, double kk, const double* x, double* y) {
  DeviceState* d = h->dev;
  IFL_HIP(hipSetDevice(d->device));
  hipStream_t s = stream_of(h);
  const int64_t L = h->op.field_len;
  ifl_status st = ensure_stage(d, L);
  if (st != IFL_OK) return st;
  st = load_field(h, x, is_device_ptr(x), s);
  if (st != IFL_OK) return st;
  const bool ydev = is_device_ptr(y);
  double* dst = ydev ? y : d->w.stage_out;
  IFL_HIP(hipMemsetAsync(dst, 0, sizeof(double) * L, s));
  const double c = h->opt.gamma / std::pow(kk, 2.0 * h->op.order);
  const unsigned nb = (unsigned)((d->m.n_slices + kWavesPerBlock - 1) / kWavesPerBlock);
  k_apply<<<nb, kBlock, 0, s>>>(mat_view(d->m), d->w.phi, c, d->m.entity, dst);
  IFL_HIP(hipGetLastError());
  if (!ydev) IFL_HIP(hipMemcpyAsync(y, dst, sizeof(double) * L, hipMemcpyDeviceToHost, s));
  IFL_HIP(hipStreamSynchronize(s));
  return IFL_OK;
}

ifl_status device_project_cells(Handle* h, const double* cells, double* out) {
  DeviceState* d = h->dev;
  const HostOperator& op = h->op;
  IFL_HIP(hipSetDevice(d->device));
  hipStream_t s = stream_of(h);
  const int64_t nd = op.n / 2, L = op.field_len, nc2 = 2 * op.n_cells;
  ifl_status st;
  if (!d->proj_ptr) {
    if ((st = upload(&d->proj_ptr, op.proj_ptr)) || (st = upload(&d->proj_tri, op.proj_tri)) ||
        (st = upload(&d->proj_w, op.proj_w)) || (st = dalloc(&d->proj_in, (size_t)nc2)))
      return st;
  }
  if ((st = ensure_stage(d, L)) != IFL_OK) return st;
  const double* src = cells;
  if (!is_device_ptr(cells)) {
    IFL_HIP(hipMemcpyAsync(d->proj_in, cells, sizeof(double) * nc2, hipMemcpyHostToDevice, s));
    src = d->proj_in;
  }
  const bool odev = is_device_ptr(out);
  double* dst = odev ? out : d->w.stage_out;
  IFL_HIP(hipMemsetAsync(dst, 0, sizeof(double) * L, s));
  const unsigned nb = (unsigned)((nd + kBlock - 1) / kBlock);
  k_project_cells<<<nb, kBlock, 0, s>>>(nd, d->proj_ptr, d->proj_tri, d->proj_w, d->m.entity, src, dst);
  IFL_HIP(hipGetLastError());
  if (!odev) IFL_HIP(hipMemcpyAsync(out, dst, sizeof(double) * L, hipMemcpyDeviceToHost, s));
  IFL_HIP(hipStreamSynchronize(s));
  return IFL_OK;
}

std::string device_profile_kernel(Handle* h) { return h->dev->prof_kernel; }

ifl_status device_profile_read(Handle* h, int64_t* launches, double* total_ms, double* bytes, int32_t reset) {
  DeviceState* d = h->dev;
  if (launches) *launches = d->prof_launches;
  if (total_ms) *total_ms = d->prof_ms;
  if (bytes) *bytes = d->prof_launches ? d->prof_bytes / d->prof_launches : 0.0;
  if (reset) {
    d->prof_launches = 0;
    d->prof_ms = 0.0;
    d->prof_bytes = 0.0;
  }
  return IFL_OK;
}

}  // namespace ifl
