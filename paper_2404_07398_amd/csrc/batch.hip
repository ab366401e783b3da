// Multi-RHS batched solver: many (field, scale) columns share one pass over
// the matrix stream of K_n.
//
// Every column is an independent Jacobi-PCG solve of S_j x = M phi_j with
// S_j = M + c_j K_n (Sect. 2.2.2, residual form x0 = phi_j). A tile holds R
// slots; vectors are stored rows x R with the R columns of a row contiguous.
// A lane owns C consecutive columns of one row (C x 4 B = 16 B for FP32,
// C x 8 B = 16 B for FP64), so vector traffic moves in 16-byte loads and
// stores and each lane carries C independent FMA chains; the R / C lanes of
// a row share the row's sliced-ELL entries (same address within the group),
// and a gather of a neighbour's R values is one contiguous segment. HBM
// traffic per column-iteration is the vector traffic plus 1/R of the matrix
// stream.
//
// Per-column state (alpha, beta, rho, stopping, residual replacement) lives
// in device memory; after each reduction phase a small kernel with one
// workgroup per column finishes that column's sum in a fixed order. A tile
// advances in chunks of L iterations (4 or 8) and columns enter only at
// chunk boundaries, so all live columns share the chunk position. Inside a
// chunk only z (the preconditioned residual) and p change; the directions
// of the chunk are kept in L buffers and x is updated once, at the
// chunk's last iteration (in FP64, in every precision), from them and each
// column's alpha history. Every running column's residual is then replaced
// by its FP64 true residual, in one pass for the whole tile, and a column
// stops only on such a replaced residual (in FP64 tiles as well: a recursive
// residual drifts from the true one when S is badly conditioned). A column's
// arithmetic and reduction order depend neither on the other columns, nor
// on its slot, nor on when it entered, so a solve gives bitwise the same
// result alone or in a full tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "batch.h"

namespace ifl {

#define IFL_HIPB(expr)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(IFL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

namespace {

constexpr int kW = 64;            // wavefront
constexpr int kB = 512;           // threads per block
constexpr int kWpb = kB / kW;     // waves per block
constexpr int kFinThreads = 256;  // per-column finalize workgroup
constexpr int kUnroll = 8;        // sliced-ELL entries loaded together per row
constexpr double kU = 1.1102230246251565e-16;
constexpr double kFloor = 8.0;

enum { Q_PQ = 0, Q_RZ, Q_RR, Q_BB, Q_FL, Q_EN, Q_ZU, Q_UU, Q_COUNT };

// Lane geometry of a tile of R columns of type T.
template <typename T, int R>
struct Geo {
  static constexpr int C = (int)(16 / sizeof(T)) < R ? (int)(16 / sizeof(T)) : R;  // columns per lane
  static constexpr int LPR = R / C;                                              // lanes per row
  static constexpr int RPW = kW / LPR;                                           // rows per wavefront
};

template <typename T, int C>
struct alignas(sizeof(T) * C) Pack {
  T v[C];
};

template <typename T, int C>
__device__ __forceinline__ Pack<T, C> vload(const T* p) {
  return *reinterpret_cast<const Pack<T, C>*>(p);
}
template <typename T, int C>
__device__ __forceinline__ void vstore(T* p, const Pack<T, C>& x) {
  *reinterpret_cast<Pack<T, C>*>(p) = x;
}

struct BMat {
  int64_t n, n_slices;
  const int32_t* row_of;  // caller index -> row (-1: no dof)
  int64_t field_len;
  const int64_t* sptr;
  const int32_t* col;
  const double* val64;
  const float* val32;
  const double* kdiag;
  const double* mass;
  const int64_t* entity;
  // 2 x 2-block sliced ELL of a two-component operator (pair kernels)
  int64_t nb, nb_slices;
  const int64_t* psptr;
  const int32_t* pcol;
  const double* pval64;
  const float* pval32;
};

template <typename T>
struct BVec {
  T* z[kChunk];  // preconditioned residual diag(S)^-1 r of each iteration of a chunk but the last
  T* u[2];       // diag(S)^-1 S p (two buffers)
  T* p[kChunk];  // p[kChunk - 1]: the direction carried from one chunk to the next
  double* x;     // FP64 solution
  double* phi;   // FP64 field per column
};

struct OutPtrs {
  double* p[64];
};

struct FieldPtrs {
  const double* p[64];
};

template <typename T>
__device__ __forceinline__ const T* bval(const BMat& m);
template <>
__device__ __forceinline__ const double* bval<double>(const BMat& m) { return m.val64; }
template <>
__device__ __forceinline__ const float* bval<float>(const BMat& m) { return m.val32; }

template <typename T>
__device__ __forceinline__ const T* pval(const BMat& m);
template <>
__device__ __forceinline__ const double* pval<double>(const BMat& m) { return m.pval64; }
template <>
__device__ __forceinline__ const float* pval<float>(const BMat& m) { return m.pval32; }

// partial-sum slot of this block
__device__ __forceinline__ int lblock(int) { return blockIdx.x; }

// Per-column block sums. Lane l carries columns (l % LPR) * C + c; the
// result for column t is returned in thread t (t < R), fixed order.
template <int R, int C, int NV>
__device__ __forceinline__ void col_sum(double (&v)[NV][C], double* lds /* NV * kWpb * R */, double (&out)[NV]) {
  constexpr int LPR = R / C;
  const int lane = threadIdx.x % kW, wid = threadIdx.x / kW;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      double s = v[i][c];
#pragma unroll
      for (int off = 32; off >= LPR; off >>= 1) s += __shfl_xor(s, off, kW);
      if (lane < LPR) lds[(i * kWpb + wid) * R + lane * C + c] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < R) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < kWpb; ++w) s += lds[(i * kWpb + w) * R + threadIdx.x];
      out[i] = s;
    }
  }
}

// Task walk of this block and wavefront (a task is RPW consecutive rows).
// XCD x (hardware dispatches workgroups round-robin over the 8 XCDs, so
// block b runs on XCD b % 8) owns a contiguous eighth of the tasks; inside
// it, the XCD's blocks and wavefronts take consecutive tasks in turn. With G
// no larger than the resident block count, the rows in flight on one XCD
// form a narrow band that advances through its eighth, so the rows that a
// band's gathers reach (the RCM neighbours before and after it) were touched
// shortly before or are touched shortly after, in the same XCD's L2.
struct Walk {
  int64_t t, end, stride;
};

__device__ __forceinline__ Walk task_walk(int64_t ntasks, int G) {
  const int b = blockIdx.x, wid = threadIdx.x / kW;
  if (G % 8) return {(int64_t)b * kWpb + wid, ntasks, (int64_t)G * kWpb};
  const int64_t per = (ntasks + 7) / 8;
  const int64_t begin = (int64_t)(b % 8) * per;
  return {begin + (int64_t)(b / 8) * kWpb + wid, min(begin + per, ntasks), (int64_t)(G / 8) * kWpb};
}

__device__ __forceinline__ bool live(const BSlot& s) { return s.active && s.done == 0; }

// Sliced-ELL row product: a[c] += sum_k val_k * comb(c, x0[k], x1[k]) over
// the row's entries in order, kUnroll entries at a time (index and value
// loads, then the 16-byte gathers of the operands, then the FMAs). Loads
// past the row's end stay in bounds (the next slice, or the zero tail after
// the last slice) and their value is replaced by 0, so they leave a
// unchanged.
template <typename V, typename T, int R, int C, bool TWO, typename Comb, int U = kUnroll>
__device__ __forceinline__ void row_product(const BMat& m, const V* __restrict__ val, int64_t base, int w,
                                            int64_t l, int j0, const T* __restrict__ x0,
                                            const T* __restrict__ x1, Comb comb, T (&a)[C], int k_begin = 0) {
  for (int k0 = k_begin; k0 < w; k0 += U) {
    int32_t cu[U];
    V vu[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = base + (int64_t)(k0 + u) * kW + l;
      cu[u] = m.col[e];
      const V vv = val[e];
      vu[u] = k0 + u < w ? vv : (V)0;
    }
    Pack<T, C> g0[U], g1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t off = (int64_t)cu[u] * R + j0;
      g0[u] = vload<T, C>(x0 + off);
      if constexpr (TWO) g1[u] = vload<T, C>(x1 + off);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < C; ++c) a[c] = fma((T)vu[u], comb(c, g0[u].v[c], TWO ? g1[u].v[c] : (T)0), a[c]);
  }
}

// Both sums of the FP64 residual over a row's entries from k_begin on, in
// one pass over the gathers: a[c] += val_k x[k], aa[c] += |val_k| |x[k]|.
template <int R, int C, int U = kUnroll>
__device__ __forceinline__ void row_product_abs2(const BMat& m, int64_t base, int w, int64_t l, int j0,
                                                 const double* __restrict__ x, double (&a)[C], double (&aa)[C],
                                                 int k_begin) {
  for (int k0 = k_begin; k0 < w; k0 += U) {
    int32_t cu[U];
    double vu[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = base + (int64_t)(k0 + u) * kW + l;
      cu[u] = m.col[e];
      const double vv = m.val64[e];
      vu[u] = k0 + u < w ? vv : 0.0;
    }
    Pack<double, C> g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = vload<double, C>(x + (int64_t)cu[u] * R + j0);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        a[c] = fma(vu[u], g[u].v[c], a[c]);
        aa[c] = fma(fabs(vu[u]), fabs(g[u].v[c]), aa[c]);
      }
  }
}

// combiner of row_product for a single gathered operand
struct Ident {
  __device__ double operator()(int, double xx, double) const { return xx; }
};

// ------------------------------------------------------------ iteration
// Off-diagonal entries per row that the gathering kernels load in their
// software-pipelined head: a class sized to the matrix (6 for the scalar
// first-order operator on triangle meshes, 12 for the interleaved vertex
// vectors, 20 for the biharmonic operator); rows with more entries finish
// the rest in steps of the same width, unpipelined.
constexpr int kHeadClasses[] = {6, 12, 20};

// a / d in the iteration kernels: FP32 tiles multiply by the hardware
// reciprocal (1 ulp), a rounding of the kind their recurrences already
// carry; FP64 tiles divide
__device__ __forceinline__ float over(float a, float d) { return a * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double over(double a, double d) { return a / d; }

// Lanes of a row share the row's matrix entries: each of the LPR lanes of a
// row (consecutive lanes, LPR dividing 32) loads every LPR-th entry, and
// ds_swizzle (bit mode, within 32 lanes) hands lane SRC's copy to the others
// of its row. The swizzle runs on the LDS crossbar, not the vector memory
// path, which the gathers keep busy.
template <int LPR, int SRC>
__device__ __forceinline__ int row_share(int x) {
  constexpr int kPattern = (0x1F & ~(LPR - 1)) | (SRC << 5);
  return __builtin_amdgcn_ds_swizzle(x, kPattern);
}
template <int LPR, int SRC>
__device__ __forceinline__ float row_share(float x) {
  return __int_as_float(row_share<LPR, SRC>(__float_as_int(x)));
}
template <int LPR, int SRC>
__device__ __forceinline__ double row_share(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = row_share<LPR, SRC>((int)(b & 0xffffffffll)), hi = row_share<LPR, SRC>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <typename F, int... I>
__device__ __forceinline__ void unroll_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0..N-1 (i usable as a template argument)
template <int N, typename F>
__device__ __forceinline__ void unroll(F&& f) {
  unroll_seq(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ int64_t wave_uniform(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One CG iteration per launch, with u = diag(S)^-1 S p in place of q = S p
// (d = diag(S) = M + c diag(K_n), the Jacobi preconditioner; z = d^-1 r is
// the residual state, r = d z is formed where it is needed):
//
//  FUSED (iterations 1..L-1 of a chunk of L), given alpha_k-1 and beta_k:
//    z_k = z_k-1 - alpha_k-1 u_k-1        (own row and every gathered neighbour)
//    u_k = z_k + d^-1 c K_off z_k + beta_k u_k-1   (= d^-1 S p_k, as
//          S p_k = S z_k + beta_k S p_k-1 with p_k = z_k + beta_k p_k-1)
//  so z and u are the only gathered operands and the only vectors a row
//  reads and writes: the kernel reads z_k-1, u_k-1 and writes z_k (kept in
//  z[k] for the x update) and u_k. The chunk's last iteration stores
//  nothing: its u is never read, and the x update forms its z from z_L-2 and
//  u_L-2. The directions p_k are never formed here; the chunk's x update
//  rebuilds them from z_0..z_L-1 and the carried p_-1.
//  DIRECT (the first iteration of a chunk, after the FP64 residual
//  replacement has set z_0): p_0 = z_0 + beta_0 p_-1 from the carried
//  direction, u_0 = d^-1 S p_0 from p_0 of the row and its gathered
//  neighbours, so the recurrence for u never spans more than a chunk.
//
// Partials per column (one grid-level reduction per iteration, finished by
// kf_step): sum d z_k u_k = (z_k, q_k), sum d u_k^2 = (q_k, d^-1 q_k), and
//   DIRECT: sum d p_0 u_0 = (p_0, q_0);
//   FUSED:  sum d u_k-1 z_k = (q_k-1, z_k) and rho_k = (r_k, z_k) = sum d z_k^2.
// With S symmetric, (p_k, q_k) = (z_k, q_k) + beta_k (p_k-1, q_k) and
// (p_k-1, q_k) = (q_k-1, p_k) = (q_k-1, z_k) + beta_k (p_k-1, q_k-1), which
// gives (p_k, q_k) from the partials and the last iteration's (p, q) with
// no conjugacy assumed. Then alpha_k = rho_k / (p_k, q_k) and the next rho =
// (r - alpha q, z - alpha d^-1 q) = rho - 2 alpha (q, z) + alpha^2 (q, d^-1 q)
// gives beta for the next launch before the next z exists.
//
// The loop over a wavefront's tasks is software-pipelined so that a task
// costs about one memory round trip instead of three. While the gathers of
// task i are in flight, the slice bounds of task i + 2 and the column
// indices of task i + 1 are loaded; after task i's row is computed, the
// values and own-row operands of task i + 1 are loaded, and they arrive
// under the gathers of task i + 1. Vector memory operations complete in
// issue order, so waiting for a batch of loads never waits for the loads
// issued after it.
template <typename T, int R, bool FUSED, int H, bool KEEP>
__device__ __forceinline__ void iter_body(const BMat& m, const BVec<T>& v, const BSlot* slots, double* part, int G,
                                          int Gp, int k, int L) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR, RPW = Gm::RPW;
  constexpr int NQ = FUSED ? 4 : 3;
  __shared__ double lds[NQ * kWpb * R];
  const int lane = threadIdx.x % kW;
  const int j0 = (lane % LPR) * C, rsub = lane / LPR;
  T alpha[C], beta[C], cc[C];
  double c64[C];
  bool on[C];
  bool any = false;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const BSlot& sl = slots[j0 + c];
    on[c] = live(sl);
    alpha[c] = on[c] ? (T)sl.alpha : (T)0;
    beta[c] = on[c] ? (T)sl.beta : (T)0;
    cc[c] = (T)sl.c;
    c64[c] = sl.c;
    any |= on[c];
  }
  // buffers: iteration k reads z[k - 1] (DIRECT: z[0], set by the
  // replacement) and writes z[k]; u alternates, u_k in u[k & 1]; DIRECT
  // reads the carried direction p_-1 in p[L - 1]
  const T* __restrict__ zin = v.z[FUSED ? k - 1 : 0];
  T* __restrict__ zout = v.z[k];
  const T* __restrict__ uin = v.u[(k + 1) & 1];
  T* __restrict__ uout = v.u[k & 1];
  const T* __restrict__ pin = v.p[L - 1];
  const T* __restrict__ val = bval<T>(m);
  // value of a gathered neighbour: z_k (FUSED) or p_0 (DIRECT); g1 is u or p
  const auto comb = [&](int c, T g0, T g1) { return FUSED ? fma(-alpha[c], g1, g0) : fma(beta[c], g1, g0); };
  double acc[NQ][C] = {};
  // the whole wave walks the tasks if any of its lanes has a live column
  // (the lanes of a row share the row's entries); lanes whose columns have
  // all stopped rewrite those columns' vectors, which nothing reads, and add
  // nothing to the partials
  if (__any(any)) {
    const Walk wk = task_walk(m.n_slices * LPR, G);
    const int64_t first = wave_uniform(wk.t), end = wk.end, stride = wk.stride;
    const int64_t last_slice = m.n_slices - 1;
    // a task's rows lie in one slice; out-of-range tasks are clamped so that
    // every load of the loop body is issued unconditionally (a fixed count
    // of memory operations per iteration keeps the compiler's wait counts
    // exact), and their results are discarded
    auto slice_of = [&](int64_t t) { return min((t * RPW) / kW, last_slice); };
    // entries of the head: lane lc of a row loads entries lc, lc + LPR, ...
    // (the last entry again past H), shared across the row by row_share
    constexpr int NL = (H + LPR - 1) / LPR;
    const int lc = lane % LPR;
    int32_t cu[H], cl[NL];
    T vu[H], vl[NL];
    Pack<T, C> zi, gi;  // own row: z and (FUSED) u or (DIRECT) p
    double mi, kd;
    int64_t base, nb, ne;  // this task's slice base; next task's raw slice bounds
    int w;
    auto fetch_idx = [&](int64_t t, int64_t sb) {
      const int64_t l = (t * RPW + rsub) % kW;
#pragma unroll
      for (int i = 0; i < NL; ++i) cl[i] = m.col[sb + (int64_t)min(lc + i * LPR, H - 1) * kW + l];
    };
    auto share_idx = [&]() {
      unroll<H>([&](auto U) {
        constexpr int u = decltype(U)::value;
        if constexpr (LPR == 1) cu[u] = cl[u];
        else cu[u] = row_share<LPR, u % LPR>(cl[u / LPR]);
      });
    };
    auto share_val = [&]() {
      unroll<H>([&](auto U) {
        constexpr int u = decltype(U)::value;
        if constexpr (LPR == 1) vu[u] = vl[u];
        else vu[u] = row_share<LPR, u % LPR>(vl[u / LPR]);
      });
    };
    // values are loaded raw (entries past the width are masked where they
    // are used, so that no instruction consumes the loads early)
    auto fetch_rest = [&](int64_t t, int64_t sb) {
      const int64_t row = min(t * RPW + rsub, m.n_slices * kW - 1), l = row % kW;
#pragma unroll
      for (int i = 0; i < NL; ++i) vl[i] = val[sb + (int64_t)min(lc + i * LPR, H - 1) * kW + l];
      const int64_t idx = row * R + j0;
      zi = vload<T, C>(zin + idx);
      gi = vload<T, C>((FUSED ? uin : pin) + idx);
      mi = m.mass[row];
      kd = m.kdiag[row];
    };
    {
      const int64_t s0 = slice_of(first);
      base = wave_uniform(m.sptr[s0]);
      w = (int)((wave_uniform(m.sptr[s0 + 1]) - base) / kW);
      fetch_idx(first, base);
      fetch_rest(first, base);
      share_idx();
      const int64_t s1 = slice_of(first + stride);
      nb = m.sptr[s1];
      ne = m.sptr[s1 + 1];
    }
    for (int64_t t = first; t < end; t += stride) {
      const int64_t row = t * RPW + rsub;
      const int32_t self = (int32_t)min(row, m.n - 1);
      // (a) gathers of this task; entries past the row's width (padding of
      // value 0) gather the row itself, a line that is loaded anyway
      Pack<T, C> g0[H], g1[H];
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const int64_t off = (int64_t)(u < w ? cu[u] : self) * R + j0;
        g0[u] = vload<T, C>(zin + off);
        g1[u] = vload<T, C>((FUSED ? uin : pin) + off);
      }
      const int64_t cbase = base;
      const int cw = w;
      // (b) slice bounds two tasks ahead, (c) indices of the next task
      const int64_t tn = t + stride < end ? t + stride : t;
      const int64_t s2 = slice_of(t + 2 * stride);
      const int64_t nb2 = m.sptr[s2], ne2 = m.sptr[s2 + 1];
      base = wave_uniform(nb);
      w = (int)((wave_uniform(ne) - base) / kW);
      fetch_idx(tn, base);
      nb = nb2;
      ne = ne2;
      // (d) this task's row (rows past the last dof are padding: zero mass,
      // diagonal and entries; their results are discarded)
      share_val();
      T a[C] = {};
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const T vm = u < cw ? vu[u] : (T)0;
#pragma unroll
        for (int c = 0; c < C; ++c) a[c] = fma(vm, comb(c, g0[u].v[c], g1[u].v[c]), a[c]);
      }
      if (cw > H)
        row_product<T, T, R, C, true, decltype(comb), H>(m, val, cbase, cw, row % kW, j0, zin,
                                                         FUSED ? uin : pin, comb, a, H);
      const bool real = row < m.n;
      const int64_t idx = row * R + j0;
      Pack<T, C> zn, un;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const T d = real ? (T)(mi + c64[c] * kd) : (T)1;
        // the row's weight in the column's partials (0 where the row or the
        // column does not count); each product below is the weight times a
        // vector in T, i.e. r = d z or d u, so no new range is needed, and
        // it is summed in FP64
        const T dw = on[c] && real ? d : (T)0;
        const T su = over(cc[c] * a[c], d);  // d^-1 c K_off applied to the gathered operand
        if constexpr (FUSED) {
          zn.v[c] = fma(-alpha[c], gi.v[c], zi.v[c]);
          un.v[c] = fma(beta[c], gi.v[c], zn.v[c] + su);
        } else {
          zn.v[c] = zi.v[c];
          un.v[c] = fma(beta[c], gi.v[c], zi.v[c]) + su;
        }
        const double rz = (double)(dw * zn.v[c]), ru = (double)(dw * un.v[c]), uu = (double)un.v[c];
        if constexpr (FUSED) {
          acc[0][c] = fma(rz, (double)gi.v[c], acc[0][c]);
          acc[NQ - 1][c] = fma(rz, (double)zn.v[c], acc[NQ - 1][c]);
        } else {
          acc[0][c] = fma(ru, (double)fma(beta[c], gi.v[c], zi.v[c]), acc[0][c]);
        }
        acc[1][c] = fma(rz, uu, acc[1][c]);
        acc[2][c] = fma(ru, uu, acc[2][c]);
      }
      if constexpr (KEEP) {
        if (real) {
          vstore<T, C>(uout + idx, un);
          if constexpr (FUSED) vstore<T, C>(zout + idx, zn);
        }
      }
      // (e) values and own row of the next task; its indices to every lane
      fetch_rest(tn, base);
      share_idx();
    }
  }
  double tot[NQ];
  col_sum<R, C, NQ>(acc, lds, tot);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_PQ * R + threadIdx.x) * Gp + lb] = tot[0];
    part[(Q_ZU * R + threadIdx.x) * Gp + lb] = tot[1];
    part[(Q_UU * R + threadIdx.x) * Gp + lb] = tot[2];
    if constexpr (FUSED) part[(Q_RZ * R + threadIdx.x) * Gp + lb] = tot[NQ - 1];
  }
}

// iterations 0..L-2 of a chunk (FUSED: 1..L-2)
template <typename T, int R, bool FUSED, int H>
__global__ __launch_bounds__(kB) void kb_iter(BMat m, BVec<T> v, const BSlot* slots, double* part, int G, int Gp,
                                              int k, int L) {
  iter_body<T, R, FUSED, H, true>(m, v, slots, part, G, Gp, k, L);
}

// the chunk's last iteration (k = L - 1): partials only, nothing stored
template <typename T, int R, int H>
__global__ __launch_bounds__(kB) void kb_iter_last(BMat m, BVec<T> v, const BSlot* slots, double* part, int G,
                                                   int Gp, int k, int L) {
  iter_body<T, R, true, H, false>(m, v, slots, part, G, Gp, k, L);
}

// The chunk's x update, at its last iteration, in FP64 in every precision:
// the directions are rebuilt from the chunk's z_k (z_L-1 from z_L-2 and
// u_L-2, the FP32 update the last iteration applied) and the carried p_-1,
// p_k = z_k + beta_k p_k-1 (in FP64), x += sum_k alpha_k p_k (alpha_k = 0
// for a column that was not iterating), and p_L-1 is carried to the next
// chunk in place of p_-1 (columns that did not iterate keep theirs).
// A one-pass launch: one thread per row and lane (a streaming pass runs
// faster with a thread per element than walking the rows with the resident
// workgroups), the columns' alpha and beta histories staged in LDS once per
// block of kXB threads.
constexpr int kXB = 1024;
template <typename T, int R, int L>
__global__ __launch_bounds__(kXB) void kb_xupdate(BMat m, BVec<T> v, const BSlot* slots) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR;
  __shared__ double hist[2 * L * R];  // alpha_hist[k] of column j at k R + j, beta_hist after them
  for (int i = threadIdx.x; i < 2 * L * R; i += kXB) {
    const int j = i % R, k = (i / R) % L;
    hist[i] = i < L * R ? slots[j].alpha_hist[k] : slots[j].beta_hist[k];
  }
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * kXB + threadIdx.x;
  const int64_t row = g / LPR;
  if (row >= m.n) return;
  const int j0 = (int)(g % LPR) * C;
  double ah[L][C], bh[L][C];
  bool moved[C];
  bool any = false;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    moved[c] = false;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      ah[i][c] = hist[i * R + j0 + c];
      bh[i][c] = hist[(L + i) * R + j0 + c];
      moved[c] |= ah[i][c] != 0.0;
    }
    any |= moved[c];
  }
  if (!any) return;
  const int64_t idx = row * R + j0;
  Pack<T, C> zk[L];
#pragma unroll
  for (int i = 0; i < L - 1; ++i) zk[i] = vload<T, C>(v.z[i] + idx);
  zk[L - 1] = vload<T, C>(v.u[(L - 2) & 1] + idx);
  Pack<double, C> xv = vload<double, C>(v.x + idx);
  Pack<T, C> pc = vload<T, C>(v.p[L - 1] + idx);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    zk[L - 1].v[c] = fma(-(T)ah[L - 2][c], zk[L - 1].v[c], zk[L - 2].v[c]);
    double pd = (double)pc.v[c];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      pd = fma(bh[i][c], pd, (double)zk[i].v[c]);
      xv.v[c] = fma(ah[i][c], pd, xv.v[c]);
    }
    if (moved[c]) pc.v[c] = (T)pd;
  }
  vstore<T, C>(v.p[L - 1] + idx, pc);
  vstore<double, C>(v.x + idx, xv);
}

// FP64 residual passes, software-pipelined like kb_iter (the gathered
// operand is FP64: 16 B per lane and entry for FP64 tiles, 32 B for mixed).
//
// START (the columns in 'mask', scales cs): x = phi, p = 0 and the residual
// of the residual form r0 = M phi - S phi = -c K_n phi, z = r0 / diag(S), with
// the partials of (r, z), (r, r) and ||M phi||^2. Other columns' vectors are
// left unchanged.
//
// REPLACE (at the end of every chunk, after its x update): the
// residual of every running column is replaced by its FP64 true residual
// r = M phi - S x (FP64 values and x), z = r / diag(S), with the partials of
// (r, z), (r, r) and of the attainable-accuracy norm
// || |M phi| + |M x| + c |K_n| |x| ||^2. z of columns that are not running is
// overwritten with values nothing reads (a column that enters is started
// from scratch).
template <typename T, int R, bool START, int H>
__global__ __launch_bounds__(kB) void kb_residual(BMat m, BVec<T> v, const BSlot* slots, double* part, int G,
                                                  int Gp, uint64_t mask, SlotScales cs, int L) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR, RPW = Gm::RPW;
  __shared__ double lds[3 * kWpb * R];
  const int lane = threadIdx.x % kW;
  const int j0 = (lane % LPR) * C, rsub = lane / LPR;
  bool on[C];
  double cc[C];
  bool any = false, all = true;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    if constexpr (START) {
      on[c] = ((mask >> (j0 + c)) & 1ull) != 0;
      cc[c] = cs.c[j0 + c];
    } else {
      on[c] = live(slots[j0 + c]);
      cc[c] = slots[j0 + c].c;
    }
    any |= on[c];
    all &= on[c];
  }
  const double* __restrict__ src = START ? v.phi : v.x;  // the gathered operand
  T* __restrict__ pprev = v.p[L - 1];  // the chunk's first iteration reads it as p
  const Ident ident;
  double acc[3][C] = {};
  // REPLACE with the first-order head: the whole wave walks the tasks if any
  // of its lanes has a live column, and the lanes of a row share the row's
  // entries (as kb_iter; with the wider heads the shared copies push the
  // FP64 pass past the register file); START: only lanes with an entering
  // column, each loading its entries
  constexpr bool SHARE = !START && LPR > 1 && H <= 6;
  bool run;
  if constexpr (SHARE) run = __any(any);
  else run = any;
  if (run) {
    const Walk wk = task_walk(m.n_slices * LPR, G);
    const int64_t first = wave_uniform(wk.t), end = wk.end, stride = wk.stride;
    const int64_t last_slice = m.n_slices - 1;
    auto slice_of = [&](int64_t t) { return min((t * RPW) / kW, last_slice); };
    constexpr int LS = SHARE ? LPR : 1;  // lanes that split a row's entries
    constexpr int NL = (H + LS - 1) / LS;
    const int lc = SHARE ? lane % LPR : 0;
    int32_t cu[H], cl[NL];
    double vu[H], vl[NL];
    Pack<double, C> ph, xv;
    double mi, kd;
    int64_t base, nb, ne;
    int w;
    auto fetch_idx = [&](int64_t t, int64_t sb) {
      const int64_t l = (t * RPW + rsub) % kW;
#pragma unroll
      for (int i = 0; i < NL; ++i) cl[i] = m.col[sb + (int64_t)min(lc + i * LS, H - 1) * kW + l];
    };
    auto share_idx = [&]() {
      unroll<H>([&](auto U) {
        constexpr int u = decltype(U)::value;
        if constexpr (LS == 1) cu[u] = cl[u];
        else cu[u] = row_share<LS, u % LS>(cl[u / LS]);
      });
    };
    auto share_val = [&]() {
      unroll<H>([&](auto U) {
        constexpr int u = decltype(U)::value;
        if constexpr (LS == 1) vu[u] = vl[u];
        else vu[u] = row_share<LS, u % LS>(vl[u / LS]);
      });
    };
    auto fetch_rest = [&](int64_t t, int64_t sb) {
      const int64_t row = min(t * RPW + rsub, m.n_slices * kW - 1), l = row % kW;
#pragma unroll
      for (int i = 0; i < NL; ++i) vl[i] = m.val64[sb + (int64_t)min(lc + i * LS, H - 1) * kW + l];
      const int64_t idx = row * R + j0;
      ph = vload<double, C>(v.phi + idx);
      if constexpr (!START) xv = vload<double, C>(v.x + idx);
      mi = m.mass[row];
      kd = m.kdiag[row];
    };
    {
      const int64_t s0 = slice_of(first);
      base = wave_uniform(m.sptr[s0]);
      w = (int)((wave_uniform(m.sptr[s0 + 1]) - base) / kW);
      fetch_idx(first, base);
      fetch_rest(first, base);
      share_idx();
      const int64_t s1 = slice_of(first + stride);
      nb = m.sptr[s1];
      ne = m.sptr[s1 + 1];
    }
    for (int64_t t = first; t < end; t += stride) {
      const int64_t row = t * RPW + rsub;
      const int32_t self = (int32_t)min(row, m.n - 1);
      Pack<double, C> gx[H];
#pragma unroll
      for (int u = 0; u < H; ++u) gx[u] = vload<double, C>(src + (int64_t)(u < w ? cu[u] : self) * R + j0);
      const int64_t cbase = base;
      const int cw = w;
      const int64_t tn = t + stride < end ? t + stride : t;
      const int64_t s2 = slice_of(t + 2 * stride);
      const int64_t nb2 = m.sptr[s2], ne2 = m.sptr[s2 + 1];
      base = wave_uniform(nb);
      w = (int)((wave_uniform(ne) - base) / kW);
      fetch_idx(tn, base);
      nb = nb2;
      ne = ne2;
      share_val();
      double a[C] = {}, aa[C] = {};  // sum val x, sum |val| |x| (REPLACE)
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const double vm = u < cw ? vu[u] : 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          a[c] = fma(vm, gx[u].v[c], a[c]);
          if constexpr (!START) aa[c] = fma(fabs(vm), fabs(gx[u].v[c]), aa[c]);
        }
      }
      if (cw > H) {
        if constexpr (START)
          row_product<double, double, R, C, false, decltype(ident), H>(
              m, m.val64, cbase, cw, row % kW, j0, src, nullptr, ident, a, H);
        else
          row_product_abs2<R, C, H>(m, cbase, cw, row % kW, j0, src, a, aa, H);
      }
      const bool real = row < m.n;
      const int64_t idx = row * R + j0;
      if constexpr (START) {
        if (real) {
          // columns of this lane that do not start keep their state
          Pack<double, C> xo = ph;
          Pack<T, C> zo, po = {};
          if (!all) {
            xo = vload<double, C>(v.x + idx);
            zo = vload<T, C>(v.z[0] + idx);
            po = vload<T, C>(pprev + idx);
          }
#pragma unroll
          for (int c = 0; c < C; ++c) {
            if (!on[c]) continue;
            const double r64 = -cc[c] * (kd * ph.v[c] + a[c]);
            const T rt = (T)r64;
            const T d = (T)(mi + cc[c] * kd);
            xo.v[c] = ph.v[c];
            zo.v[c] = rt / d;
            po.v[c] = (T)0;
            acc[0][c] += (double)rt * (double)zo.v[c];
            acc[1][c] += r64 * r64;
            acc[2][c] += (mi * ph.v[c]) * (mi * ph.v[c]);
          }
          vstore<double, C>(v.x + idx, xo);
          vstore<T, C>(v.z[0] + idx, zo);
          vstore<T, C>(pprev + idx, po);
        }
      } else {
        Pack<T, C> zv;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const double xf = xv.v[c];
          const double r64 = mi * (ph.v[c] - xf) - cc[c] * (kd * xf + a[c]);
          const T rt = (T)r64;
          const T d = (T)(mi + cc[c] * kd);
          zv.v[c] = rt / d;
          if (on[c] && real) {
            const double mag = fabs(mi * ph.v[c]) + fabs(mi * xf) + cc[c] * (fabs(kd * xf) + aa[c]);
            acc[0][c] += (double)rt * (double)zv.v[c];
            acc[1][c] += r64 * r64;
            acc[2][c] += mag * mag;
          }
        }
        if (real) vstore<T, C>(v.z[0] + idx, zv);
      }
      fetch_rest(tn, base);
      share_idx();
    }
  }
  double tot[3];
  col_sum<R, C, 3>(acc, lds, tot);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_RZ * R + threadIdx.x) * Gp + lb] = tot[0];
    part[(Q_RR * R + threadIdx.x) * Gp + lb] = tot[1];
    part[((START ? Q_BB : Q_FL) * R + threadIdx.x) * Gp + lb] = tot[2];
  }
}

// ------------------------------------------------------------ 2 x 2 blocks
// Pair forms of kb_iter and kb_residual for two-component operators (rows
// 2b and 2b + 1 are the two components of block row b). A task is RPW block
// rows; a lane handles its C columns of both rows of a block row, and a
// neighbour block's two rows are gathered together: two 16-byte loads per
// gathered vector and neighbour for the pair of rows, where the row forms
// make four (each row gathers both components of every neighbour). The
// per-row arithmetic is that of the row forms; a block row's sums run over
// its blocks in increasing block column, component 2j before 2j + 1, the
// order of the row forms' sorted entries. The vectors keep their row
// layout, so the streaming kernels are shared.

// Blocks k_begin .. w - 1 of a block row in steps of U (past the pipelined
// head): a[r][c] += sum_blocks v[2r] comb(x(2j)) + v[2r + 1] comb(x(2j + 1)).
// Entries past the row's end are in bounds (next slice, or the zero tail)
// and their values are replaced by 0.
template <typename V, typename T, int R, int C, bool TWO, typename Comb, int U>
__device__ __forceinline__ void pair_product(const BMat& m, const V* __restrict__ val, int64_t base, int w,
                                             int64_t l, int j0, const T* __restrict__ x0,
                                             const T* __restrict__ x1, Comb comb, T (&a)[2][C], int k_begin) {
  for (int k0 = k_begin; k0 < w; k0 += U) {
    int32_t cu[U];
    Pack<V, 4> vu[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = base + (int64_t)(k0 + u) * kW + l;
      cu[u] = m.pcol[e];
      vu[u] = vload<V, 4>(val + 4 * e);
    }
    Pack<T, C> g0[U][2], g1[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t off = (int64_t)cu[u] * (2 * R) + j0;
      g0[u][0] = vload<T, C>(x0 + off);
      g0[u][1] = vload<T, C>(x0 + off + R);
      if constexpr (TWO) {
        g1[u][0] = vload<T, C>(x1 + off);
        g1[u][1] = vload<T, C>(x1 + off + R);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = k0 + u < w;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const T xu = comb(c, g0[u][0].v[c], TWO ? g1[u][0].v[c] : (T)0);
        const T xv = comb(c, g0[u][1].v[c], TWO ? g1[u][1].v[c] : (T)0);
        a[0][c] = fma(in ? (T)vu[u].v[0] : (T)0, xu, a[0][c]);
        a[0][c] = fma(in ? (T)vu[u].v[1] : (T)0, xv, a[0][c]);
        a[1][c] = fma(in ? (T)vu[u].v[2] : (T)0, xu, a[1][c]);
        a[1][c] = fma(in ? (T)vu[u].v[3] : (T)0, xv, a[1][c]);
      }
    }
  }
}

// The FP64 residual's two sums over blocks k_begin .. w - 1: a += v x,
// aa += |v| |x| (pair form of row_product_abs2).
template <int R, int C, int U>
__device__ __forceinline__ void pair_product_abs2(const BMat& m, int64_t base, int w, int64_t l, int j0,
                                                  const double* __restrict__ x, double (&a)[2][C],
                                                  double (&aa)[2][C], int k_begin) {
  for (int k0 = k_begin; k0 < w; k0 += U) {
    int32_t cu[U];
    Pack<double, 4> vu[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = base + (int64_t)(k0 + u) * kW + l;
      cu[u] = m.pcol[e];
      vu[u] = vload<double, 4>(m.pval64 + 4 * e);
    }
    Pack<double, C> g[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t off = (int64_t)cu[u] * (2 * R) + j0;
      g[u][0] = vload<double, C>(x + off);
      g[u][1] = vload<double, C>(x + off + R);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = k0 + u < w;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const double v0 = in ? vu[u].v[2 * r] : 0.0, v1 = in ? vu[u].v[2 * r + 1] : 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          a[r][c] = fma(v0, g[u][0].v[c], a[r][c]);
          a[r][c] = fma(v1, g[u][1].v[c], a[r][c]);
          aa[r][c] = fma(fabs(v0), fabs(g[u][0].v[c]), aa[r][c]);
          aa[r][c] = fma(fabs(v1), fabs(g[u][1].v[c]), aa[r][c]);
        }
      }
    }
  }
}

// kb_iter on 2 x 2 blocks (same forms, buffers and partials).
template <typename T, int R, bool FUSED, int H, bool KEEP>
__device__ __forceinline__ void pair_body(const BMat& m, const BVec<T>& v, const BSlot* slots, double* part, int G,
                                          int Gp, int k, int L) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR, RPW = Gm::RPW;
  constexpr int NQ = FUSED ? 4 : 3;
  __shared__ double lds[NQ * kWpb * R];
  const int lane = threadIdx.x % kW;
  const int j0 = (lane % LPR) * C, bsub = lane / LPR;
  T alpha[C], beta[C], cc[C];
  double c64[C];
  bool on[C];
  bool any = false;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const BSlot& sl = slots[j0 + c];
    on[c] = live(sl);
    alpha[c] = on[c] ? (T)sl.alpha : (T)0;
    beta[c] = on[c] ? (T)sl.beta : (T)0;
    cc[c] = (T)sl.c;
    c64[c] = sl.c;
    any |= on[c];
  }
  // buffers as in kb_iter (z-and-u form)
  const T* __restrict__ zin = v.z[FUSED ? k - 1 : 0];
  T* __restrict__ zout = v.z[k];
  const T* __restrict__ uin = v.u[(k + 1) & 1];
  T* __restrict__ uout = v.u[k & 1];
  const T* __restrict__ pin = v.p[L - 1];
  const T* __restrict__ g1src = FUSED ? uin : pin;
  const T* __restrict__ val = pval<T>(m);
  const auto comb = [&](int c, T g0, T g1) { return FUSED ? fma(-alpha[c], g1, g0) : fma(beta[c], g1, g0); };
  double acc[NQ][C] = {};
  if (any) {
    const Walk wk = task_walk(m.nb_slices * LPR, G);
    const int64_t first = wave_uniform(wk.t), end = wk.end, stride = wk.stride;
    const int64_t last_slice = m.nb_slices - 1;
    const int64_t last_row = m.n_slices * kW - 1;  // vectors, mass and diagonal hold n_slices * 64 rows
    auto slice_of = [&](int64_t t) { return min((t * RPW) / kW, last_slice); };
    int32_t cu[H];
    Pack<T, 4> vu[H];
    Pack<T, C> zi[2], gi[2];  // own rows: z and (FUSED) u or (DIRECT) p
    double mi[2], kd[2];
    int64_t base, nb, ne;
    int w;
    auto fetch_idx = [&](int64_t t, int64_t sb) {
      const int64_t l = (t * RPW + bsub) % kW;
#pragma unroll
      for (int u = 0; u < H; ++u) cu[u] = m.pcol[sb + (int64_t)u * kW + l];
    };
    auto fetch_rest = [&](int64_t t, int64_t sb) {
      const int64_t brow = min(t * RPW + bsub, m.nb_slices * kW - 1), l = brow % kW;
#pragma unroll
      for (int u = 0; u < H; ++u) vu[u] = vload<T, 4>(val + 4 * (sb + (int64_t)u * kW + l));
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int64_t row = min(2 * brow + r, last_row), idx = row * R + j0;
        zi[r] = vload<T, C>(zin + idx);
        gi[r] = vload<T, C>(g1src + idx);
        mi[r] = m.mass[row];
        kd[r] = m.kdiag[row];
      }
    };
    {
      const int64_t s0 = slice_of(first);
      base = wave_uniform(m.psptr[s0]);
      w = (int)((wave_uniform(m.psptr[s0 + 1]) - base) / kW);
      fetch_idx(first, base);
      fetch_rest(first, base);
      const int64_t s1 = slice_of(first + stride);
      nb = m.psptr[s1];
      ne = m.psptr[s1 + 1];
    }
    for (int64_t t = first; t < end; t += stride) {
      const int64_t brow = t * RPW + bsub;
      const int64_t self = min(brow, m.nb - 1);
      // (a) gathers of this task: both rows of every neighbour block
      Pack<T, C> g0[H][2], g1[H][2];
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const int64_t off = (u < w ? (int64_t)cu[u] : self) * (2 * R) + j0;
        g0[u][0] = vload<T, C>(zin + off);
        g0[u][1] = vload<T, C>(zin + off + R);
        g1[u][0] = vload<T, C>(g1src + off);
        g1[u][1] = vload<T, C>(g1src + off + R);
      }
      const int64_t cbase = base;
      const int cw = w;
      // (b) slice bounds two tasks ahead, (c) indices of the next task
      const int64_t tn = t + stride < end ? t + stride : t;
      const int64_t s2 = slice_of(t + 2 * stride);
      const int64_t nb2 = m.psptr[s2], ne2 = m.psptr[s2 + 1];
      base = wave_uniform(nb);
      w = (int)((wave_uniform(ne) - base) / kW);
      fetch_idx(tn, base);
      nb = nb2;
      ne = ne2;
      // (d) the two rows of this block row
      T a[2][C] = {};
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const bool in = u < cw;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const T xu = comb(c, g0[u][0].v[c], g1[u][0].v[c]);
          const T xv = comb(c, g0[u][1].v[c], g1[u][1].v[c]);
          a[0][c] = fma(in ? vu[u].v[0] : (T)0, xu, a[0][c]);
          a[0][c] = fma(in ? vu[u].v[1] : (T)0, xv, a[0][c]);
          a[1][c] = fma(in ? vu[u].v[2] : (T)0, xu, a[1][c]);
          a[1][c] = fma(in ? vu[u].v[3] : (T)0, xv, a[1][c]);
        }
      }
      if (cw > H)
        pair_product<T, T, R, C, true, decltype(comb), H>(m, val, cbase, cw, brow % kW, j0, zin, g1src, comb, a,
                                                           H);
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int64_t row = 2 * brow + r;
        const bool real = row < m.n;
        const int64_t idx = row * R + j0;
        Pack<T, C> zn, un;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const T d = real ? (T)(mi[r] + c64[c] * kd[r]) : (T)1;
          const T dw = on[c] && real ? d : (T)0;  // the row's weight in the partials (as kb_iter)
          const T su = over(cc[c] * a[r][c], d);
          T pn = 0;
          if constexpr (FUSED) {
            zn.v[c] = fma(-alpha[c], gi[r].v[c], zi[r].v[c]);
            un.v[c] = fma(beta[c], gi[r].v[c], zn.v[c] + su);
          } else {
            zn.v[c] = zi[r].v[c];
            pn = fma(beta[c], gi[r].v[c], zi[r].v[c]);
            un.v[c] = pn + su;
          }
          const double rz = (double)(dw * zn.v[c]), ru = (double)(dw * un.v[c]), uu = (double)un.v[c];
          if constexpr (FUSED) {
            acc[0][c] = fma(rz, (double)gi[r].v[c], acc[0][c]);
            acc[NQ - 1][c] = fma(rz, (double)zn.v[c], acc[NQ - 1][c]);
          } else {
            acc[0][c] = fma(ru, (double)pn, acc[0][c]);
          }
          acc[1][c] = fma(rz, uu, acc[1][c]);
          acc[2][c] = fma(ru, uu, acc[2][c]);
        }
        if constexpr (KEEP) {
          if (real) {
            vstore<T, C>(uout + idx, un);
            if constexpr (FUSED) vstore<T, C>(zout + idx, zn);
          }
        }
      }
      // (e) values and own rows of the next task
      fetch_rest(tn, base);
    }
  }
  double tot[NQ];
  col_sum<R, C, NQ>(acc, lds, tot);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_PQ * R + threadIdx.x) * Gp + lb] = tot[0];
    part[(Q_ZU * R + threadIdx.x) * Gp + lb] = tot[1];
    part[(Q_UU * R + threadIdx.x) * Gp + lb] = tot[2];
    if constexpr (FUSED) part[(Q_RZ * R + threadIdx.x) * Gp + lb] = tot[NQ - 1];
  }
}

template <typename T, int R, bool FUSED, int H>
__global__ __launch_bounds__(kB) void kb_iter2(BMat m, BVec<T> v, const BSlot* slots, double* part, int G, int Gp,
                                               int k, int L) {
  pair_body<T, R, FUSED, H, true>(m, v, slots, part, G, Gp, k, L);
}

// the chunk's last iteration on 2 x 2 blocks: partials only
template <typename T, int R, int H>
__global__ __launch_bounds__(kB) void kb_iter2_last(BMat m, BVec<T> v, const BSlot* slots, double* part, int G,
                                                    int Gp, int k, int L) {
  pair_body<T, R, true, H, false>(m, v, slots, part, G, Gp, k, L);
}

// kb_residual on 2 x 2 blocks (same START / REPLACE forms and partials).
template <typename T, int R, bool START, int H>
__global__ __launch_bounds__(kB) void kb_residual2(BMat m, BVec<T> v, const BSlot* slots, double* part, int G,
                                                   int Gp, uint64_t mask, SlotScales cs, int L) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR, RPW = Gm::RPW;
  __shared__ double lds[3 * kWpb * R];
  const int lane = threadIdx.x % kW;
  const int j0 = (lane % LPR) * C, bsub = lane / LPR;
  bool on[C];
  double cc[C];
  bool any = false, all = true;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    if constexpr (START) {
      on[c] = ((mask >> (j0 + c)) & 1ull) != 0;
      cc[c] = cs.c[j0 + c];
    } else {
      on[c] = live(slots[j0 + c]);
      cc[c] = slots[j0 + c].c;
    }
    any |= on[c];
    all &= on[c];
  }
  const double* __restrict__ src = START ? v.phi : v.x;
  T* __restrict__ pprev = v.p[L - 1];
  const Ident ident;
  double acc[3][C] = {};
  if (any) {
    const Walk wk = task_walk(m.nb_slices * LPR, G);
    const int64_t first = wave_uniform(wk.t), end = wk.end, stride = wk.stride;
    const int64_t last_slice = m.nb_slices - 1;
    const int64_t last_row = m.n_slices * kW - 1;
    auto slice_of = [&](int64_t t) { return min((t * RPW) / kW, last_slice); };
    int32_t cu[H];
    Pack<double, 4> vu[H];
    Pack<double, C> ph[2], xv[2];
    double mi[2], kd[2];
    int64_t base, nb, ne;
    int w;
    auto fetch_idx = [&](int64_t t, int64_t sb) {
      const int64_t l = (t * RPW + bsub) % kW;
#pragma unroll
      for (int u = 0; u < H; ++u) cu[u] = m.pcol[sb + (int64_t)u * kW + l];
    };
    auto fetch_rest = [&](int64_t t, int64_t sb) {
      const int64_t brow = min(t * RPW + bsub, m.nb_slices * kW - 1), l = brow % kW;
#pragma unroll
      for (int u = 0; u < H; ++u) vu[u] = vload<double, 4>(m.pval64 + 4 * (sb + (int64_t)u * kW + l));
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int64_t row = min(2 * brow + r, last_row), idx = row * R + j0;
        ph[r] = vload<double, C>(v.phi + idx);
        if constexpr (!START) xv[r] = vload<double, C>(v.x + idx);
        mi[r] = m.mass[row];
        kd[r] = m.kdiag[row];
      }
    };
    {
      const int64_t s0 = slice_of(first);
      base = wave_uniform(m.psptr[s0]);
      w = (int)((wave_uniform(m.psptr[s0 + 1]) - base) / kW);
      fetch_idx(first, base);
      fetch_rest(first, base);
      const int64_t s1 = slice_of(first + stride);
      nb = m.psptr[s1];
      ne = m.psptr[s1 + 1];
    }
    for (int64_t t = first; t < end; t += stride) {
      const int64_t brow = t * RPW + bsub;
      const int64_t self = min(brow, m.nb - 1);
      Pack<double, C> gx[H][2];
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const int64_t off = (u < w ? (int64_t)cu[u] : self) * (2 * R) + j0;
        gx[u][0] = vload<double, C>(src + off);
        gx[u][1] = vload<double, C>(src + off + R);
      }
      const int64_t cbase = base;
      const int cw = w;
      const int64_t tn = t + stride < end ? t + stride : t;
      const int64_t s2 = slice_of(t + 2 * stride);
      const int64_t nb2 = m.psptr[s2], ne2 = m.psptr[s2 + 1];
      base = wave_uniform(nb);
      w = (int)((wave_uniform(ne) - base) / kW);
      fetch_idx(tn, base);
      nb = nb2;
      ne = ne2;
      double a[2][C] = {}, aa[2][C] = {};  // sum val x, sum |val| |x| (REPLACE)
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int u = 0; u < H; ++u) {
          const bool in = u < cw;
          const double v0 = in ? vu[u].v[2 * r] : 0.0, v1 = in ? vu[u].v[2 * r + 1] : 0.0;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            a[r][c] = fma(v0, gx[u][0].v[c], a[r][c]);
            a[r][c] = fma(v1, gx[u][1].v[c], a[r][c]);
            if constexpr (!START) {
              aa[r][c] = fma(fabs(v0), fabs(gx[u][0].v[c]), aa[r][c]);
              aa[r][c] = fma(fabs(v1), fabs(gx[u][1].v[c]), aa[r][c]);
            }
          }
        }
      if (cw > H) {
        if constexpr (START)
          pair_product<double, double, R, C, false, decltype(ident), H>(m, m.pval64, cbase, cw, brow % kW, j0, src,
                                                                         nullptr, ident, a, H);
        else
          pair_product_abs2<R, C, H>(m, cbase, cw, brow % kW, j0, src, a, aa, H);
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int64_t row = 2 * brow + r;
        const bool real = row < m.n;
        const int64_t idx = row * R + j0;
        if constexpr (START) {
          if (real) {
            Pack<double, C> xo = ph[r];
            Pack<T, C> zo, po = {};
            if (!all) {
              xo = vload<double, C>(v.x + idx);
              zo = vload<T, C>(v.z[0] + idx);
              po = vload<T, C>(pprev + idx);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
              if (!on[c]) continue;
              const double r64 = -cc[c] * (kd[r] * ph[r].v[c] + a[r][c]);
              const T rt = (T)r64;
              const T d = (T)(mi[r] + cc[c] * kd[r]);
              xo.v[c] = ph[r].v[c];
              zo.v[c] = rt / d;
              po.v[c] = (T)0;
              acc[0][c] += (double)rt * (double)zo.v[c];
              acc[1][c] += r64 * r64;
              acc[2][c] += (mi[r] * ph[r].v[c]) * (mi[r] * ph[r].v[c]);
            }
            vstore<double, C>(v.x + idx, xo);
            vstore<T, C>(v.z[0] + idx, zo);
            vstore<T, C>(pprev + idx, po);
          }
        } else {
          Pack<T, C> zv;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const double xf = xv[r].v[c];
            const double r64 = mi[r] * (ph[r].v[c] - xf) - cc[c] * (kd[r] * xf + a[r][c]);
            const T rt = (T)r64;
            const T d = (T)(mi[r] + cc[c] * kd[r]);
            zv.v[c] = rt / d;
            if (on[c] && real) {
              const double mag =
                  fabs(mi[r] * ph[r].v[c]) + fabs(mi[r] * xf) + cc[c] * (fabs(kd[r] * xf) + aa[r][c]);
              acc[0][c] += (double)rt * (double)zv.v[c];
              acc[1][c] += r64 * r64;
              acc[2][c] += mag * mag;
            }
          }
          if (real) vstore<T, C>(v.z[0] + idx, zv);
        }
      }
      fetch_rest(tn, base);
    }
  }
  double tot[3];
  col_sum<R, C, 3>(acc, lds, tot);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_RZ * R + threadIdx.x) * Gp + lb] = tot[0];
    part[(Q_RR * R + threadIdx.x) * Gp + lb] = tot[1];
    part[((START ? Q_BB : Q_FL) * R + threadIdx.x) * Gp + lb] = tot[2];
  }
}

// ------------------------------------------------------- complex tiles
// A complex tile (BatchWork::cx) runs Jacobi-COCG on complex-shifted
// first-order systems (M + sigma K) y = M phi, one per column pair: real
// columns 2j and 2j + 1 hold the real and imaginary parts of complex column
// j (vectors, alpha, beta, rho and sigma alike: sigma_re in slot 2j's c,
// sigma_im in slot 2j + 1's). K is real, so the gathered products are those
// of the real kernels, column by column; the per-row arithmetic is complex,
// with the symmetric bilinear form (no conjugation) in place of the inner
// product and the Hermitian norm |r|^2 for the stopping test. A lane owns
// an even number of columns, so both parts of a complex value are in one
// lane. The order-2 filter is the real part of one such solve per column.

// (r, i) += (ar + i ai)(br + i bi)
__device__ __forceinline__ void cmul_acc(double ar, double ai, double br, double bi, double& r, double& i) {
  r += ar * br - ai * bi;
  i += ar * bi + ai * br;
}

// the complex value of a gathered neighbour for the column pair at lane
// elements 2q, 2q + 1: z - alpha u (FUSED) or z + beta p (DIRECT)
template <typename T, int C, bool FUSED>
__device__ __forceinline__ void comb_cx(const T (&alpha)[C], const T (&beta)[C], int q, const Pack<T, C>& g0,
                                        const Pack<T, C>& g1, T& cr, T& ci) {
  const T xr = g1.v[2 * q], xi = g1.v[2 * q + 1], zr = g0.v[2 * q], zi = g0.v[2 * q + 1];
  if constexpr (FUSED) {
    const T ar = alpha[2 * q], ai = alpha[2 * q + 1];
    cr = fma(-ar, xr, fma(ai, xi, zr));
    ci = fma(-ar, xi, fma(-ai, xr, zi));
  } else {
    const T br = beta[2 * q], bi = beta[2 * q + 1];
    cr = fma(br, xr, fma(-bi, xi, zr));
    ci = fma(br, xi, fma(bi, xr, zi));
  }
}

// Entries k_begin .. w - 1 of a row (past the pipelined head), complex
// combiner (the row form's row_product).
template <typename T, int R, int C, bool FUSED, int U>
__device__ __forceinline__ void row_product_cx(const BMat& m, const T* __restrict__ val, int64_t base, int w,
                                               int64_t l, int j0, const T* __restrict__ x0,
                                               const T* __restrict__ x1, const T (&alpha)[C], const T (&beta)[C],
                                               T (&a)[C], int k_begin) {
  for (int k0 = k_begin; k0 < w; k0 += U) {
    int32_t cu[U];
    T vu[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = base + (int64_t)(k0 + u) * kW + l;
      cu[u] = m.col[e];
      const T vv = val[e];
      vu[u] = k0 + u < w ? vv : (T)0;
    }
    Pack<T, C> g0[U], g1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t off = (int64_t)cu[u] * R + j0;
      g0[u] = vload<T, C>(x0 + off);
      g1[u] = vload<T, C>(x1 + off);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < C / 2; ++q) {
        T cr, ci;
        comb_cx<T, C, FUSED>(alpha, beta, q, g0[u], g1[u], cr, ci);
        a[2 * q] = fma(vu[u], cr, a[2 * q]);
        a[2 * q + 1] = fma(vu[u], ci, a[2 * q + 1]);
      }
  }
}

// kb_iter for complex tiles (same forms, buffers, pipelining and partials,
// the z-and-u form of the scalar tiles; the partials are the real and
// imaginary parts of the complex sums, in the bilinear form x^T y that COCG
// uses, for which S is symmetric).
__device__ __forceinline__ void cfma(double ar, double ai, double br, double bi, double& r, double& i) {
  r = fma(ar, br, fma(-ai, bi, r));
  i = fma(ar, bi, fma(ai, br, i));
}

template <typename T, int R, bool FUSED, int H, bool KEEP>
__device__ __forceinline__ void cx_body(const BMat& m, const BVec<T>& v, const BSlot* slots, double* part, int G,
                                        int Gp, int k, int L) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR, RPW = Gm::RPW;
  static_assert(C % 2 == 0, "a lane holds whole complex values");
  constexpr int NQ = FUSED ? 4 : 3;
  __shared__ double lds[NQ * kWpb * R];
  const int lane = threadIdx.x % kW;
  const int j0 = (lane % LPR) * C, rsub = lane / LPR;
  T alpha[C], beta[C], cc[C];
  double c64[C];
  bool on[C];
  bool any = false;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const BSlot& sl = slots[j0 + c];
    on[c] = live(sl);
    alpha[c] = on[c] ? (T)sl.alpha : (T)0;
    beta[c] = on[c] ? (T)sl.beta : (T)0;
    cc[c] = (T)sl.c;
    c64[c] = sl.c;
    any |= on[c];
  }
  // buffers as in kb_iter: iteration k reads z[k - 1] (DIRECT: z[0]) and
  // writes z[k]; u_k in u[k & 1]; DIRECT reads the carried p_-1 in p[L - 1]
  const T* __restrict__ zin = v.z[FUSED ? k - 1 : 0];
  T* __restrict__ zout = v.z[k];
  const T* __restrict__ uin = v.u[(k + 1) & 1];
  T* __restrict__ uout = v.u[k & 1];
  const T* __restrict__ pin = v.p[L - 1];
  const T* __restrict__ g1src = FUSED ? uin : pin;
  const T* __restrict__ val = bval<T>(m);
  double acc[NQ][C] = {};
  if (__any(any)) {  // as kb_iter: the whole wave, the row's lanes share its entries
    const Walk wk = task_walk(m.n_slices * LPR, G);
    const int64_t first = wave_uniform(wk.t), end = wk.end, stride = wk.stride;
    const int64_t last_slice = m.n_slices - 1;
    auto slice_of = [&](int64_t t) { return min((t * RPW) / kW, last_slice); };
    constexpr int NL = (H + LPR - 1) / LPR;
    const int lc = lane % LPR;
    int32_t cu[H], cl[NL];
    T vu[H], vl[NL];
    Pack<T, C> zi, gi;  // own row: z and (FUSED) u or (DIRECT) p
    double mi, kd;
    int64_t base, nb, ne;
    int w;
    auto fetch_idx = [&](int64_t t, int64_t sb) {
      const int64_t l = (t * RPW + rsub) % kW;
#pragma unroll
      for (int i = 0; i < NL; ++i) cl[i] = m.col[sb + (int64_t)min(lc + i * LPR, H - 1) * kW + l];
    };
    auto share_idx = [&]() {
      unroll<H>([&](auto U) {
        constexpr int u = decltype(U)::value;
        if constexpr (LPR == 1) cu[u] = cl[u];
        else cu[u] = row_share<LPR, u % LPR>(cl[u / LPR]);
      });
    };
    auto share_val = [&]() {
      unroll<H>([&](auto U) {
        constexpr int u = decltype(U)::value;
        if constexpr (LPR == 1) vu[u] = vl[u];
        else vu[u] = row_share<LPR, u % LPR>(vl[u / LPR]);
      });
    };
    auto fetch_rest = [&](int64_t t, int64_t sb) {
      const int64_t row = min(t * RPW + rsub, m.n_slices * kW - 1), l = row % kW;
#pragma unroll
      for (int i = 0; i < NL; ++i) vl[i] = val[sb + (int64_t)min(lc + i * LPR, H - 1) * kW + l];
      const int64_t idx = row * R + j0;
      zi = vload<T, C>(zin + idx);
      gi = vload<T, C>(g1src + idx);
      mi = m.mass[row];
      kd = m.kdiag[row];
    };
    {
      const int64_t s0 = slice_of(first);
      base = wave_uniform(m.sptr[s0]);
      w = (int)((wave_uniform(m.sptr[s0 + 1]) - base) / kW);
      fetch_idx(first, base);
      fetch_rest(first, base);
      share_idx();
      const int64_t s1 = slice_of(first + stride);
      nb = m.sptr[s1];
      ne = m.sptr[s1 + 1];
    }
    for (int64_t t = first; t < end; t += stride) {
      const int64_t row = t * RPW + rsub;
      const int32_t self = (int32_t)min(row, m.n - 1);
      Pack<T, C> g0[H], g1[H];
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const int64_t off = (int64_t)(u < w ? cu[u] : self) * R + j0;
        g0[u] = vload<T, C>(zin + off);
        g1[u] = vload<T, C>(g1src + off);
      }
      const int64_t cbase = base;
      const int cw = w;
      const int64_t tn = t + stride < end ? t + stride : t;
      const int64_t s2 = slice_of(t + 2 * stride);
      const int64_t nb2 = m.sptr[s2], ne2 = m.sptr[s2 + 1];
      base = wave_uniform(nb);
      w = (int)((wave_uniform(ne) - base) / kW);
      fetch_idx(tn, base);
      nb = nb2;
      ne = ne2;
      share_val();
      T a[C] = {};
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const T vm = u < cw ? vu[u] : (T)0;
#pragma unroll
        for (int q = 0; q < C / 2; ++q) {
          T cr, ci;
          comb_cx<T, C, FUSED>(alpha, beta, q, g0[u], g1[u], cr, ci);
          a[2 * q] = fma(vm, cr, a[2 * q]);
          a[2 * q + 1] = fma(vm, ci, a[2 * q + 1]);
        }
      }
      if (cw > H)
        row_product_cx<T, R, C, FUSED, H>(m, val, cbase, cw, row % kW, j0, zin, g1src, alpha, beta, a, H);
      const bool real = row < m.n;
      const int64_t idx = row * R + j0;
      Pack<T, C> zn, un;
#pragma unroll
      for (int q = 0; q < C / 2; ++q) {
        const int e0 = 2 * q, e1 = 2 * q + 1;
        // d = diag(S) = M + sigma diag(K) (complex), padding rows 1
        const T dr = real ? (T)(mi + c64[e0] * kd) : (T)1, di = real ? (T)(c64[e1] * kd) : (T)0;
        const T gr = gi.v[e0], gim = gi.v[e1];
        T zr, zim;
        if constexpr (FUSED) {
          zr = fma(-alpha[e0], gr, fma(alpha[e1], gim, zi.v[e0]));
          zim = fma(-alpha[e0], gim, fma(-alpha[e1], gr, zi.v[e1]));
        } else {
          zr = zi.v[e0];
          zim = zi.v[e1];
        }
        // d^-1 sigma K_off x (x = z' when FUSED, p' when DIRECT)
        const T sr = cc[e0] * a[e0] - cc[e1] * a[e1], si = cc[e0] * a[e1] + cc[e1] * a[e0];
        const T rden = over((T)1, dr * dr + di * di);
        const T wr = (sr * dr + si * di) * rden, wi = (si * dr - sr * di) * rden;
        T ur, uim, pr = 0, pim = 0;
        if constexpr (FUSED) {
          ur = fma(beta[e0], gr, fma(-beta[e1], gim, zr + wr));
          uim = fma(beta[e0], gim, fma(beta[e1], gr, zim + wi));
        } else {
          pr = fma(beta[e0], gr, fma(-beta[e1], gim, zr));
          pim = fma(beta[e0], gim, fma(beta[e1], gr, zim));
          ur = pr + wr;
          uim = pim + wi;
        }
        zn.v[e0] = zr;
        zn.v[e1] = zim;
        un.v[e0] = ur;
        un.v[e1] = uim;
        // the row's weight d (0 where the row or the column pair does not
        // count); d u and d z are formed in T (they are r-sized) and each
        // complex product is summed in FP64 with FMAs
        const bool use = on[e0] && real;
        const T wr0 = use ? dr : (T)0, wi0 = use ? di : (T)0;
        const double dur = (double)(wr0 * ur - wi0 * uim), dui = (double)(wr0 * uim + wi0 * ur);
        const double zr64 = (double)zr, zi64 = (double)zim, ur64 = (double)ur, ui64 = (double)uim;
        if constexpr (FUSED) {
          // (q_k-1, z_k) = sum (d u_k-1) z_k
          const double qr = (double)(wr0 * gr - wi0 * gim), qi = (double)(wr0 * gim + wi0 * gr);
          cfma(qr, qi, zr64, zi64, acc[0][e0], acc[0][e1]);
          const double dzr = (double)(wr0 * zr - wi0 * zim), dzi = (double)(wr0 * zim + wi0 * zr);
          cfma(dzr, dzi, zr64, zi64, acc[NQ - 1][e0], acc[NQ - 1][e1]);
        } else {
          cfma(dur, dui, (double)pr, (double)pim, acc[0][e0], acc[0][e1]);
        }
        cfma(dur, dui, zr64, zi64, acc[1][e0], acc[1][e1]);
        cfma(dur, dui, ur64, ui64, acc[2][e0], acc[2][e1]);
      }
      if constexpr (KEEP) {
        if (real) {
          vstore<T, C>(uout + idx, un);
          if constexpr (FUSED) vstore<T, C>(zout + idx, zn);
        }
      }
      fetch_rest(tn, base);
      share_idx();
    }
  }
  double tot[NQ];
  col_sum<R, C, NQ>(acc, lds, tot);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_PQ * R + threadIdx.x) * Gp + lb] = tot[0];
    part[(Q_ZU * R + threadIdx.x) * Gp + lb] = tot[1];
    part[(Q_UU * R + threadIdx.x) * Gp + lb] = tot[2];
    if constexpr (FUSED) part[(Q_RZ * R + threadIdx.x) * Gp + lb] = tot[NQ - 1];
  }
}

template <typename T, int R, bool FUSED, int H>
__global__ __launch_bounds__(kB) void kbc_iter(BMat m, BVec<T> v, const BSlot* slots, double* part, int G, int Gp,
                                               int k, int L) {
  cx_body<T, R, FUSED, H, true>(m, v, slots, part, G, Gp, k, L);
}

// the chunk's last iteration of a complex tile: partials only
template <typename T, int R, int H>
__global__ __launch_bounds__(kB) void kbc_iter_last(BMat m, BVec<T> v, const BSlot* slots, double* part, int G,
                                                    int Gp, int k, int L) {
  cx_body<T, R, true, H, false>(m, v, slots, part, G, Gp, k, L);
}

// The complex tile's x update at the chunk's end, as kb_xupdate's
// form in complex FP64: z_L-1 = z_L-2 - alpha_L-2 u_L-2 (as the last
// iteration formed it), p_k = z_k + beta_k p_k-1 from the carried p_-1, x
// += sum_k alpha_k p_k, and p_L-1 carried (pairs that did not iterate keep
// theirs).
template <typename T, int R, int L>
__global__ __launch_bounds__(kB) void kbc_xupdate(BMat m, BVec<T> v, const BSlot* slots, int G) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR, RPW = Gm::RPW;
  const int lane = threadIdx.x % kW;
  const int j0 = (lane % LPR) * C, rsub = lane / LPR;
  double ah[L][C], bh[L][C];
  bool moved[C];
  bool any = false;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const BSlot& sl = slots[j0 + c];
    moved[c] = false;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      ah[i][c] = sl.alpha_hist[i];
      bh[i][c] = sl.beta_hist[i];
      moved[c] |= ah[i][c] != 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < C / 2; ++q) {
    moved[2 * q] = moved[2 * q + 1] = moved[2 * q] || moved[2 * q + 1];
    any |= moved[2 * q];
  }
  if (!any) return;
  for (Walk wk = task_walk(m.n_slices * LPR, G); wk.t < wk.end; wk.t += wk.stride) {
    const int64_t row = wk.t * RPW + rsub;
    if (row >= m.n) continue;
    const int64_t idx = row * R + j0;
    Pack<T, C> zk[L];
#pragma unroll
    for (int i = 0; i < L - 1; ++i) zk[i] = vload<T, C>(v.z[i] + idx);
    zk[L - 1] = vload<T, C>(v.u[(L - 2) & 1] + idx);
    Pack<double, C> xv = vload<double, C>(v.x + idx);
    Pack<T, C> pc = vload<T, C>(v.p[L - 1] + idx);
#pragma unroll
    for (int q = 0; q < C / 2; ++q) {
      const int e0 = 2 * q, e1 = 2 * q + 1;
      {
        const T ar = (T)ah[L - 2][e0], ai = (T)ah[L - 2][e1];
        const T ur = zk[L - 1].v[e0], ui = zk[L - 1].v[e1];
        zk[L - 1].v[e0] = fma(-ar, ur, fma(ai, ui, zk[L - 2].v[e0]));
        zk[L - 1].v[e1] = fma(-ar, ui, fma(-ai, ur, zk[L - 2].v[e1]));
      }
      double pr = (double)pc.v[e0], pi = (double)pc.v[e1];
#pragma unroll
      for (int i = 0; i < L; ++i) {
        const double br = bh[i][e0], bi = bh[i][e1];
        const double nr = fma(br, pr, fma(-bi, pi, (double)zk[i].v[e0]));
        const double ni = fma(br, pi, fma(bi, pr, (double)zk[i].v[e1]));
        pr = nr;
        pi = ni;
        cfma(ah[i][e0], ah[i][e1], pr, pi, xv.v[e0], xv.v[e1]);
      }
      if (moved[e0]) {
        pc.v[e0] = (T)pr;
        pc.v[e1] = (T)pi;
      }
    }
    vstore<T, C>(v.p[L - 1] + idx, pc);
    vstore<double, C>(v.x + idx, xv);
  }
}

// kb_residual for complex tiles: START (x = phi, p = 0, r0 = M phi - S phi =
// -sigma K phi) and REPLACE (r = M phi - S x in FP64), z = r / diag(S), with
// the partials of (r, z) (complex), |r|^2 and ||M phi||^2 or the
// attainable-accuracy norm (both parts of a column pair add up).
template <typename T, int R, bool START, int H>
__global__ __launch_bounds__(kB) void kbc_residual(BMat m, BVec<T> v, const BSlot* slots, double* part, int G,
                                                   int Gp, uint64_t mask, SlotScales cs, int L) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR, RPW = Gm::RPW;
  static_assert(C % 2 == 0, "a lane holds whole complex values");
  __shared__ double lds[3 * kWpb * R];
  const int lane = threadIdx.x % kW;
  const int j0 = (lane % LPR) * C, rsub = lane / LPR;
  bool on[C];
  double cc[C];
  bool any = false, all = true;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    if constexpr (START) {
      on[c] = ((mask >> (j0 + c)) & 1ull) != 0;
      cc[c] = cs.c[j0 + c];
    } else {
      on[c] = live(slots[j0 + c]);
      cc[c] = slots[j0 + c].c;
    }
    any |= on[c];
    all &= on[c];
  }
  const double* __restrict__ src = START ? v.phi : v.x;
  T* __restrict__ pprev = v.p[L - 1];
  const Ident ident;
  double acc[3][C] = {};
  if (any) {
    const Walk wk = task_walk(m.n_slices * LPR, G);
    const int64_t first = wave_uniform(wk.t), end = wk.end, stride = wk.stride;
    const int64_t last_slice = m.n_slices - 1;
    auto slice_of = [&](int64_t t) { return min((t * RPW) / kW, last_slice); };
    int32_t cu[H];
    double vu[H];
    Pack<double, C> ph, xv;
    double mi, kd;
    int64_t base, nb, ne;
    int w;
    auto fetch_idx = [&](int64_t t, int64_t sb) {
      const int64_t l = (t * RPW + rsub) % kW;
#pragma unroll
      for (int u = 0; u < H; ++u) cu[u] = m.col[sb + (int64_t)u * kW + l];
    };
    auto fetch_rest = [&](int64_t t, int64_t sb) {
      const int64_t row = min(t * RPW + rsub, m.n_slices * kW - 1), l = row % kW;
#pragma unroll
      for (int u = 0; u < H; ++u) vu[u] = m.val64[sb + (int64_t)u * kW + l];
      const int64_t idx = row * R + j0;
      ph = vload<double, C>(v.phi + idx);
      if constexpr (!START) xv = vload<double, C>(v.x + idx);
      mi = m.mass[row];
      kd = m.kdiag[row];
    };
    {
      const int64_t s0 = slice_of(first);
      base = wave_uniform(m.sptr[s0]);
      w = (int)((wave_uniform(m.sptr[s0 + 1]) - base) / kW);
      fetch_idx(first, base);
      fetch_rest(first, base);
      const int64_t s1 = slice_of(first + stride);
      nb = m.sptr[s1];
      ne = m.sptr[s1 + 1];
    }
    for (int64_t t = first; t < end; t += stride) {
      const int64_t row = t * RPW + rsub;
      const int32_t self = (int32_t)min(row, m.n - 1);
      Pack<double, C> gx[H];
#pragma unroll
      for (int u = 0; u < H; ++u) gx[u] = vload<double, C>(src + (int64_t)(u < w ? cu[u] : self) * R + j0);
      const int64_t cbase = base;
      const int cw = w;
      const int64_t tn = t + stride < end ? t + stride : t;
      const int64_t s2 = slice_of(t + 2 * stride);
      const int64_t nb2 = m.sptr[s2], ne2 = m.sptr[s2 + 1];
      base = wave_uniform(nb);
      w = (int)((wave_uniform(ne) - base) / kW);
      fetch_idx(tn, base);
      nb = nb2;
      ne = ne2;
      double a[C] = {}, aa[C] = {};
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const double vm = u < cw ? vu[u] : 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          a[c] = fma(vm, gx[u].v[c], a[c]);
          if constexpr (!START) aa[c] = fma(fabs(vm), fabs(gx[u].v[c]), aa[c]);
        }
      }
      if (cw > H) {
        if constexpr (START)
          row_product<double, double, R, C, false, decltype(ident), H>(m, m.val64, cbase, cw, row % kW, j0, src,
                                                                        nullptr, ident, a, H);
        else
          row_product_abs2<R, C, H>(m, cbase, cw, row % kW, j0, src, a, aa, H);
      }
      const bool real = row < m.n;
      const int64_t idx = row * R + j0;
      if constexpr (START) {
        if (real) {
          Pack<double, C> xo = ph;
          Pack<T, C> zo, po = {};
          if (!all) {
            xo = vload<double, C>(v.x + idx);
            zo = vload<T, C>(v.z[0] + idx);
            po = vload<T, C>(pprev + idx);
          }
#pragma unroll
          for (int q = 0; q < C / 2; ++q) {
            const int e0 = 2 * q, e1 = 2 * q + 1;
            if (!on[e0]) continue;
            const double tr = kd * ph.v[e0] + a[e0], ti = kd * ph.v[e1] + a[e1];
            const double rr64 = -(cc[e0] * tr - cc[e1] * ti), ri64 = -(cc[e0] * ti + cc[e1] * tr);
            const T rtr = (T)rr64, rti = (T)ri64;
            const T dr = (T)(mi + cc[e0] * kd), di = (T)(cc[e1] * kd);
            const T den = dr * dr + di * di;
            const T zr = (rtr * dr + rti * di) / den, zim = (rti * dr - rtr * di) / den;
            xo.v[e0] = ph.v[e0];
            xo.v[e1] = ph.v[e1];
            zo.v[e0] = zr;
            zo.v[e1] = zim;
            po.v[e0] = (T)0;
            po.v[e1] = (T)0;
            cmul_acc((double)rtr, (double)rti, (double)zr, (double)zim, acc[0][e0], acc[0][e1]);
            acc[1][e0] += rr64 * rr64;
            acc[1][e1] += ri64 * ri64;
            acc[2][e0] += (mi * ph.v[e0]) * (mi * ph.v[e0]);
            acc[2][e1] += (mi * ph.v[e1]) * (mi * ph.v[e1]);
          }
          vstore<double, C>(v.x + idx, xo);
          vstore<T, C>(v.z[0] + idx, zo);
          vstore<T, C>(pprev + idx, po);
        }
      } else {
        Pack<T, C> zv;
#pragma unroll
        for (int q = 0; q < C / 2; ++q) {
          const int e0 = 2 * q, e1 = 2 * q + 1;
          const double xr = xv.v[e0], xim = xv.v[e1];
          const double tr = kd * xr + a[e0], ti = kd * xim + a[e1];
          const double rr64 = mi * (ph.v[e0] - xr) - (cc[e0] * tr - cc[e1] * ti);
          const double ri64 = mi * (ph.v[e1] - xim) - (cc[e0] * ti + cc[e1] * tr);
          const T rtr = (T)rr64, rti = (T)ri64;
          const T dr = (T)(mi + cc[e0] * kd), di = (T)(cc[e1] * kd);
          const T den = dr * dr + di * di;
          zv.v[e0] = (rtr * dr + rti * di) / den;
          zv.v[e1] = (rti * dr - rtr * di) / den;
          if (on[e0] && real) {
            const double sabs = sqrt(cc[e0] * cc[e0] + cc[e1] * cc[e1]);
            const double m0 = fabs(mi * ph.v[e0]) + fabs(mi * xr) + sabs * (fabs(kd * xr) + aa[e0]);
            const double m1 = fabs(mi * ph.v[e1]) + fabs(mi * xim) + sabs * (fabs(kd * xim) + aa[e1]);
            cmul_acc((double)rtr, (double)rti, (double)zv.v[e0], (double)zv.v[e1], acc[0][e0], acc[0][e1]);
            acc[1][e0] += rr64 * rr64;
            acc[1][e1] += ri64 * ri64;
            acc[2][e0] += m0 * m0;
            acc[2][e1] += m1 * m1;
          }
        }
        if (real) vstore<T, C>(v.z[0] + idx, zv);
      }
      fetch_rest(tn, base);
    }
  }
  double tot[3];
  col_sum<R, C, 3>(acc, lds, tot);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_RZ * R + threadIdx.x) * Gp + lb] = tot[0];
    part[(Q_RR * R + threadIdx.x) * Gp + lb] = tot[1];
    part[((START ? Q_BB : Q_FL) * R + threadIdx.x) * Gp + lb] = tot[2];
  }
}

// End of a column: partials of sum M x^2 (kb_out writes x out). A column
// stops right after a replacement, whose FP64 true residual is that of this
// very x, so no residual is formed here.
template <typename T, int R>
__global__ __launch_bounds__(kB) void kb_finish(BMat m, BVec<T> v, const BSlot* slots, double* part, int G, int Gp,
                                                uint64_t mask) {
  using Gm = Geo<T, R>;
  constexpr int C = Gm::C, LPR = Gm::LPR, RPW = Gm::RPW;
  __shared__ double lds[1 * kWpb * R];
  const int lane = threadIdx.x % kW;
  const int j0 = (lane % LPR) * C, rsub = lane / LPR;
  bool on[C];
  bool any = false;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    on[c] = ((mask >> (j0 + c)) & 1ull) != 0;
    any |= on[c];
  }
  // at a chunk boundary x holds the whole solution (the chunk's x update
  // has run)
  double acc[1][C] = {};
  if (any) {
    for (Walk wk = task_walk(m.n_slices * LPR, G); wk.t < wk.end; wk.t += wk.stride) {
      const int64_t row = wk.t * RPW + rsub;
      if (row >= m.n) continue;
      const int64_t idx = row * R + j0;
      const Pack<double, C> xv = vload<double, C>(v.x + idx);
      const double mi = m.mass[row];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (!on[c]) continue;
        const double xi = xv.v[c];
        acc[0][c] += mi * xi * xi;
      }
    }
  }
  double tot[1];
  col_sum<R, C, 1>(acc, lds, tot);
  if (threadIdx.x < R) part[(Q_EN * R + threadIdx.x) * Gp + lblock(G)] = tot[0];
}

// x of the columns in 'mask' to the caller's numbering, one caller entry per
// thread: coalesced writes (0 where there is no dof). Each thread loads all
// of its row's wanted columns before it stores any: as far as the compiler
// knows a store could change x, so interleaved loads would each wait for
// the store before them, and the row's lines would be fetched again.
template <int R>
__global__ void kb_out(const double* __restrict__ x, OutPtrs out, uint64_t mask, const int32_t* __restrict__ row_of,
                       int64_t L) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= L) return;
  const int64_t i = row_of[v];
  if constexpr (R == 1) {
    if (mask & 1ull) out.p[0][v] = i >= 0 ? x[i] : 0.0;
  } else {
    constexpr int NP = R / 2;
    Pack<double, 2> xv[NP];
#pragma unroll
    for (int jp = 0; jp < NP; ++jp) {
      xv[jp] = {};
      if (i >= 0 && ((mask >> (2 * jp)) & 3ull)) xv[jp] = vload<double, 2>(x + i * R + 2 * jp);
    }
#pragma unroll
    for (int jp = 0; jp < NP; ++jp) {
      const uint64_t bits = (mask >> (2 * jp)) & 3ull;
      if (bits & 1ull) out.p[2 * jp][v] = xv[jp].v[0];
      if (bits & 2ull) out.p[2 * jp + 1][v] = xv[jp].v[1];
    }
  }
}

// Columns of one tile into another of a different width (same precision), at
// a chunk boundary: z, the chunk's last direction p[L - 1] (the next
// chunk's first iteration forms u from it, so u is not carried), x and phi of
// each mapped column, one row per thread.
struct ColMap {
  int n;
  int src[64], dst[64];
};

template <typename T>
__global__ void kb_move_cols(const T* __restrict__ zs, const T* __restrict__ ps, const double* __restrict__ xs,
                             const double* __restrict__ fs, int RS, T* __restrict__ zd, T* __restrict__ pd,
                             double* __restrict__ xd, double* __restrict__ fd, int RD, ColMap map, int64_t n_pad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  for (int c = 0; c < map.n; ++c) {
    const int64_t a = i * RS + map.src[c], b = i * RD + map.dst[c];
    zd[b] = zs[a];
    pd[b] = ps[a];
    xd[b] = xs[a];
    fd[b] = fs[a];
  }
}

// slots of the moved columns; the other slots of the destination are idle
__global__ void kf_move_slots(const BSlot* __restrict__ src, BSlot* __restrict__ dst, int RD, ColMap map) {
  const int j = threadIdx.x;
  if (j >= RD) return;
  int from = -1;
  for (int c = 0; c < map.n; ++c)
    if (map.dst[c] == j) from = map.src[c];
  if (from >= 0) {
    dst[j] = src[from];
  } else {
    dst[j].active = 0;
    dst[j].done = 0;
  }
}

// fields -> the columns in 'mask' of the rows x R field array, one row per
// thread (the new columns of a row are written together). The fields are in
// the caller's numbering (read through entity) or, 'internal', already in
// row order (contiguous reads).
__global__ void kb_gather_cols(FieldPtrs src, uint64_t mask, const int64_t* __restrict__ entity, int64_t n, int R,
                               int internal, double* __restrict__ phi, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t e = internal ? i : entity[i];
  bool bad = false;
  if (R == 1) {
    if (mask & 1ull) {
      const double v = src.p[0][e];
      bad = !isfinite(v);
      phi[i] = v;
    }
  } else {
    for (int j = 0; j < R; j += 2) {
      const uint64_t bits = (mask >> j) & 3ull;
      if (!bits) continue;
      Pack<double, 2> pv;
      if (bits == 3ull) {
        pv.v[0] = src.p[j][e];
        pv.v[1] = src.p[j + 1][e];
        bad |= !isfinite(pv.v[0]) || !isfinite(pv.v[1]);
        vstore<double, 2>(phi + i * R + j, pv);
      } else {
        const int jj = bits == 1ull ? j : j + 1;
        const double vv = src.p[jj][e];
        bad |= !isfinite(vv);
        phi[i * R + jj] = vv;
      }
    }
  }
  if (bad) atomicOr(flag, 1);
}

// n_fields fields in the caller's numbering (stride L) -> row order (stride
// n_pad), one field per grid row; non-finite wet entries raise the flag
__global__ void kb_permute(const double* __restrict__ src, int64_t L, const int64_t* __restrict__ entity, int64_t n,
                           int64_t n_pad, double* __restrict__ dst, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t f = blockIdx.y;
  const double v = src[f * L + entity[i]];
  if (!isfinite(v)) atomicOr(flag, 1);
  dst[f * n_pad + i] = v;
}

// caller numbering -> column j of the rows x R field array
__global__ void kb_gather(const double* __restrict__ src, const int64_t* __restrict__ entity, int64_t n, int R,
                          int j, double* __restrict__ phi, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = src[entity[i]];
  if (!isfinite(v)) atomicOr(flag, 1);
  phi[i * R + j] = v;
}

// Pseudo-random column in [-1, 1) for timing trials: splitmix64 (Vigna) of
// the row index and a seed.
__global__ void kb_synth(int64_t n, int R, int j, uint64_t seed, double* __restrict__ phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t x = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  phi[i * R + j] = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// ------------------------------------------------------------ finalizers
__device__ __forceinline__ double fin_sum(const double* a, int G, double* lds) {
  double s = 0.0;
  for (int i = threadIdx.x; i < G; i += kFinThreads) s += a[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, kW);
  const int lane = threadIdx.x % kW, wid = threadIdx.x / kW;
  if (lane == 0) lds[wid] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kFinThreads / kW; ++w) t += lds[w];
  __syncthreads();
  return t;
}

// After iteration k of a chunk (kb_iter, kb_iter2): alpha_k = rho_k / (p,
// q), kept in the column's alpha history at position k (0 for columns not
// iterating) beside the beta the launch used; the next rho from the
// recurrence rho - 2 alpha (q, z) + alpha^2 (q, d^-1 q), and beta = next rho
// / rho_k for the next launch. rho_k is the exact (r, z) of the z the launch
// formed (k >= 1), or that of the replacement or start (k = 0). (p, q) is
// the launch's partial (k = 0), or (z, q) + beta ((q_prev, z) + beta (p,
// q)_prev) from the partials of the z-and-u form (k >= 1). No stopping
// test: a column is tested on its replaced FP64 residual only, in
// kf_replace.
__global__ __launch_bounds__(kFinThreads) void kf_step(BSlot* slots, const double* part, int G, int Gp, int R,
                                                        int k) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  BSlot& s = slots[j];
  if (!live(s)) {
    if (threadIdx.x == 0) {
      s.alpha_hist[k] = 0.0;
      s.beta_hist[k] = 0.0;
    }
    return;
  }
  const double p0 = fin_sum(part + (Q_PQ * R + j) * Gp, G, lds);
  const double zu = fin_sum(part + (Q_ZU * R + j) * Gp, G, lds);
  const double uu = fin_sum(part + (Q_UU * R + j) * Gp, G, lds);
  const double rz = k > 0 ? fin_sum(part + (Q_RZ * R + j) * Gp, G, lds) : 0.0;
  if (threadIdx.x == 0) {
    const double b = s.beta;
    const double pq = k > 0 ? zu + b * (p0 + b * s.pq) : p0;
    const double rho = k > 0 ? rz : s.rho;
    const double a = rho / pq;
    s.iters += 1;
    s.beta_hist[k] = b;
    if (!(pq > 0.0) || !isfinite(a)) {
      s.done = 2;
      s.alpha_hist[k] = 0.0;
    } else {
      const double next = rho - 2.0 * a * zu + a * a * uu;
      s.rho = rho;
      s.pq = pq;
      s.alpha = a;
      s.alpha_hist[k] = a;
      s.beta = next / rho;
      s.rr_true = 0;
    }
  }
}

// After the chunk's x update and its FP64 replacement pass: rho and beta
// from the replaced residual, and the stopping test
__global__ __launch_bounds__(kFinThreads) void kf_replace(BSlot* slots, const double* part, int G, int Gp, int R,
                                                           int max_iter) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  BSlot& s = slots[j];
  if (!live(s)) return;
  const double rz = fin_sum(part + (Q_RZ * R + j) * Gp, G, lds);
  const double rr = fin_sum(part + (Q_RR * R + j) * Gp, G, lds);
  const double fl = fin_sum(part + (Q_FL * R + j) * Gp, G, lds);
  if (threadIdx.x == 0) {
    s.rho_prev = s.rho;
    s.rho = rz;
    s.beta = rz / s.rho_prev;
    s.rr = rr;
    s.rr_true = 1;
    s.updates += 1;
    const double floor2 = fl * (kFloor * kU) * (kFloor * kU);
    if (rr <= fmax(s.tol2, floor2)) s.done = 1;
    else if (s.iters >= max_iter) s.done = 3;
  }
}

// start of a column (after the start pass)
__global__ __launch_bounds__(kFinThreads) void kf_init(BSlot* slots, const double* part, int G, int Gp, int R, uint64_t mask,
                                                        double rtol, SlotScales cs) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  if (!((mask >> j) & 1ull)) return;
  BSlot& s = slots[j];
  const double rz = fin_sum(part + (Q_RZ * R + j) * Gp, G, lds);
  const double rr = fin_sum(part + (Q_RR * R + j) * Gp, G, lds);
  const double bb = fin_sum(part + (Q_BB * R + j) * Gp, G, lds);
  if (threadIdx.x == 0) {
    s.c = cs.c[j];
    s.rho = rz;
    s.rho_prev = INFINITY;
    s.beta = 0.0;
    s.alpha = 0.0;
    s.rr = rr;
    s.bb = bb;
    s.tol2 = rtol * rtol * bb;
    s.iters = 0;
    s.updates = 0;
    s.rr_true = 1;
    s.active = 1;
    s.done = rr <= s.tol2 ? 1 : 0;
  }
}

__global__ void kf_release(BSlot* slots, int R, uint64_t mask) {
  const int j = threadIdx.x;
  if (j < R && ((mask >> j) & 1ull)) {
    slots[j].active = 0;
    slots[j].done = 0;
  }
}

__global__ __launch_bounds__(kFinThreads) void kf_finish(BSlot* slots, const double* part, int G, int Gp, int R,
                                                          uint64_t mask) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  if (!((mask >> j) & 1ull)) return;
  BSlot& s = slots[j];
  const double en = fin_sum(part + (Q_EN * R + j) * Gp, G, lds);
  if (threadIdx.x == 0) {
    s.res2 = s.rr;  // the FP64 true residual of the last replacement
    s.energy2 = en;
  }
}

// Finalizers of complex tiles: block q handles the column pair (2q, 2q + 1)
// and keeps both slots' counters and flags equal.
__device__ __forceinline__ void cdiv(double ar, double ai, double br, double bi, double& r, double& i) {
  const double den = br * br + bi * bi;
  r = (ar * br + ai * bi) / den;
  i = (ai * br - ar * bi) / den;
}

__global__ __launch_bounds__(kFinThreads) void kfc_step(BSlot* slots, const double* part, int G, int Gp, int R,
                                                         int k) {
  __shared__ double lds[kFinThreads / kW];
  const int j = 2 * blockIdx.x;
  BSlot& s = slots[j];
  BSlot& t = slots[j + 1];
  if (!live(s)) {
    if (threadIdx.x == 0) s.alpha_hist[k] = t.alpha_hist[k] = s.beta_hist[k] = t.beta_hist[k] = 0.0;
    return;
  }
  const double p0r = fin_sum(part + (Q_PQ * R + j) * Gp, G, lds), p0i = fin_sum(part + (Q_PQ * R + j + 1) * Gp, G, lds);
  const double zur = fin_sum(part + (Q_ZU * R + j) * Gp, G, lds), zui = fin_sum(part + (Q_ZU * R + j + 1) * Gp, G, lds);
  const double uur = fin_sum(part + (Q_UU * R + j) * Gp, G, lds), uui = fin_sum(part + (Q_UU * R + j + 1) * Gp, G, lds);
  const double rzr = k > 0 ? fin_sum(part + (Q_RZ * R + j) * Gp, G, lds) : 0.0;
  const double rzi = k > 0 ? fin_sum(part + (Q_RZ * R + j + 1) * Gp, G, lds) : 0.0;
  if (threadIdx.x == 0) {
    // (p, q) = (z, q) + beta ((q_prev, z) + beta (p, q)_prev) for k >= 1 (as kf_step)
    const double b0r = s.beta, b0i = t.beta;
    double pqr = p0r, pqi = p0i;
    if (k > 0) {
      const double hr = p0r + (b0r * s.pq - b0i * t.pq), hi = p0i + (b0r * t.pq + b0i * s.pq);
      pqr = zur + (b0r * hr - b0i * hi);
      pqi = zui + (b0r * hi + b0i * hr);
    }
    s.beta_hist[k] = b0r;
    t.beta_hist[k] = b0i;
    const double rr = k > 0 ? rzr : s.rho, ri = k > 0 ? rzi : t.rho;
    double ar, ai;
    cdiv(rr, ri, pqr, pqi, ar, ai);
    s.iters += 1;
    t.iters += 1;
    if (!(pqr * pqr + pqi * pqi > 0.0) || !isfinite(ar) || !isfinite(ai)) {
      s.done = t.done = 2;
      s.alpha_hist[k] = t.alpha_hist[k] = 0.0;
    } else {
      // next rho = rho - 2 alpha (q, z) + alpha^2 (q, d^-1 q)
      const double a2r = ar * ar - ai * ai, a2i = 2.0 * ar * ai;
      const double nr = rr - 2.0 * (ar * zur - ai * zui) + (a2r * uur - a2i * uui);
      const double ni = ri - 2.0 * (ar * zui + ai * zur) + (a2r * uui + a2i * uur);
      double br, bi;
      cdiv(nr, ni, rr, ri, br, bi);
      s.rho = rr;
      t.rho = ri;
      s.pq = pqr;
      t.pq = pqi;
      s.alpha = ar;
      t.alpha = ai;
      s.alpha_hist[k] = ar;
      t.alpha_hist[k] = ai;
      s.beta = br;
      t.beta = bi;
      s.rr_true = t.rr_true = 0;
    }
  }
}

// A column pair whose FP64 true residual stops falling (mixed precision at
// the tightened tolerance can stall near it) restarts its directions once
// (beta = 0) after two chunk ends without a 10% fall, stops as converged
// after four if it meets the plain rtol on the shifted system (the
// attainable accuracy; the tightened target is then out of reach), and as
// not converged after 32.
__global__ __launch_bounds__(kFinThreads) void kfc_replace(BSlot* slots, const double* part, int G, int Gp, int R,
                                                            int max_iter, double g) {
  __shared__ double lds[kFinThreads / kW];
  const int j = 2 * blockIdx.x;
  BSlot& s = slots[j];
  BSlot& t = slots[j + 1];
  if (!live(s)) return;
  const double rzr = fin_sum(part + (Q_RZ * R + j) * Gp, G, lds), rzi = fin_sum(part + (Q_RZ * R + j + 1) * Gp, G, lds);
  const double rr = fin_sum(part + (Q_RR * R + j) * Gp, G, lds) + fin_sum(part + (Q_RR * R + j + 1) * Gp, G, lds);
  const double fl = fin_sum(part + (Q_FL * R + j) * Gp, G, lds) + fin_sum(part + (Q_FL * R + j + 1) * Gp, G, lds);
  if (threadIdx.x == 0) {
    s.rho_prev = s.rho;
    t.rho_prev = t.rho;
    double br, bi;
    cdiv(rzr, rzi, s.rho_prev, t.rho_prev, br, bi);
    s.rho = rzr;
    t.rho = rzi;
    s.beta = br;
    t.beta = bi;
    s.rr = t.rr = rr;
    s.rr_true = t.rr_true = 1;
    s.updates += 1;
    t.updates += 1;
    const double floor2 = fl * (kFloor * kU) * (kFloor * kU);
    if (rr < 0.9 * s.rr_best) {
      s.rr_best = t.rr_best = rr;
      s.stall = t.stall = 0;
    } else {
      s.stall = t.stall = s.stall + 1;
    }
    const double f = 1.0 + sqrt(s.c * s.c + t.c * t.c) * g;  // tol2 = (rtol / f)^2 bb
    if (rr <= fmax(s.tol2, floor2)) {
      s.done = t.done = 1;
    } else if (s.stall >= 4 && rr <= s.tol2 * f * f) {
      s.done = t.done = 1;
    } else if (s.iters >= max_iter || s.stall >= 32) {
      s.done = t.done = 3;
    } else if (s.stall == 2) {
      s.beta = t.beta = 0.0;
    }
  }
}

__global__ __launch_bounds__(kFinThreads) void kfc_init(BSlot* slots, const double* part, int G, int Gp, int R,
                                                         uint64_t mask, double rtol, SlotScales cs, double g) {
  __shared__ double lds[kFinThreads / kW];
  const int j = 2 * blockIdx.x;
  if (!((mask >> j) & 1ull)) return;
  BSlot& s = slots[j];
  BSlot& t = slots[j + 1];
  const double rzr = fin_sum(part + (Q_RZ * R + j) * Gp, G, lds), rzi = fin_sum(part + (Q_RZ * R + j + 1) * Gp, G, lds);
  const double rr = fin_sum(part + (Q_RR * R + j) * Gp, G, lds) + fin_sum(part + (Q_RR * R + j + 1) * Gp, G, lds);
  const double bb = fin_sum(part + (Q_BB * R + j) * Gp, G, lds) + fin_sum(part + (Q_BB * R + j + 1) * Gp, G, lds);
  if (threadIdx.x == 0) {
    s.c = cs.c[j];
    t.c = cs.c[j + 1];
    s.rho = rzr;
    t.rho = rzi;
    s.rho_prev = t.rho_prev = INFINITY;
    s.beta = t.beta = 0.0;
    s.alpha = t.alpha = 0.0;
    s.rr = t.rr = rr;
    s.bb = t.bb = bb;
    const double tol = rtol / (1.0 + sqrt(cs.c[j] * cs.c[j] + cs.c[j + 1] * cs.c[j + 1]) * g);
    s.tol2 = t.tol2 = tol * tol * bb;
    s.iters = t.iters = 0;
    s.updates = t.updates = 0;
    s.rr_true = t.rr_true = 1;
    s.rr_best = t.rr_best = rr;
    s.stall = t.stall = 0;
    s.active = t.active = 1;
    s.done = t.done = rr <= s.tol2 ? 1 : 0;
  }
}

template <typename T>
BVec<T> bvec(BatchWork& w) {
  BVec<T> v{};
  if constexpr (sizeof(T) == 4) {
    for (int i = 0; i < 2; ++i) v.u[i] = w.u32[i];
    for (int i = 0; i < kChunk; ++i) {
      v.z[i] = w.z32[i];
      v.p[i] = w.p32[i];
    }
  } else {
    for (int i = 0; i < 2; ++i) v.u[i] = w.u64[i];
    for (int i = 0; i < kChunk; ++i) {
      v.z[i] = w.z64[i];
      v.p[i] = w.p64[i];
    }
  }
  v.x = w.x;
  v.phi = w.phi;
  return v;
}

template <typename T>
ifl_status dalloc_b(T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(IFL_ENOMEM, std::string("hipMalloc failed (batched work space): ") + hipGetErrorString(e));
  }
  return IFL_OK;
}

// ----------------------------------------------------------- launchers
// Grid sizes of a tile: G for the kernels that gather (SpMV, replacement,
// start, finish), Gu for the streaming update, Gp >= both the stride of the
// partial-sum array.
struct Grids {
  int G, Gu, Gp;
};

template <int R, int H>
struct LaunchH {
  template <typename T>
  static void iter(const BMat& m, BatchWork& w, Grids g, hipStream_t s, int k) {
    if (k == 0) kb_iter<T, R, false, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
    else if (k < w.chunk - 1)
      kb_iter<T, R, true, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
    else kb_iter_last<T, R, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
  }
  template <typename T>
  static void replace(const BMat& m, BatchWork& w, Grids g, hipStream_t s) {
    kb_residual<T, R, false, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, 0ull, SlotScales{},
                                                    w.chunk);
  }
  template <typename T>
  static void start(const BMat& m, BatchWork& w, Grids g, hipStream_t s, uint64_t mask, const SlotScales& cs) {
    kb_residual<T, R, true, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, mask, cs, w.chunk);
  }
};

// the pair kernels of a two-component operator, head of H blocks
template <int R, int H>
struct LaunchP {
  template <typename T>
  static void iter(const BMat& m, BatchWork& w, Grids g, hipStream_t s, int k) {
    if (k == 0) kb_iter2<T, R, false, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
    else if (k < w.chunk - 1)
      kb_iter2<T, R, true, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
    else kb_iter2_last<T, R, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
  }
  template <typename T>
  static void replace(const BMat& m, BatchWork& w, Grids g, hipStream_t s) {
    kb_residual2<T, R, false, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, 0ull, SlotScales{},
                                                     w.chunk);
  }
  template <typename T>
  static void start(const BMat& m, BatchWork& w, Grids g, hipStream_t s, uint64_t mask, const SlotScales& cs) {
    kb_residual2<T, R, true, H><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, mask, cs, w.chunk);
  }
};

template <int R>
struct Launch {
  // the gathering kernels for the matrix's form and head class
  template <typename T, typename F>
  static void by_head(const BMat& m, int head, F f) {
    if (m.psptr) {
      f(LaunchP<R, 6>{});
    } else if (head <= 6) {
      f(LaunchH<R, 6>{});
    } else if (head <= 12) {
      f(LaunchH<R, 12>{});
    } else {
      f(LaunchH<R, 20>{});
    }
  }
  // iteration k (0..L-1) of a chunk of L: one fused iteration kernel and its
  // finalizer; the last one also applies the chunk's x update and the FP64
  // residual replacement of every running column, whose true residual is
  // the only one that may stop a column (in both precisions: a recursive
  // residual drifts from the true one when S is badly conditioned)
  template <typename T>
  static void step(const BMat& m, BatchWork& w, Grids g, hipStream_t s, const BatchParams& prm, int k, int head) {
    if constexpr (R >= 2) {
      if (w.cx) {
        step_cx<T>(m, w, g, s, prm, k);
        return;
      }
    }
    if (prm.ev_begin) (void)hipEventRecord(prm.ev_begin, s);
    by_head<T>(m, head, [&](auto L) { L.template iter<T>(m, w, g, s, k); });
    if (prm.ev_end) (void)hipEventRecord(prm.ev_end, s);
    kf_step<<<R, kFinThreads, 0, s>>>(w.slots, w.part, g.G, g.Gp, R, k);
    if (k == w.chunk - 1) {
      const int64_t xthreads = m.n * Geo<T, R>::LPR;
      if (xthreads > 0)
        kb_xupdate<T, R, kChunk><<<(unsigned)((xthreads + kXB - 1) / kXB), kXB, 0, s>>>(m, bvec<T>(w), w.slots);
      by_head<T>(m, head, [&](auto L) { L.template replace<T>(m, w, g, s); });
      kf_replace<<<R, kFinThreads, 0, s>>>(w.slots, w.part, g.G, g.Gp, R, prm.max_iter);
    }
  }
  // complex tiles (the first-order operator, head of 6 entries)
  template <typename T>
  static void step_cx(const BMat& m, BatchWork& w, Grids g, hipStream_t s, const BatchParams& prm, int k) {
    if (prm.ev_begin) (void)hipEventRecord(prm.ev_begin, s);
    if (k == 0) kbc_iter<T, R, false, 6><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
    else if (k < w.chunk - 1)
      kbc_iter<T, R, true, 6><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
    else kbc_iter_last<T, R, 6><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, k, w.chunk);
    if (prm.ev_end) (void)hipEventRecord(prm.ev_end, s);
    kfc_step<<<R / 2, kFinThreads, 0, s>>>(w.slots, w.part, g.G, g.Gp, R, k);
    if (k == w.chunk - 1) {
      kbc_xupdate<T, R, kChunk><<<g.Gu, kB, 0, s>>>(m, bvec<T>(w), w.slots, g.Gu);
      kbc_residual<T, R, false, 6><<<g.G, kB, 0, s>>>(m, bvec<T>(w), w.slots, w.part, g.G, g.Gp, 0ull,
                                                       SlotScales{}, w.chunk);
      kfc_replace<<<R / 2, kFinThreads, 0, s>>>(w.slots, w.part, g.G, g.Gp, R, prm.max_iter, w.cx_g);
    }
  }
  static void iterate(const BMat& m, BatchWork& w, Grids g, hipStream_t s, const BatchParams& prm, int k, int head) {
    if (w.mixed) step<float>(m, w, g, s, prm, k, head);
    else step<double>(m, w, g, s, prm, k, head);
  }
  static void init(const BMat& m, BatchWork& w, Grids g, hipStream_t s, uint64_t mask, const SlotScales& cs,
                   double rtol, int head) {
    if constexpr (R >= 2) {
      if (w.cx) {
        if (w.mixed)
          kbc_residual<float, R, true, 6><<<g.G, kB, 0, s>>>(m, bvec<float>(w), w.slots, w.part, g.G, g.Gp, mask, cs,
                                                             w.chunk);
        else
          kbc_residual<double, R, true, 6><<<g.G, kB, 0, s>>>(m, bvec<double>(w), w.slots, w.part, g.G, g.Gp, mask,
                                                              cs, w.chunk);
        kfc_init<<<R / 2, kFinThreads, 0, s>>>(w.slots, w.part, g.G, g.Gp, R, mask, rtol, cs, w.cx_g);
        return;
      }
    }
    if (w.mixed) by_head<float>(m, head, [&](auto L) { L.template start<float>(m, w, g, s, mask, cs); });
    else by_head<double>(m, head, [&](auto L) { L.template start<double>(m, w, g, s, mask, cs); });
    kf_init<<<R, kFinThreads, 0, s>>>(w.slots, w.part, g.G, g.Gp, R, mask, rtol, cs);
  }
  static void finish(const BMat& m, BatchWork& w, Grids g, hipStream_t s, uint64_t mask, const OutPtrs& out) {
    if (w.mixed) kb_finish<float, R><<<g.G, kB, 0, s>>>(m, bvec<float>(w), w.slots, w.part, g.G, g.Gp, mask);
    else kb_finish<double, R><<<g.G, kB, 0, s>>>(m, bvec<double>(w), w.slots, w.part, g.G, g.Gp, mask);
    bool any_out = false;
    for (int j = 0; j < R; ++j) any_out |= ((mask >> j) & 1ull) && out.p[j];
    if (any_out) {
      uint64_t omask = 0;
      for (int j = 0; j < R; ++j)
        if (((mask >> j) & 1ull) && out.p[j]) omask |= 1ull << j;
      kb_out<R><<<(unsigned)((m.field_len + 255) / 256), 256, 0, s>>>(w.x, out, omask, m.row_of, m.field_len);
    }
    kf_finish<<<R, kFinThreads, 0, s>>>(w.slots, w.part, g.G, g.Gp, R, mask);
  }
};

template <template <int> class F, typename... A>
void dispatch_R(int R, A&&... a) {
  switch (R) {
    case 1: F<1>::run(a...); break;
    case 2: F<2>::run(a...); break;
    case 4: F<4>::run(a...); break;
    case 8: F<8>::run(a...); break;
    case 16: F<16>::run(a...); break;
    case 32: F<32>::run(a...); break;
    default: F<64>::run(a...); break;
  }
}

template <int R>
struct DoIterate {
  static void run(const BMat& m, BatchWork& w, Grids g, hipStream_t s, const BatchParams& p, int k, int head) {
    Launch<R>::iterate(m, w, g, s, p, k, head);
  }
};
template <int R>
struct DoInit {
  static void run(const BMat& m, BatchWork& w, Grids g, hipStream_t s, uint64_t mask, const SlotScales& cs,
                  double rtol, int head) {
    Launch<R>::init(m, w, g, s, mask, cs, rtol, head);
  }
};
template <int R>
struct DoFinish {
  static void run(const BMat& m, BatchWork& w, Grids g, hipStream_t s, uint64_t mask, const OutPtrs& o) {
    Launch<R>::finish(m, w, g, s, mask, o);
  }
};

template <typename T>
int occupancy_of(int R) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (R) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_iter<T, 1, true, 6>, kB, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_iter<T, 2, true, 6>, kB, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_iter<T, 4, true, 6>, kB, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_iter<T, 8, true, 6>, kB, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_iter<T, 16, true, 6>, kB, 0); break;
    case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_iter<T, 32, true, 6>, kB, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_iter<T, 64, true, 6>, kB, 0); break;
  }
  return e == hipSuccess ? nb : 0;
}

}  // namespace

// ----------------------------------------------------------------- host
int batch_resident_blocks(int R, bool mixed, int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) cus = 256;
  int per = mixed ? occupancy_of<float>(R) : occupancy_of<double>(R);
  if (per <= 0) per = 1;
  return per * cus;
}

int batch_lanes_per_row(int R, bool mixed) {
  const int C = std::min(mixed ? 4 : 2, R);
  return R / C;
}

ifl_status batch_alloc(BatchWork* w, const BatchMatrix& bm, int R, bool mixed, bool cx) {
  const size_t nr = (size_t)bm.n_pad * R;
  // the x update (kb_xupdate<T, R, kChunk>) reads the chunk's z buffers
  if (bm.chunk != kChunk) return fail(IFL_EINVAL, "tile chunk length differs from the kernels' kChunk");
  const int chunk = bm.chunk;
  ifl_status st;
  std::vector<void*> vecs;  // the precision's vectors, zeroed below
  size_t es = 0;
  // z[0..chunk - 1), u[0..2), the carried direction p[chunk - 1]
  auto pick = [&](auto& z, auto& u, auto& dir) {
    std::vector<std::remove_reference_t<decltype(z[0])>*> all = {&u[0], &u[1], &dir[chunk - 1]};
    for (int i = 0; i < chunk - 1; ++i) all.push_back(&z[i]);
    return all;
  };
  if (mixed) {
    es = sizeof(float);
    for (float** p : pick(w->z32, w->u32, w->p32)) {
      if ((st = dalloc_b(p, nr))) return st;
      vecs.push_back(*p);
    }
  } else {
    es = sizeof(double);
    for (double** p : pick(w->z64, w->u64, w->p64)) {
      if ((st = dalloc_b(p, nr))) return st;
      vecs.push_back(*p);
    }
  }
  w->cx = cx;
  if ((st = dalloc_b(&w->x, nr)) || (st = dalloc_b(&w->phi, nr)) ||
      (st = dalloc_b(&w->part, (size_t)Q_COUNT * R * std::max(bm.G, bm.Gu))) || (st = dalloc_b(&w->slots, (size_t)R)) ||
      (st = dalloc_b(&w->flag, 1)))
    return st;
  IFL_HIPB(hipHostMalloc((void**)&w->slots_host, sizeof(BSlot) * R, hipHostMallocDefault));
  IFL_HIPB(hipMemset(w->slots, 0, sizeof(BSlot) * R));
  IFL_HIPB(hipMemset(w->x, 0, sizeof(double) * nr));
  IFL_HIPB(hipMemset(w->phi, 0, sizeof(double) * nr));
  for (void* p : vecs) IFL_HIPB(hipMemset(p, 0, es * nr));
  // hipMemset of device memory may return before it completes, and the
  // tile's kernels run on streams that do not wait for the null stream
  IFL_HIPB(hipDeviceSynchronize());
  w->R = R;
  w->G = bm.G;
  w->Gu = bm.Gu;
  w->mixed = mixed;
  w->iter = 0;
  w->chunk = chunk;
  return IFL_OK;
}

// Four iterations for every order. Eight were measured on first-order
// tiles: the per-iteration cost fell (one x update and one FP64 replacement
// per eight iterations) but the iteration count rose more (12% on the
// level-9 sphere, 80% on the vertex vector Laplacian), since a column stops
// only at a chunk's end and the FP32 recurrences of z and u run twice as
// long between replacements.
int chunk_for_order(int) { return kChunk; }

void batch_free(BatchWork* w) {
  if (w->chunk_exec) (void)hipGraphExecDestroy(w->chunk_exec);
  std::vector<void*> ptrs = {w->u32[0], w->u32[1], w->u64[0], w->u64[1], w->x,
                             w->phi,    w->part,   w->slots,  w->flag};
  for (int i = 0; i < kChunk; ++i) {
    ptrs.push_back(w->z32[i]);
    ptrs.push_back(w->z64[i]);
    ptrs.push_back(w->p32[i]);
    ptrs.push_back(w->p64[i]);
  }
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (w->slots_host) (void)hipHostFree(w->slots_host);
  *w = BatchWork();
}

size_t batch_bytes(int64_t n_pad, int R, bool mixed, int chunk) {
  // z (x chunk - 1), u (x2), p, and x, phi
  const size_t per = (size_t)(chunk + 2) * (mixed ? 4 : 8) + 8 + 8;
  return (size_t)n_pad * R * per;
}

static Grids grids(const BatchMatrix& bm) { return Grids{bm.G, bm.Gu, std::max(bm.G, bm.Gu)}; }

static bool same_grids(const BatchMatrix& bm, const BatchWork& w) { return bm.G == w.G && bm.Gu == w.Gu; }

static BMat bmat(const BatchMatrix& bm) {
  return BMat{bm.n,     bm.n_slices,  bm.row_of, bm.field_len, bm.sptr, bm.col,    bm.val64,
              bm.val32, bm.kdiag,     bm.mass,   bm.entity,    bm.nb,   bm.nb_slices, bm.psptr,
              bm.pcol,  bm.pval64,    bm.pval32};
}

ifl_status batch_clear_flag(BatchWork& w, hipStream_t s) {
  IFL_HIPB(hipMemsetAsync(w.flag, 0, sizeof(int), s));
  return IFL_OK;
}

ifl_status batch_load_column(const BatchMatrix& bm, BatchWork& w, int slot, const double* field_dev, hipStream_t s) {
  kb_gather<<<(unsigned)((bm.n + 255) / 256), 256, 0, s>>>(field_dev, bm.entity, bm.n, w.R, slot, w.phi, w.flag);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

ifl_status batch_load_synthetic(const BatchMatrix& bm, BatchWork& w, int slot, uint64_t seed, hipStream_t s) {
  if (slot < 0 || slot >= w.R) return fail(IFL_EINVAL, "slot out of range");
  kb_synth<<<(unsigned)((bm.n + 255) / 256), 256, 0, s>>>(bm.n, w.R, slot, seed, w.phi);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

ifl_status batch_load_columns(const BatchMatrix& bm, BatchWork& w, uint64_t mask, const double* const* fields_dev,
                              bool internal, hipStream_t s) {
  FieldPtrs f{};
  for (int j = 0; j < w.R; ++j) {
    if (!((mask >> j) & 1ull)) continue;
    if (!fields_dev[j]) return fail(IFL_EINVAL, "field pointer of a loaded slot is NULL");
    f.p[j] = fields_dev[j];
  }
  if (w.R < 64 && (mask >> w.R)) return fail(IFL_EINVAL, "slot mask beyond the tile");
  kb_gather_cols<<<(unsigned)((bm.n + 255) / 256), 256, 0, s>>>(f, mask, bm.entity, bm.n, w.R, internal ? 1 : 0,
                                                                w.phi, w.flag);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

ifl_status batch_permute_fields(const BatchMatrix& bm, const double* src, int64_t L, int n_fields, double* dst,
                                int* flag, hipStream_t s) {
  if (n_fields <= 0) return IFL_OK;
  if (n_fields > 65535) return fail(IFL_EINVAL, "too many fields in one call (max 65535)");
  const dim3 grid((unsigned)((bm.n + 255) / 256), (unsigned)n_fields);
  kb_permute<<<grid, 256, 0, s>>>(src, L, bm.entity, bm.n, bm.n_pad, dst, flag);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

ifl_status batch_check_flag(BatchWork& w, hipStream_t s, bool* bad) {
  int flag = 0;
  IFL_HIPB(hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  IFL_HIPB(hipStreamSynchronize(s));
  *bad = flag != 0;
  return IFL_OK;
}

ifl_status batch_init(const BatchMatrix& bm, BatchWork& w, uint64_t mask, const SlotScales& cs, double rtol,
                      hipStream_t s) {
  if (!same_grids(bm, w)) return fail(IFL_EINVAL, "tile work space was sized for other grid sizes");
  if (w.iter % w.chunk != 0)
    return fail(IFL_EINVAL, "columns may only enter a tile at chunk boundaries");
  dispatch_R<DoInit>(w.R, bmat(bm), w, grids(bm), s, mask, cs, rtol, bm.head);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

double batch_spmv_bytes(const BatchMatrix& bm, int64_t nnz_stored, bool mixed, int live) {
  const double vb = mixed ? 4.0 : 8.0;
  // pair kernels: block entries (index + four values) over slices of block rows
  if (bm.pairs)
    return (double)bm.pnnz * (4.0 + 4.0 * vb) + 8.0 * (bm.nb_slices + 1) + 16.0 * bm.n + 4.0 * vb * bm.n * live;
  // z and u read, z and u written per column
  return (double)nnz_stored * (4.0 + vb) + 8.0 * (bm.n_slices + 1) + 16.0 * bm.n + 4.0 * vb * bm.n * live;
}

// Capture one chunk (w.chunk iterations, no timing events) into w.chunk_exec.
// The kernel arguments of a tile do not change from one chunk to the next, so
// the one graph serves every chunk until max_iter changes.
static ifl_status capture_chunk(const BMat& m, const BatchMatrix& bm, BatchWork& w, const BatchParams& prm,
                                hipStream_t s) {
  if (w.chunk_exec) {
    (void)hipGraphExecDestroy(w.chunk_exec);
    w.chunk_exec = nullptr;
  }
  BatchParams p = prm;
  p.ev_begin = p.ev_end = nullptr;
  IFL_HIPB(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < w.chunk; ++k) dispatch_R<DoIterate>(w.R, m, w, grids(bm), s, p, k, bm.head);
  hipGraph_t g = nullptr;
  const hipError_t e1 = hipStreamEndCapture(s, &g);
  const hipError_t e2 = hipGetLastError();
  if (e1 != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return fail(IFL_EDEVICE, std::string("capturing a chunk failed: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  const hipError_t e3 = hipGraphInstantiate(&w.chunk_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) {
    w.chunk_exec = nullptr;
    return fail(IFL_EDEVICE, std::string("instantiating a chunk graph failed: ") + hipGetErrorString(e3));
  }
  w.chunk_max_iter = prm.max_iter;
  return IFL_OK;
}

ifl_status batch_iterate(const BatchMatrix& bm, BatchWork& w, int n_iter, const BatchParams& prm, hipStream_t s) {
  if (!same_grids(bm, w)) return fail(IFL_EINVAL, "tile work space was sized for other grid sizes");
  if (n_iter % w.chunk != 0) return fail(IFL_EINVAL, "batched iterations come in multiples of the tile's chunk");
  const BMat m = bmat(bm);
  // the timing events (if any) go around the SpMV of the call's second
  // iteration (the recurrence form that stores z and u, twice per chunk); the
  // chunk holding it is launched directly
  BatchParams rest = prm;
  rest.ev_begin = rest.ev_end = nullptr;
  const bool events = prm.ev_begin || prm.ev_end;
  for (int i = 0; i < n_iter;) {
    const bool timed = events && i <= 1;
    if (!timed && prm.graphs && !w.graphs_broken && w.iter % w.chunk == 0 && n_iter - i >= w.chunk) {
      if (!w.chunk_exec || w.chunk_max_iter != prm.max_iter) {
        if (capture_chunk(m, bm, w, prm, s) != IFL_OK) {
          // launch directly from now on; the stream is out of capture mode
          w.graphs_broken = true;
          (void)hipGetLastError();
          continue;
        }
      }
      IFL_HIPB(hipGraphLaunch(w.chunk_exec, s));
      w.iter += w.chunk;
      i += w.chunk;
      continue;
    }
    const int k = (int)(w.iter % w.chunk);
    dispatch_R<DoIterate>(w.R, m, w, grids(bm), s, i == 1 ? prm : rest, k, bm.head);
    ++w.iter;
    ++i;
  }
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

ifl_status batch_finish(const BatchMatrix& bm, BatchWork& w, uint64_t mask, double* const* out, hipStream_t s) {
  if (!same_grids(bm, w)) return fail(IFL_EINVAL, "tile work space was sized for other grid sizes");
  OutPtrs o;
  for (int j = 0; j < 64; ++j) o.p[j] = (j < w.R && out) ? out[j] : nullptr;
  dispatch_R<DoFinish>(w.R, bmat(bm), w, grids(bm), s, mask, o);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

ifl_status batch_read_slots(BatchWork& w, hipStream_t s) {
  IFL_HIPB(hipMemcpyAsync(w.slots_host, w.slots, sizeof(BSlot) * w.R, hipMemcpyDeviceToHost, s));
  IFL_HIPB(hipStreamSynchronize(s));
  return IFL_OK;
}

ifl_status batch_move_columns(const BatchMatrix& bm, BatchWork& src, BatchWork& dst, const int* from, const int* to,
                              int n, hipStream_t s) {
  if (src.mixed != dst.mixed) return fail(IFL_EINVAL, "tiles of different precision");
  if (src.iter % src.chunk != 0 || src.chunk != dst.chunk)
    return fail(IFL_EINVAL, "columns move only at chunk boundaries, between tiles of one chunk length");
  if (n < 0 || n > dst.R || n > src.R) return fail(IFL_EINVAL, "too many columns to move");
  ColMap map{};
  map.n = n;
  for (int c = 0; c < n; ++c) {
    if (from[c] < 0 || from[c] >= src.R || to[c] < 0 || to[c] >= dst.R)
      return fail(IFL_EINVAL, "column slot out of range");
    map.src[c] = from[c];
    map.dst[c] = to[c];
  }
  const unsigned nb = (unsigned)((bm.n_pad + 255) / 256);
  if (src.mixed)
    kb_move_cols<float><<<nb, 256, 0, s>>>(src.z32[0], src.p32[src.chunk - 1], src.x, src.phi, src.R, dst.z32[0],
                                            dst.p32[dst.chunk - 1], dst.x, dst.phi, dst.R, map, bm.n_pad);
  else
    kb_move_cols<double><<<nb, 256, 0, s>>>(src.z64[0], src.p64[src.chunk - 1], src.x, src.phi, src.R, dst.z64[0],
                                             dst.p64[dst.chunk - 1], dst.x, dst.phi, dst.R, map, bm.n_pad);
  kf_move_slots<<<1, 64, 0, s>>>(src.slots, dst.slots, dst.R, map);
  IFL_HIPB(hipGetLastError());
  dst.iter = 0;
  return IFL_OK;
}

ifl_status batch_release(BatchWork& w, uint64_t mask, hipStream_t s) {
  kf_release<<<1, 64, 0, s>>>(w.slots, w.R, mask);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

}  // namespace ifl
