// Multi-RHS batched solver: many (field, scale) columns share one pass over
// the matrix stream of K_n.
//
// Every column is an independent Jacobi-PCG solve of S_j x = M phi_j with
// S_j = M + c_j K_n (Sect. 2.2.2, residual form x0 = phi_j). A tile holds R
// slots; vectors are stored rows x R with the R columns of a row contiguous,
// and a wavefront covers 64/R consecutive rows x R columns, lane = column.
// Each sliced-ELL entry (index, value) is then loaded once per row for all R
// columns (identical addresses within a row's lanes are served by one
// request), and the gather of a neighbour's R values is one contiguous
// segment. HBM traffic per column-iteration is the vector traffic plus
// 1/R of the matrix stream.
//
// Per-column state (alpha, beta, rho, stopping, residual replacement) lives
// in device memory; after each reduction phase a small kernel with one
// workgroup per column finishes that column's sum in a fixed order. A
// column's arithmetic and reduction order do not depend on the other
// columns, on its slot index or on when it entered the tile, so a solve
// gives bitwise the same result alone or in a full tile. Finished columns
// leave the tile and new ones take their slots between iterations
// (continuous batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
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

enum { Q_PQ = 0, Q_RZ, Q_RR, Q_BB, Q_FL, Q_RES, Q_EN, Q_COUNT };

struct BMat {
  int64_t n, n_slices;
  const int64_t* sptr;
  const int32_t* col;
  const double* val64;
  const float* val32;
  const double* kdiag;
  const double* mass;
  const int64_t* entity;
};

template <typename T>
struct BVec {
  T* r;
  T* z;
  T* p0;
  T* p1;
  T* q;
  float* xacc;   // mixed: FP32 increments since the last fold
  double* x;     // FP64 solution
  double* phi;   // FP64 field per column
};

struct OutPtrs {
  double* p[64];
};

template <typename T>
__device__ __forceinline__ const T* bval(const BMat& m);
template <>
__device__ __forceinline__ const double* bval<double>(const BMat& m) { return m.val64; }
template <>
__device__ __forceinline__ const float* bval<float>(const BMat& m) { return m.val32; }

__device__ __forceinline__ int lblock(int G) {
  const int b = blockIdx.x;
  if (G % 8) return b;
  return (b % 8) * (G / 8) + b / 8;
}

// Per-column block sums: lane l carries column l % R. Result for column t
// in thread t (t < R), fixed order.
template <int R, int NV>
__device__ __forceinline__ void col_sum(double (&v)[NV], double* lds /* NV*kWpb*R */) {
  const int lane = threadIdx.x % kW, wid = threadIdx.x / kW;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = v[i];
#pragma unroll
    for (int off = 32; off >= R; off >>= 1) s += __shfl_xor(s, off, kW);
    if (lane < R) lds[(i * kWpb + wid) * R + lane] = s;
  }
  __syncthreads();
  if (threadIdx.x < R) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < kWpb; ++w) s += lds[(i * kWpb + w) * R + threadIdx.x];
      v[i] = s;
    }
  }
}

struct Range {
  int64_t begin, end;
};

// contiguous task range of this logical block; a task is 64/R rows
__device__ __forceinline__ Range task_range(int64_t ntasks, int G) {
  const int lb = lblock(G);
  const int64_t per = (ntasks + G - 1) / G;
  const int64_t b = (int64_t)lb * per;
  return {b, min(b + per, ntasks)};
}

__device__ __forceinline__ bool live(const BSlot& s) { return s.active && s.done == 0; }

// ------------------------------------------------------------ iteration
template <typename T, int R>
__global__ __launch_bounds__(kB) void kb_dir_spmv(BMat m, BVec<T> v, BSlot* slots, double* part, int G) {
  __shared__ double lds[1 * kWpb * R];
  constexpr int RPW = kW / R;
  const int lane = threadIdx.x % kW, wid = threadIdx.x / kW;
  const int j = lane % R, rsub = lane / R;
  const BSlot& sl = slots[j];
  const bool on = live(sl);
  const T beta = (T)sl.beta;
  const T c = (T)sl.c;
  const double c64 = sl.c;
  const int par = sl.iters & 1;
  const T* __restrict__ pin = par ? v.p1 : v.p0;
  T* __restrict__ pout = par ? v.p0 : v.p1;
  const T* __restrict__ z = v.z;
  const T* __restrict__ val = bval<T>(m);
  const int64_t ntasks = m.n_slices * R;  // tasks of 64/R rows
  const Range rg = task_range(ntasks, G);
  double acc[1] = {0.0};
  if (on) {
    for (int64_t t = rg.begin + wid; t < rg.end; t += kWpb) {
      const int64_t row = t * RPW + rsub;
      if (row >= m.n) continue;
      const int64_t s = row / kW, l = row % kW;
      const int64_t base = m.sptr[s];
      const int w = (int)((m.sptr[s + 1] - base) / kW);
      // Entries are taken kUnroll at a time: all index / value loads, then
      // all gathers, then the FMAs in entry order (the summation order is
      // that of the plain loop; the unrolling only raises the number of
      // loads in flight per wavefront).
      T a = (T)0;
      for (int k0 = 0; k0 < w; k0 += kUnroll) {
        int32_t cu[kUnroll];
        T vu[kUnroll], zu[kUnroll], pu[kUnroll];
        // loads past the row's end stay in bounds (next slice or the zero
        // tail of the arrays); their values are replaced by 0
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int64_t e = base + (int64_t)(k0 + u) * kW + l;
          cu[u] = m.col[e];
          const T vv = val[e];
          vu[u] = k0 + u < w ? vv : (T)0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int64_t cj = (int64_t)cu[u] * R + j;
          zu[u] = z[cj];
          pu[u] = pin[cj];
        }
        // entries past the row's end have value 0 and gather row 0 (finite):
        // their FMA leaves a unchanged, so no branch keeps the gathers apart
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) a = fma(vu[u], fma(beta, pu[u], zu[u]), a);
      }
      const int64_t idx = row * R + j;
      const T pn = fma(beta, pin[idx], z[idx]);
      const T d = (T)(m.mass[row] + c64 * m.kdiag[row]);
      const T qv = fma(d, pn, c * a);
      pout[idx] = pn;
      v.q[idx] = qv;
      acc[0] += (double)pn * (double)qv;
    }
  }
  col_sum<R, 1>(acc, lds);
  if (threadIdx.x < R) part[(Q_PQ * R + threadIdx.x) * G + lblock(G)] = acc[0];
}

template <typename T, bool MIXED, int R>
__global__ __launch_bounds__(kB) void kb_update(BMat m, BVec<T> v, BSlot* slots, double* part, int G) {
  __shared__ double lds[2 * kWpb * R];
  constexpr int RPW = kW / R;
  const int lane = threadIdx.x % kW, wid = threadIdx.x / kW;
  const int j = lane % R, rsub = lane / R;
  const BSlot& sl = slots[j];
  const bool on = live(sl);
  const double a64 = sl.alpha;
  const T alpha = (T)a64;
  const double c64 = sl.c;
  const int par = sl.iters & 1;
  const T* __restrict__ p = par ? v.p0 : v.p1;  // written by kb_dir_spmv this iteration
  const int64_t ntasks = m.n_slices * R;  // tasks of 64/R rows
  const Range rg = task_range(ntasks, G);
  double acc[2] = {0.0, 0.0};
  if (on) {
    for (int64_t t = rg.begin + wid; t < rg.end; t += kWpb) {
      const int64_t row = t * RPW + rsub;
      if (row >= m.n) continue;
      const int64_t idx = row * R + j;
      const T pv = p[idx];
      if (MIXED) v.xacc[idx] = fma(alpha, pv, v.xacc[idx]);
      else v.x[idx] = fma(a64, (double)pv, v.x[idx]);
      const T rv = fma(-alpha, v.q[idx], v.r[idx]);
      const T d = (T)(m.mass[row] + c64 * m.kdiag[row]);
      const T zv = rv / d;
      v.r[idx] = rv;
      v.z[idx] = zv;
      acc[0] += (double)rv * (double)zv;
      acc[1] += (double)rv * (double)rv;
    }
  }
  col_sum<R, 2>(acc, lds);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_RZ * R + threadIdx.x) * G + lb] = acc[0];
    part[(Q_RR * R + threadIdx.x) * G + lb] = acc[1];
  }
}

// mixed: fold the FP32 increments into the FP64 solution for flagged columns
template <int R>
__global__ __launch_bounds__(kB) void kb_fold(BMat m, BVec<float> v, const BSlot* slots, int G) {
  constexpr int RPW = kW / R;
  const int lane = threadIdx.x % kW, wid = threadIdx.x / kW;
  const int j = lane % R, rsub = lane / R;
  if (!slots[j].fold) return;
  const int64_t ntasks = m.n_slices * R;  // tasks of 64/R rows
  const Range rg = task_range(ntasks, G);
  for (int64_t t = rg.begin + wid; t < rg.end; t += kWpb) {
    const int64_t row = t * RPW + rsub;
    if (row >= m.n) continue;
    const int64_t idx = row * R + j;
    v.x[idx] += (double)v.xacc[idx];
    v.xacc[idx] = 0.0f;
  }
}

// FP64 residual r = M phi - S x (FP64 values and x) for flagged columns
// (mode 0: residual replacement of a mixed solve) or for the columns being
// initialised (mode 1: x = phi first, r0 = -c K_n phi).
template <typename T, int R, int MODE>
__global__ __launch_bounds__(kB) void kb_residual(BMat m, BVec<T> v, const BSlot* slots, double* part, int G,
                                                  uint64_t mask, SlotScales cs) {
  __shared__ double lds[4 * kWpb * R];
  constexpr int RPW = kW / R;
  const int lane = threadIdx.x % kW, wid = threadIdx.x / kW;
  const int j = lane % R, rsub = lane / R;
  const BSlot& sl = slots[j];
  const bool on = MODE == 0 ? (sl.fold != 0) : ((mask >> j) & 1ull) != 0;
  const double c = MODE == 0 ? sl.c : cs.c[j];
  const int64_t ntasks = m.n_slices * R;  // tasks of 64/R rows
  const Range rg = task_range(ntasks, G);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // rz, rr, floor (mode 0) or bb (mode 1)
  if (on) {
    const double* __restrict__ src = MODE == 0 ? v.x : v.phi;
    for (int64_t t = rg.begin + wid; t < rg.end; t += kWpb) {
      const int64_t row = t * RPW + rsub;
      if (row >= m.n) continue;
      const int64_t s = row / kW, l = row % kW;
      const int64_t base = m.sptr[s];
      const int w = (int)((m.sptr[s + 1] - base) / kW);
      double a = 0.0, aa = 0.0;
      for (int k = 0; k < w; ++k) {
        const int64_t e = base + (int64_t)k * kW + l;
        const double tv = m.val64[e] * src[(int64_t)m.col[e] * R + j];
        a += tv;
        aa += fabs(tv);
      }
      const int64_t idx = row * R + j;
      const double mi = m.mass[row], kd = m.kdiag[row];
      const double ph = v.phi[idx];
      const double xi = MODE == 0 ? v.x[idx] : ph;
      double r64;
      if (MODE == 0) {
        r64 = mi * (ph - xi) - c * (kd * xi + a);
        const double mag = fabs(mi * ph) + fabs(mi * xi) + c * (fabs(kd * xi) + aa);
        acc[2] += mag * mag;
      } else {
        r64 = -c * (kd * ph + a);
        v.x[idx] = ph;
        if (v.xacc) v.xacc[idx] = 0.0f;
        v.p0[idx] = (T)0;
        v.p1[idx] = (T)0;
        acc[3] += (mi * ph) * (mi * ph);
      }
      const T rt = (T)r64;
      const T d = (T)(mi + c * kd);
      const T zt = rt / d;
      v.r[idx] = rt;
      v.z[idx] = zt;
      acc[0] += (double)rt * (double)zt;
      acc[1] += r64 * r64;
    }
  }
  col_sum<R, 4>(acc, lds);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_RZ * R + threadIdx.x) * G + lb] = acc[0];
    part[(Q_RR * R + threadIdx.x) * G + lb] = acc[1];
    part[(Q_FL * R + threadIdx.x) * G + lb] = acc[2];
    part[(Q_BB * R + threadIdx.x) * G + lb] = acc[3];
  }
}

// End of a column: x (+ increments) to the caller's numbering, partials of
// the true residual and of sum M x^2.
template <int R>
__global__ __launch_bounds__(kB) void kb_finish(BMat m, BVec<float> vf, BVec<double> vd, bool mixed,
                                                const BSlot* slots, double* part, int G, uint64_t mask,
                                                OutPtrs out) {
  __shared__ double lds[2 * kWpb * R];
  constexpr int RPW = kW / R;
  const int lane = threadIdx.x % kW, wid = threadIdx.x / kW;
  const int j = lane % R, rsub = lane / R;
  const bool on = ((mask >> j) & 1ull) != 0;
  const double c = slots[j].c;
  const double* __restrict__ x = mixed ? vf.x : vd.x;
  const float* __restrict__ xacc = mixed ? vf.xacc : nullptr;
  const double* __restrict__ phi = mixed ? vf.phi : vd.phi;
  double* __restrict__ o = out.p[j];
  const int64_t ntasks = m.n_slices * R;  // tasks of 64/R rows
  const Range rg = task_range(ntasks, G);
  double acc[2] = {0.0, 0.0};
  if (on) {
    for (int64_t t = rg.begin + wid; t < rg.end; t += kWpb) {
      const int64_t row = t * RPW + rsub;
      if (row >= m.n) continue;
      const int64_t s = row / kW, l = row % kW;
      const int64_t base = m.sptr[s];
      const int w = (int)((m.sptr[s + 1] - base) / kW);
      double a = 0.0;
      for (int k = 0; k < w; ++k) {
        const int64_t e = base + (int64_t)k * kW + l;
        const int64_t cj = (int64_t)m.col[e] * R + j;
        const double xj = xacc ? x[cj] + (double)xacc[cj] : x[cj];
        a += m.val64[e] * xj;
      }
      const int64_t idx = row * R + j;
      const double xi = xacc ? x[idx] + (double)xacc[idx] : x[idx];
      const double mi = m.mass[row];
      const double r64 = mi * (phi[idx] - xi) - c * (m.kdiag[row] * xi + a);
      if (o) o[m.entity[row]] = xi;
      acc[0] += r64 * r64;
      acc[1] += mi * xi * xi;
    }
  }
  col_sum<R, 2>(acc, lds);
  if (threadIdx.x < R) {
    const int lb = lblock(G);
    part[(Q_RES * R + threadIdx.x) * G + lb] = acc[0];
    part[(Q_EN * R + threadIdx.x) * G + lb] = acc[1];
  }
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

// phase 1 (after kb_dir_spmv): alpha = rho / (p, q)
__global__ __launch_bounds__(kFinThreads) void kf_alpha(BSlot* slots, const double* part, int G, int R) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  BSlot& s = slots[j];
  if (!live(s)) return;
  const double pq = fin_sum(part + (Q_PQ * R + j) * G, G, lds);
  if (threadIdx.x == 0) {
    const double a = s.rho / pq;
    if (!(pq > 0.0) || !isfinite(a)) s.done = 2;
    else s.alpha = a;
  }
}

// phase 2 (after kb_update): rho, beta, stopping test / fold decision
__global__ __launch_bounds__(kFinThreads) void kf_beta(BSlot* slots, const double* part, int G, int R, int mixed,
                                                        int max_iter, int fold_every, double delta2) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  BSlot& s = slots[j];
  if (!live(s)) return;
  const double rz = fin_sum(part + (Q_RZ * R + j) * G, G, lds);
  const double rr = fin_sum(part + (Q_RR * R + j) * G, G, lds);
  if (threadIdx.x == 0) {
    s.rho_prev = s.rho;
    s.rho = rz;
    s.beta = rz / s.rho_prev;
    s.rr = rr;
    s.iters += 1;
    if (!mixed) {
      if (rr <= s.tol2) s.done = 1;
    } else {
      s.rr_true = 0;
      s.fold = (rr <= s.tol2 || (s.iters % fold_every == 0 && rr <= delta2 * s.rr_ref)) ? 1 : 0;
    }
    if (s.done == 0 && s.iters >= max_iter) {
      if (mixed) s.fold = 1;  // finish with an FP64 residual; done = 3 set after it
      else s.done = 3;
    }
  }
}

// phase 3 (mixed, after kb_residual mode 0): replaced residual
__global__ __launch_bounds__(kFinThreads) void kf_replace(BSlot* slots, const double* part, int G, int R,
                                                           int max_iter) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  BSlot& s = slots[j];
  if (!s.active || !s.fold) return;
  const double rz = fin_sum(part + (Q_RZ * R + j) * G, G, lds);
  const double rr = fin_sum(part + (Q_RR * R + j) * G, G, lds);
  const double fl = fin_sum(part + (Q_FL * R + j) * G, G, lds);
  if (threadIdx.x == 0) {
    s.rho = rz;
    s.beta = rz / s.rho_prev;
    s.rr = rr;
    s.rr_ref = rr;
    s.rr_true = 1;
    s.updates += 1;
    s.fold = 0;
    const double floor2 = fl * (kFloor * kU) * (kFloor * kU);
    if (rr <= fmax(s.tol2, floor2)) s.done = 1;
    else if (s.iters >= max_iter) s.done = 3;
  }
}

// start of a column (after kb_residual mode 1)
__global__ __launch_bounds__(kFinThreads) void kf_init(BSlot* slots, const double* part, int G, int R, uint64_t mask,
                                                        double rtol, SlotScales cs) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  if (!((mask >> j) & 1ull)) return;
  BSlot& s = slots[j];
  const double rz = fin_sum(part + (Q_RZ * R + j) * G, G, lds);
  const double rr = fin_sum(part + (Q_RR * R + j) * G, G, lds);
  const double bb = fin_sum(part + (Q_BB * R + j) * G, G, lds);
  if (threadIdx.x == 0) {
    s.c = cs.c[j];
    s.rho = rz;
    s.rho_prev = INFINITY;
    s.beta = 0.0;
    s.alpha = 0.0;
    s.rr = rr;
    s.bb = bb;
    s.tol2 = rtol * rtol * bb;
    s.rr_ref = rr;
    s.iters = 0;
    s.updates = 0;
    s.rr_true = 1;
    s.fold = 0;
    s.active = 1;
    s.done = rr <= s.tol2 ? 1 : 0;
  }
}

__global__ void kf_release(BSlot* slots, int R, uint64_t mask) {
  const int j = threadIdx.x;
  if (j < R && ((mask >> j) & 1ull)) {
    slots[j].active = 0;
    slots[j].done = 0;
    slots[j].fold = 0;
  }
}

__global__ __launch_bounds__(kFinThreads) void kf_finish(BSlot* slots, const double* part, int G, int R,
                                                          uint64_t mask) {
  __shared__ double lds[kFinThreads / kW];
  const int j = blockIdx.x;
  if (!((mask >> j) & 1ull)) return;
  BSlot& s = slots[j];
  const double res = fin_sum(part + (Q_RES * R + j) * G, G, lds);
  const double en = fin_sum(part + (Q_EN * R + j) * G, G, lds);
  if (threadIdx.x == 0) {
    s.res2 = res;
    s.energy2 = en;
  }
}

template <typename T>
BVec<T> bvec(BatchWork& w) {
  if constexpr (sizeof(T) == 4) {
    return BVec<T>{w.r32, w.z32, w.p32[0], w.p32[1], w.q32, w.xacc, w.x, w.phi};
  } else {
    return BVec<T>{w.r64, w.z64, w.p64[0], w.p64[1], w.q64, nullptr, w.x, w.phi};
  }
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
template <int R>
struct Launch {
  static void iterate(const BMat& m, BatchWork& w, bool mixed, int G, hipStream_t s, const BatchParams& prm) {
    if (prm.ev_begin) (void)hipEventRecord(prm.ev_begin, s);
    if (mixed) kb_dir_spmv<float, R><<<G, kB, 0, s>>>(m, bvec<float>(w), w.slots, w.part, G);
    else kb_dir_spmv<double, R><<<G, kB, 0, s>>>(m, bvec<double>(w), w.slots, w.part, G);
    if (prm.ev_end) (void)hipEventRecord(prm.ev_end, s);
    if (mixed) {
      BVec<float> v = bvec<float>(w);
      kf_alpha<<<R, kFinThreads, 0, s>>>(w.slots, w.part, G, R);
      kb_update<float, true, R><<<G, kB, 0, s>>>(m, v, w.slots, w.part, G);
      kf_beta<<<R, kFinThreads, 0, s>>>(w.slots, w.part, G, R, 1, prm.max_iter, prm.fold_every, prm.delta2);
      kb_fold<R><<<G, kB, 0, s>>>(m, v, w.slots, G);
      kb_residual<float, R, 0><<<G, kB, 0, s>>>(m, v, w.slots, w.part, G, 0ull, SlotScales{});
      kf_replace<<<R, kFinThreads, 0, s>>>(w.slots, w.part, G, R, prm.max_iter);
    } else {
      BVec<double> v = bvec<double>(w);
      kf_alpha<<<R, kFinThreads, 0, s>>>(w.slots, w.part, G, R);
      kb_update<double, false, R><<<G, kB, 0, s>>>(m, v, w.slots, w.part, G);
      kf_beta<<<R, kFinThreads, 0, s>>>(w.slots, w.part, G, R, 0, prm.max_iter, prm.fold_every, prm.delta2);
    }
  }
  static void init(const BMat& m, BatchWork& w, bool mixed, int G, hipStream_t s, uint64_t mask,
                   const SlotScales& cs, double rtol) {
    if (mixed) kb_residual<float, R, 1><<<G, kB, 0, s>>>(m, bvec<float>(w), w.slots, w.part, G, mask, cs);
    else kb_residual<double, R, 1><<<G, kB, 0, s>>>(m, bvec<double>(w), w.slots, w.part, G, mask, cs);
    kf_init<<<R, kFinThreads, 0, s>>>(w.slots, w.part, G, R, mask, rtol, cs);
  }
  static void finish(const BMat& m, BatchWork& w, bool mixed, int G, hipStream_t s, uint64_t mask,
                     const OutPtrs& out) {
    kb_finish<R><<<G, kB, 0, s>>>(m, bvec<float>(w), bvec<double>(w), mixed, w.slots, w.part, G, mask, out);
    kf_finish<<<R, kFinThreads, 0, s>>>(w.slots, w.part, G, R, mask);
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
  static void run(const BMat& m, BatchWork& w, bool mixed, int G, hipStream_t s, const BatchParams& p) {
    Launch<R>::iterate(m, w, mixed, G, s, p);
  }
};
template <int R>
struct DoInit {
  static void run(const BMat& m, BatchWork& w, bool mixed, int G, hipStream_t s, uint64_t mask,
                  const SlotScales& cs, double rtol) {
    Launch<R>::init(m, w, mixed, G, s, mask, cs, rtol);
  }
};
template <int R>
struct DoFinish {
  static void run(const BMat& m, BatchWork& w, bool mixed, int G, hipStream_t s, uint64_t mask, const OutPtrs& o) {
    Launch<R>::finish(m, w, mixed, G, s, mask, o);
  }
};

}  // namespace

// ----------------------------------------------------------------- host
ifl_status batch_alloc(BatchWork* w, const BatchMatrix& bm, int R, bool mixed) {
  const size_t nr = (size_t)bm.n_pad * R;
  ifl_status st;
  if (mixed) {
    if ((st = dalloc_b(&w->r32, nr)) || (st = dalloc_b(&w->z32, nr)) || (st = dalloc_b(&w->p32[0], nr)) ||
        (st = dalloc_b(&w->p32[1], nr)) || (st = dalloc_b(&w->q32, nr)) || (st = dalloc_b(&w->xacc, nr)))
      return st;
  } else {
    if ((st = dalloc_b(&w->r64, nr)) || (st = dalloc_b(&w->z64, nr)) || (st = dalloc_b(&w->p64[0], nr)) ||
        (st = dalloc_b(&w->p64[1], nr)) || (st = dalloc_b(&w->q64, nr)))
      return st;
  }
  if ((st = dalloc_b(&w->x, nr)) || (st = dalloc_b(&w->phi, nr)) ||
      (st = dalloc_b(&w->part, (size_t)Q_COUNT * R * bm.G)) || (st = dalloc_b(&w->slots, (size_t)R)) ||
      (st = dalloc_b(&w->flag, 1)))
    return st;
  IFL_HIPB(hipHostMalloc((void**)&w->slots_host, sizeof(BSlot) * R, hipHostMallocDefault));
  IFL_HIPB(hipMemset(w->slots, 0, sizeof(BSlot) * R));
  IFL_HIPB(hipMemset(w->x, 0, sizeof(double) * nr));
  IFL_HIPB(hipMemset(w->phi, 0, sizeof(double) * nr));
  w->R = R;
  w->mixed = mixed;
  return IFL_OK;
}

void batch_free(BatchWork* w) {
  void* ptrs[] = {w->r32, w->z32, w->p32[0], w->p32[1], w->q32, w->xacc, w->r64, w->z64, w->p64[0], w->p64[1],
                  w->q64, w->x, w->phi, w->part, w->slots, w->flag};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (w->slots_host) (void)hipHostFree(w->slots_host);
  *w = BatchWork();
}

size_t batch_bytes(int64_t n_pad, int R, bool mixed) {
  const size_t per = mixed ? (5 * 4 + 4 + 8 + 8) : (5 * 8 + 8 + 8);
  return (size_t)n_pad * R * per;
}

static BMat bmat(const BatchMatrix& bm) {
  return BMat{bm.n, bm.n_slices, bm.sptr, bm.col, bm.val64, bm.val32, bm.kdiag, bm.mass, bm.entity};
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

ifl_status batch_check_flag(BatchWork& w, hipStream_t s, bool* bad) {
  int flag = 0;
  IFL_HIPB(hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  IFL_HIPB(hipStreamSynchronize(s));
  *bad = flag != 0;
  return IFL_OK;
}

ifl_status batch_init(const BatchMatrix& bm, BatchWork& w, uint64_t mask, const SlotScales& cs, double rtol,
                      hipStream_t s) {
  dispatch_R<DoInit>(w.R, bmat(bm), w, w.mixed, bm.G, s, mask, cs, rtol);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

double batch_spmv_bytes(const BatchMatrix& bm, int64_t nnz_stored, bool mixed, int live) {
  const double vb = mixed ? 4.0 : 8.0;
  return (double)nnz_stored * (4.0 + vb) + 8.0 * (bm.n_slices + 1) + 16.0 * bm.n + 4.0 * vb * bm.n * live;
}

ifl_status batch_iterate(const BatchMatrix& bm, BatchWork& w, int n_iter, const BatchParams& prm, hipStream_t s) {
  const BMat m = bmat(bm);
  BatchParams rest = prm;
  rest.ev_begin = rest.ev_end = nullptr;
  for (int i = 0; i < n_iter; ++i) dispatch_R<DoIterate>(w.R, m, w, w.mixed, bm.G, s, i == 0 ? prm : rest);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

ifl_status batch_finish(const BatchMatrix& bm, BatchWork& w, uint64_t mask, double* const* out, hipStream_t s) {
  OutPtrs o;
  for (int j = 0; j < 64; ++j) o.p[j] = (j < w.R && out) ? out[j] : nullptr;
  dispatch_R<DoFinish>(w.R, bmat(bm), w, w.mixed, bm.G, s, mask, o);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

ifl_status batch_read_slots(BatchWork& w, hipStream_t s) {
  IFL_HIPB(hipMemcpyAsync(w.slots_host, w.slots, sizeof(BSlot) * w.R, hipMemcpyDeviceToHost, s));
  IFL_HIPB(hipStreamSynchronize(s));
  return IFL_OK;
}

ifl_status batch_release(BatchWork& w, uint64_t mask, hipStream_t s) {
  kf_release<<<1, 64, 0, s>>>(w.slots, w.R, mask);
  IFL_HIPB(hipGetLastError());
  return IFL_OK;
}

}  // namespace ifl
