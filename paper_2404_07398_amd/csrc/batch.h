// Multi-RHS batched solver: shared declarations (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace ifl {

// A batched tile advances in chunks of kChunk CG iterations: x is updated
// and the FP64 residual replaced at the end of each chunk (where alone a
// column may stop), columns enter only at chunk boundaries, and the host
// advances a tile by whole chunks.
constexpr int kChunk = 4;  // iterations per chunk (buffers and alpha history)
int chunk_for_order(int order);

// Per-column CG state of one slot (device memory; mirrored to pinned host
// memory by batch_read_slots).
struct BSlot {
  double c;         // gamma / k^(2n)
  double alpha, beta, rho, rho_prev;
  double rr;        // current ||r||^2 (recursive, or FP64 true after a replacement)
  double tol2;      // rtol^2 ||M phi||^2
  double bb;        // ||M phi||^2
  double res2;      // final true ||M phi - S x||^2 (that of the last replacement)
  double energy2;   // final sum M x^2
  double rr_best;   // complex tiles: the smallest true ||r||^2 so far (stall detection)
  double alpha_hist[kChunk];  // alpha of each iteration of the current chunk (0 if not iterating)
  double beta_hist[kChunk];   // beta of each iteration of the current chunk (p_k = z_k + beta_k p_k-1)
  double pq;                  // (p, S p) of the last iteration
  int32_t active;   // slot holds a column
  int32_t done;     // 0 running, 1 converged, 2 breakdown, 3 max_iter
  int32_t iters;    // CG iterations of this column
  int32_t updates;  // FP64 residual replacements
  int32_t rr_true;  // rr is an FP64 true residual
  int32_t stall;    // complex tiles: chunk ends since rr_best last fell by 10%
};

// The handle's matrix as the batched kernels see it (device pointers).
struct BatchMatrix {
  int64_t n = 0, n_slices = 0, n_pad = 0;
  const int64_t* sptr = nullptr;
  const int32_t* col = nullptr;
  const double* val64 = nullptr;
  const float* val32 = nullptr;
  const double* kdiag = nullptr;
  const double* mass = nullptr;
  const int64_t* entity = nullptr;
  const int32_t* row_of = nullptr;  // caller index -> row (-1: no dof), field_len entries
  int64_t field_len = 0;
  int G = 1;   // blocks of the kernels that gather (SpMV, replacement, start, finish)
  int Gu = 1;  // blocks of the complex tiles' x update (the real tiles' x update is one-pass)
  int head = 6;  // off-diagonal entries per row in the gathering kernels' pipelined head (6, 12 or 20;
                 // with pairs: blocks per block row, 3, 6 or 12)
  // two-component operators: the gathering kernels run on 2 x 2 blocks
  // (each lane handles both component rows of a block row and gathers a
  // neighbour's two components together); the vectors keep their layout
  bool pairs = false;
  int64_t nb = 0, nb_slices = 0, pnnz = 0;  // block rows, slices of 64 of them, stored block entries
  const int64_t* psptr = nullptr;
  const int32_t* pcol = nullptr;
  const double* pval64 = nullptr;  // 4 per entry
  const float* pval32 = nullptr;
  int chunk = 4;  // iterations per chunk (chunk_for_order of the handle)
};

struct BatchParams {
  int max_iter = 20000;
  hipEvent_t ev_begin = nullptr;  // if set: recorded around the second SpMV launch
  hipEvent_t ev_end = nullptr;
  bool graphs = true;             // replay whole chunks as captured HIP graphs
};

// Algorithmic bytes of one launch of the fused iteration kernel (the second
// to fourth iteration of a chunk, the one batch_iterate times) with 'live'
// active columns: the sliced-ELL stream, mass and diagonal, and per live
// column the reads of z, u and p (each once) and the writes of z, u and p.
double batch_spmv_bytes(const BatchMatrix& bm, int64_t nnz_stored, bool mixed, int live);

// Device work space of one tile of R slots (vectors rows x R).
struct BatchWork {
  int R = 0;
  int G = 0, Gu = 0;  // grid sizes the work space (partial-sum array) was made for
  bool mixed = false;
  // complex tile: columns 2j, 2j + 1 are the real and imaginary parts of
  // one complex-shifted first-order system (Jacobi-COCG); slot 2j + 1
  // carries the imaginary parts of the scalars, sigma in its c
  bool cx = false;
  // complex tiles: a column pair stops when |r|^2 <= (rtol / (1 + |sigma| g))^2
  // ||M phi||^2, g >= ||K M^-1||_2 (the handle's bound), so that the residual
  // of S_2 itself, Re r + b K M^-1 Im r, meets rtol
  double cx_g = 0.0;
  // Vectors of a chunk: z_k of iteration k < kChunk - 1 stays in z[k] for
  // the whole chunk (z[0] from the FP64 replacement), u = diag(S)^-1 S p
  // alternates between two buffers (an iteration gathers the previous one
  // while it writes the new), and p[kChunk - 1] holds the carried direction;
  // the x update rebuilds the chunk's directions from them (p[0..kChunk - 1)
  // stay unallocated).
  float *z32[kChunk] = {}, *u32[2] = {}, *p32[kChunk] = {};
  double *z64[kChunk] = {}, *u64[2] = {}, *p64[kChunk] = {};
  double* x = nullptr;    // FP64 solution, rows x R (updated once per chunk)
  double* phi = nullptr;  // FP64 fields, rows x R
  double* part = nullptr; // per-(quantity, column, block) partial sums
  BSlot* slots = nullptr;
  BSlot* slots_host = nullptr;  // pinned
  int* flag = nullptr;
  int64_t iter = 0;       // tile iterations so far (position in the chunk)
  int chunk = 4;          // iterations per chunk (chunk_for_order)
  // one captured chunk (kChunk iterations), rebuilt when max_iter changes
  hipGraphExec_t chunk_exec = nullptr;
  int chunk_max_iter = 0;
  bool graphs_broken = false;  // capture failed once: launch directly
};

// Scale factors c_j of the slots being initialised (kernel argument).
struct SlotScales {
  double c[64];
};

// Device bytes of a tile's work space (the vectors of BatchWork).
size_t batch_bytes(int64_t n_pad, int R, bool mixed, int chunk);
// Lanes that share one row in a tile of R columns (each lane owns 16 bytes of
// columns: 4 FP32 or 2 FP64).
int batch_lanes_per_row(int R, bool mixed);
// Blocks of the batched SpMV kernel that are resident on the device at once.
int batch_resident_blocks(int R, bool mixed, int device);
// Allocate a tile of R columns; cx: a complex tile (of the first-order
// operator).
ifl_status batch_alloc(BatchWork* w, const BatchMatrix& bm, int R, bool mixed, bool cx = false);
void batch_free(BatchWork* w);

ifl_status batch_clear_flag(BatchWork& w, hipStream_t s);
// Gather one field (caller numbering, device) into column 'slot' of phi;
// non-finite entries raise the device flag (read with batch_check_flag).
ifl_status batch_load_column(const BatchMatrix& bm, BatchWork& w, int slot, const double* field_dev, hipStream_t s);
// Gather several fields at once: fields_dev[j] (device; caller numbering, or
// row order when 'internal') into column j of phi for every slot j in 'mask'.
ifl_status batch_load_columns(const BatchMatrix& bm, BatchWork& w, uint64_t mask, const double* const* fields_dev,
                              bool internal, hipStream_t s);
// n_fields device fields in the caller's numbering (stride L) -> row order
// (stride n_pad) in dst; non-finite wet entries set *flag (device int).
ifl_status batch_permute_fields(const BatchMatrix& bm, const double* src, int64_t L, int n_fields, double* dst,
                                int* flag, hipStream_t s);
ifl_status batch_check_flag(BatchWork& w, hipStream_t s, bool* bad);
// A pseudo-random column (for timing trials) into column 'slot' of phi.
ifl_status batch_load_synthetic(const BatchMatrix& bm, BatchWork& w, int slot, uint64_t seed, hipStream_t s);
// Start the columns in 'mask' (their phi columns loaded) at scales cs.
ifl_status batch_init(const BatchMatrix& bm, BatchWork& w, uint64_t mask, const SlotScales& cs, double rtol,
                      hipStream_t s);
ifl_status batch_iterate(const BatchMatrix& bm, BatchWork& w, int n_iter, const BatchParams& prm, hipStream_t s);
// Write x of the columns in 'mask' to out[slot] (caller numbering, every
// entry: 0 where there is no dof) and compute their energy into the slot
// state (their true residual is that of the last replacement).
ifl_status batch_finish(const BatchMatrix& bm, BatchWork& w, uint64_t mask, double* const* out, hipStream_t s);
ifl_status batch_read_slots(BatchWork& w, hipStream_t s);
// Move n running columns (slots from[c] of src -> to[c] of dst, a tile of
// another width and the same precision) at a chunk boundary; the other
// slots of dst become idle. Both tiles must be sized for bm's rows.
ifl_status batch_move_columns(const BatchMatrix& bm, BatchWork& src, BatchWork& dst, const int* from, const int* to,
                              int n, hipStream_t s);
ifl_status batch_release(BatchWork& w, uint64_t mask, hipStream_t s);

// The handle's matrix for tiles of R columns, and the sum of its mass
// (both need a device handle; defined with the device state).
BatchMatrix handle_batch_matrix(Handle* h, int R, bool mixed);
// Complex tiles of the order-2 shifted solves: whether the handle runs them
// (IFL_SOLVER_SHIFTED, order 2, a first-order operator with narrow rows),
// their matrix (the first-order operator), and the shift of a column at
// wavenumber k (slot 2j's and 2j + 1's c).
bool handle_cx_tiles(const Handle* h);
BatchMatrix handle_batch_matrix_k1(Handle* h, int R, bool mixed);
void cx_shift(const Handle* h, double k, double* sigma_re, double* sigma_im);
// g >= ||K M^-1||_2 for the first-order operator K of an order >= 2 handle
double handle_cx_gnorm(const Handle* h);
double handle_mass_sum(const Handle* h);

}  // namespace ifl
