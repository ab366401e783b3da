// Internal declarations of the implicit-filter library (not part of the ABI).
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "ifl.h"

namespace ifl {

// Sets the thread-local error message and returns the status.
ifl_status fail(ifl_status st, const std::string& msg);

// ----------------------------------------------------------------- host side
// The prepared operator in host memory, rows in the library's internal
// (locality) order. K_n is stored in CSR with sorted columns and its
// diagonal included; the system of a solve is S = diag(mass) + c K_n.
struct HostOperator {
  int32_t placement = IFL_VERTEX_SCALAR;
  int32_t order = 1;
  int64_t n = 0;                   // rows (unknowns)
  int64_t field_len = 0;           // length of a field in the caller's numbering
  std::vector<int64_t> entity;     // caller index of each row
  std::vector<int64_t> row_ptr;    // n + 1
  std::vector<int32_t> col;        // nnz
  std::vector<double> val;         // nnz
  std::vector<double> mass;        // n
  // order >= 2: the first-order operator K (same rows and layout), for the
  // solves of S = M + c K_n as shifted first-order systems
  std::vector<int64_t> k1_row_ptr;
  std::vector<int32_t> k1_col;
  std::vector<double> k1_val;
  int32_t n_components = 1;        // 1 (scalar) or 2 (vector)
  uint64_t mesh_hash = 0;
  // IFL_VERTEX_VECTOR only: the cell -> vertex projection R_vc u_c / M_v.
  // Rows 2d and 2d+1 are dof d; its incident active triangles are
  // proj_tri[proj_ptr[d] .. proj_ptr[d+1]) with weights (A_c / 3) / M_d.
  int64_t n_cells = 0;             // triangles of the mesh (cell field: 2 n_cells)
  std::vector<int64_t> proj_ptr;   // n / 2 + 1
  std::vector<int32_t> proj_tri;
  std::vector<double> proj_w;
};

// Mesh -> operator (prepare phase). 'reorder' selects the reverse
// Cuthill-McKee ordering of the dofs.
ifl_status build_operator(const ifl_mesh& mesh, int32_t placement, int32_t order, double cell_A,
                          int32_t reorder, HostOperator* out);

// Sliced-ELL packing used by the device kernels: rows in slices of 64
// (one wavefront); slice s stores its off-diagonal entries column-major,
// entry k of lane l at slice_ptr[s] + 64 k + l, padded to the widest row
// of the slice with (col = row, val = 0).
struct SellPack {
  int64_t n = 0;
  int64_t n_slices = 0;
  std::vector<int64_t> slice_ptr;  // n_slices + 1
  std::vector<int32_t> col;
  std::vector<double> val;
  std::vector<double> diag;        // K_n diagonal, n_slices * 64 (zero padded)
  std::vector<double> mass;        // n_slices * 64 (pads: 0)
  int32_t max_width = 0;
  int64_t stored_offdiag = 0;      // true off-diagonal entries (no padding)
};

void pack_sell(const HostOperator& op, SellPack* out);
void pack_sell_csr(int64_t n, const std::vector<int64_t>& row_ptr, const std::vector<int32_t>& col,
                   const std::vector<double>& val, const std::vector<double>& mass, SellPack* out);

// 2 x 2-block sliced ELL of a two-component operator (rows 2b and 2b + 1
// are the two components of block row b, as the vector placements number
// them): slices of 64 block rows; entry k of block row 64 s + l, at
// slice_ptr[s] + 64 k + l, holds a block column j and the four couplings
// (row 2b to 2j, row 2b to 2j + 1, row 2b + 1 to 2j, row 2b + 1 to 2j + 1)
// at val[4 (slice_ptr[s] + 64 k + l) ..]. Block columns increase along a
// block row; the diagonal of K_n is not stored (a block on the diagonal
// keeps only the coupling of the two components, and exists only if that
// coupling does); rows are padded to the slice's width with (block row,
// zeros), and kSellTail zero entries follow the last slice.
struct PairPack {
  int64_t nb = 0;        // block rows
  int64_t n_slices = 0;  // slices of 64 block rows
  std::vector<int64_t> slice_ptr;
  std::vector<int32_t> col;
  std::vector<double> val;  // 4 per entry
  int64_t stored_blocks = 0;  // blocks with a coupling (no padding)
};

// Packs op as 2 x 2 blocks; false (and out untouched) unless op has two
// components.
bool pack_pairs(const HostOperator& op, PairPack* out);

// Zero entries appended after the last slice (32 entries x 64 lanes): a
// kernel may load up to 32 entries past the end of any slice's rows without
// a bounds check.
constexpr int64_t kSellTail = 32 * 64;

// ---------------------------------------------------------------- device side
struct DeviceState;  // defined in device.hip

struct Handle {
  ifl_options opt{};
  HostOperator op;
  DeviceState* dev = nullptr;
  std::mutex mu;
};

ifl_status device_create(Handle* h);
void device_destroy(Handle* h);

// Solve n_fields x n_scales columns. fields / out may be host or device.
ifl_status device_filter(Handle* h, int32_t n_fields, const double* fields, int32_t n_scales,
                         const double* k, double* out, ifl_solve_stats* stats, double* energy);
// The one-column path with its partials and scalars in the library's static
// device work space (no allocation; device fields and outputs only).
ifl_status device_filter_noalloc(Handle* h, int32_t n_fields, const double* fields, int32_t n_scales,
                                 const double* k, double* out, ifl_solve_stats* stats);
ifl_status device_apply(Handle* h, double k, const double* x, double* y);
// Cell velocities (2 n_cells, host or device) -> the projected vertex field
// R_vc u_c / M (field_len, host or device; 0 where there is no dof).
ifl_status device_project_cells(Handle* h, const double* cells, double* out);
ifl_status device_profile_read(Handle* h, int64_t* launches, double* total_ms, double* bytes,
                               int32_t reset);
std::string device_profile_kernel(Handle* h);
ifl_status device_stream_probe(int device, int64_t bytes, int reps, double* best_gbs, double* median_gbs);
// One column of a served request on a handle of order >= 2 with
// IFL_SOLVER_SHIFTED: the field in row order (device, the handle's rows),
// wavenumber k, the result to out_dev in the caller's numbering (device;
// NULL: energy only). Runs on the handle's stream; the caller holds h->mu.
ifl_status device_solve_shifted_rows(Handle* h, const double* phi_rows, double k, double* out_dev,
                                     ifl_solve_stats* st);
// Allocates (once per handle) the work space of the shifted solves and
// returns its size in bytes; the caller holds h->mu.
ifl_status device_shift_work(Handle* h, size_t* bytes);
ifl_status device_autotune(Handle* h, ifl_tune* out);

}  // namespace ifl

// The ABI's opaque handle is the library's Handle.
struct ifl_handle : ifl::Handle {};
