/*
 * ifl.h -- C ABI of the implicit-filter library (MI355X / gfx950).
 *
 * The library solves the implicit filter of Nowak, Danilov, Mueller & Liu,
 * "Implementation of implicit filter for spatial spectra extraction":
 *
 *     (1 + gamma (-l^2 Lap)^n) phi_bar = phi            (Eq. 1, Eq. 2)
 *
 * discretised on an unstructured triangle mesh as the SPD system
 *
 *     S phi_bar = M phi,   S = M + (gamma / k^(2n)) K_n,   k = 1/l,
 *
 * with M the lumped median-dual (vertex) or triangle (cell) areas and K_n
 * the order-n Laplacian (Sect. 2.1.1 and Eq. 4/5 for vertex scalars,
 * Eq. 7 for cell vectors). The work is split into a mesh-only prepare
 * phase, run once, and a per-scale solve (Sect. 2.2): Jacobi-preconditioned
 * conjugate gradients started from x0 = phi, i.e. on the residual form
 * where S phi is subtracted from the right-hand side (Sect. 2.2.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns IFL_OK (0) or a negative ifl_status. On an error
 *    other than IFL_ENOTCONV the outputs are left untouched; the message of
 *    the last error of the calling thread is returned by ifl_last_error().
 *  - Field pointers ("fields", "field", "out") may be host memory or device
 *    memory of the handle's device; the library tells them apart with
 *    hipPointerGetAttributes. Everything else (mesh arrays, k lists, stats,
 *    energies) is host memory.
 *  - The caller owns all buffers it passes. Except for ifl_submit, no call
 *    keeps a caller pointer after it returns.
 *  - Calls on one handle are synchronous with respect to the host and are
 *    serialised by a per-handle lock; different handles may be used from
 *    different threads.
 *  - Wavenumbers k are in radians per unit of the mesh coordinates
 *    (k = 2 pi / wavelength), must be finite and > 0.
 */
#ifndef IFL_H
#define IFL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef int32_t ifl_status;
#define IFL_OK 0
#define IFL_EINVAL (-1)       /* null / NaN / Inf input, k <= 0, bad index or size */
#define IFL_EDEGENERATE (-2)  /* zero-area triangle, or no active triangle at all */
#define IFL_ENOMEM (-3)       /* host or device allocation failed */
#define IFL_ENOTCONV (-4)     /* max_iter reached or CG breakdown; out holds the last iterate */
#define IFL_EDEVICE (-5)      /* HIP runtime error, or no usable gfx950 device */
#define IFL_EUNSUPPORTED (-6) /* placement / order / option not implemented */
#define IFL_EIO (-7)          /* save / load failure or bad file */
#define IFL_ECANCELED (-8)    /* a served request cancelled by ifl_server_cancel before it finished */

/* ------------------------------------------------------------------ mesh */
#define IFL_GEOM_PLANAR 0   /* coords V x 2 (x, y) */
#define IFL_GEOM_PERIODIC 1 /* coords V x 2, doubly periodic with period[0], period[1] */
#define IFL_GEOM_SPHERE 2   /* coords V x 3 (x, y, z) on a sphere; flat facets */

typedef struct ifl_mesh {
  int64_t n_vertices;       /* V >= 3 */
  int64_t n_triangles;      /* F >= 1 */
  const double* coords;     /* host, V x 2 or V x 3, row-major */
  const int32_t* triangles; /* host, F x 3 vertex ids, 0-based; any orientation */
  int32_t geometry;         /* IFL_GEOM_* */
  int32_t reserved0;
  double period[2];         /* IFL_GEOM_PERIODIC only */
  const uint8_t* wet;       /* host, V entries, 1 = wet (ocean), 0 = dry; NULL = all wet */
} ifl_mesh;

/* Data placement (Sect. 2.1, Fig. 1). */
#define IFL_VERTEX_SCALAR 0       /* scalars on vertices, median-dual CVs, P1 FE (Sect. 2.1.1) */
#define IFL_CELL_VECTOR 1         /* (east, north) vectors on triangles, Eq. 7 (Sect. 2.1.2) */
#define IFL_VORONOI_SCALAR 2      /* scalars on vertices, quasi-hexagonal (Voronoi) CVs, Eq. 3-5 */
#define IFL_CIRCUMCENTER_SCALAR 3 /* scalars at triangle circumcentres, Eq. 6 */
#define IFL_VERTEX_VECTOR 4       /* (east, north) vectors on vertices, FE vector Laplacian (Sect. 2.1.2) */

/* Arithmetic of the solve. */
#define IFL_FP64 0  /* all vectors, matrix values, SpMV and reductions in FP64 */
#define IFL_MIXED 1 /* FP32 matrix values / vectors / SpMV, FP64 reductions, FP64 residual
                       replacement ("reliable updates") and FP64 solution accumulation */

/* How the system S = M + c K_n of an order n >= 2 is solved. */
#define IFL_SOLVER_KN 0      /* Jacobi-preconditioned CG on S itself (Sect. 2.2.2; default) */
#define IFL_SOLVER_SHIFTED 1 /* the same S^-1 M phi through first-order systems only:
                                S^-1 = (1/n) sum_j (M + s_j c^(1/n) K)^-1 with s_j = -1/w_j over the
                                roots of w^n = -1 (partial fractions of 1/(1 + y^n) in the
                                eigenvalues y of c^(1/n) M^-1 K); each complex-shifted system by
                                Jacobi-preconditioned COCG (CG in the bilinear form), a real shift
                                (odd n) by CG; conjugate shifts share one solve. Each shifted system
                                stops on its own FP64 true residual; one column at a time. */

typedef struct ifl_options {
  double gamma;      /* filter parameter (Sect. 2.1: 1/2); default 0.5 */
  double rtol;       /* stop when ||M phi - S x||_2 <= rtol * ||M phi||_2; default 1e-12 */
  int32_t max_iter;  /* CG iteration cap per solve; default 20000. Tiles (batch != 1) test their
                        columns at the end of each 4-iteration chunk, on an FP64 true residual, so
                        there the cap and the iteration counts are rounded up to a multiple of 4 */
  int32_t precision; /* IFL_FP64 (default) or IFL_MIXED */
  double cell_A;     /* stencil constant A of Eq. 7; default sqrt(3) */
  int32_t device;    /* HIP device ordinal; default 0. -1 = host-only handle: prepare,
                        export and save work, solves return IFL_EDEVICE */
  int32_t batch;     /* columns per multi-RHS tile for ifl_filter: 0 = auto (default: the autotuner's
                        width, else 32, at most a quarter of the call's columns), 1 = one solve at a
                        time, 2..64 = fixed tile (rounded down to a power of two) */
  void* stream;      /* hipStream_t to run on; NULL = the handle's own stream */
  int32_t reorder;   /* 1 = locality ordering of the rows (default): reverse Cuthill-McKee, on meshes of
                        >= 32768 dofs inside 8 Morton-curve parts; 0 = mesh order */
  int32_t profile;   /* 1 = time the SpMV launches with HIP events (ifl_profile_read) */
  int32_t graphs;    /* 1 = the batched engine replays each 4-iteration chunk of a tile as one captured
                        HIP graph (default), 0 = launches every kernel; results are bitwise equal */
  int32_t solver;    /* IFL_SOLVER_KN (default) or IFL_SOLVER_SHIFTED (orders n >= 2; n = 1 uses
                        IFL_SOLVER_KN). With SHIFTED, ifl_filter and ifl_spectrum run n = 2 in complex
                        tiles of 'batch' / 2 columns (batch 0: the library's width; scalar operators
                        with first-order rows of at most 6 entries 90% of the time), other orders and
                        batch = 1 one column at a time; the serving engine serves n = 2 in a complex
                        tile of 2 x slots real columns (slots <= 32), other orders one column at a
                        time. Each shifted system stops on its own FP64 true residual: at rtol one
                        column at a time; in n = 2 tiles at rtol / (1 + |sigma| g), g >= ||K M^-1||,
                        so that the residual of S_2 meets rtol (a tile column whose residual stalls
                        above that stops at rtol). Tiles report the shifted system's FP64 true
                        residual in rel_residual, one column at a time that of S_n */
} ifl_options;

/* Per-solve statistics (one per field x scale). */
typedef struct ifl_solve_stats {
  int32_t iterations;   /* CG iterations */
  int32_t refinements;  /* FP64 residual replacements (IFL_MIXED, and tiles of either precision) */
  int32_t status;       /* IFL_OK or IFL_ENOTCONV */
  int32_t reserved;
  double rel_residual;  /* final ||M phi - S x|| / ||M phi||, FP64 on the GPU */
  double seconds;       /* wall time of the solve (of its tile when batched) */
  double energy;        /* filtered energy of the column, 1/2 sum M x^2 / sum M (the spectra of Sect. 4) */
} ifl_solve_stats;

typedef struct ifl_handle ifl_handle;

/* Fill *opt with the defaults listed above. */
void ifl_default_options(ifl_options* opt);

/*
 * Mesh-only preparation (Sect. 2.2.1), run once per mesh and order.
 *
 * Builds, on the host, the active triangles (all three vertices wet), the
 * dofs (vertices of an active triangle for the vertex placements; active
 * triangles for IFL_CELL_VECTOR and IFL_CIRCUMCENTER_SCALAR), flat-facet
 * geometry, the lumped mass and the stiffness K, the order-n operator
 * K_n = K (M^-1 K)^(n-1), a locality ordering of the dofs, and uploads the
 * matrix to device memory owned by the handle. K and M per placement:
 *   IFL_VERTEX_SCALAR       P1 Galerkin stiffness, median-dual areas (Sect. 2.1.1);
 *   IFL_VORONOI_SCALAR      Eq. 3 (its l/d weights are the P1 cotangent weights),
 *                           circumcentric (Voronoi) cell areas; IFL_EDEGENERATE
 *                           where a cell area is not positive;
 *   IFL_CIRCUMCENTER_SCALAR Eq. 6 between triangles sharing an edge, triangle
 *                           areas; the circumcentre distance is measured through
 *                           the shared edge's midpoint; IFL_EDEGENERATE where it
 *                           is not positive (e.g. right triangles sharing their
 *                           hypotenuse);
 *   IFL_CELL_VECTOR         Eq. 7 with the change of local unit vectors between
 *                           neighbouring cells, triangle areas;
 *   IFL_VERTEX_VECTOR       D_2 = [[D~, T], [-T, D~]] of Sect. 2.1.2 on P1 elements:
 *                           D~ = stiffness + (1/R_e^2 + m^2) consistent mass, T the
 *                           metric coupling, m = tan(latitude) / R_e constant on a
 *                           triangle (taken at its centroid, R_e its mean corner
 *                           radius; m = 0 and 1/R_e^2 = 0 on planar meshes),
 *                           median-dual areas; IFL_EDEGENERATE if an active
 *                           triangle's centroid lies on the polar axis. Lon/lat
 *                           components are singular at the poles: put the poles
 *                           on land (rotated meshes do) for accurate results.
 * Fields are per vertex (L = n_vertices) for the vertex scalar placements, per
 * triangle (L = n_triangles) for IFL_CIRCUMCENTER_SCALAR, (east, north) per
 * triangle (L = 2 n_triangles) for IFL_CELL_VECTOR and (east, north) per vertex
 * (L = 2 n_vertices) for IFL_VERTEX_VECTOR, whose fields come from cell
 * velocities through ifl_project_cells.
 *
 * mesh      : host arrays, read only during the call.
 * placement : IFL_VERTEX_SCALAR, IFL_VORONOI_SCALAR, IFL_CIRCUMCENTER_SCALAR,
 *             IFL_CELL_VECTOR or IFL_VERTEX_VECTOR.
 * n         : filter order, 1 to 4 (others: IFL_EUNSUPPORTED). K_n is assembled
 *             explicitly: for vertex scalars on a triangular mesh its rows hold
 *             about 7, 19, 37 and 61 entries for n = 1..4. The condition number
 *             of S grows like gamma (lambda_max / k^2)^n, so high orders need
 *             many iterations at large scales and can stop converging there,
 *             as the paper reports for n = 2 (Sect. 4 and the "Some comments"
 *             section); on a uniform mesh n = 4 converges within 20,000
 *             iterations up to wavelengths of about 20 grid steps in FP64 and
 *             11 in mixed precision.
 * opt       : NULL for defaults; copied into the handle.
 * out       : receives the handle; release with ifl_destroy.
 * Errors    : IFL_EINVAL (bad sizes, ids out of range, non-finite coords,
 *             unknown placement), IFL_EDEGENERATE (zero-area active triangle,
 *             no active triangle, and the per-placement cases above),
 *             IFL_EUNSUPPORTED (order), IFL_ENOMEM, IFL_EDEVICE.
 */
ifl_status ifl_prepare(const ifl_mesh* mesh, int32_t placement, int32_t n,
                       const ifl_options* opt, ifl_handle** out);

/* Release the handle and all its host and device memory. NULL is a no-op. */
void ifl_destroy(ifl_handle* h);

/* Number of unknowns of the solve (dofs, times 2 for vectors). */
int64_t ifl_num_dofs(const ifl_handle* h);

/* Length of one field in the caller's numbering: V for vertex scalars, F
 * for circumcentre scalars, 2F for cell vectors and 2V for vertex vectors
 * (interleaved east, north). */
int64_t ifl_field_length(const ifl_handle* h);

/* IFL_VERTEX_VECTOR handles: the number of triangles F of the mesh (the
 * cell field of ifl_project_cells has 2F doubles); 0 for other placements. */
int64_t ifl_num_cells(const ifl_handle* h);

/* Replace the solver options of a prepared handle (gamma, rtol, max_iter,
 * precision, batch, stream, profile). Mesh-dependent fields (cell_A,
 * device, reorder) must equal the prepare-time values, else IFL_EINVAL. */
ifl_status ifl_set_options(ifl_handle* h, const ifl_options* opt);

/* Copy the handle's current options into *out (to change some of them with
 * ifl_set_options). IFL_EINVAL on NULL arguments. */
ifl_status ifl_get_options(const ifl_handle* h, ifl_options* out);

/*
 * Filter n_fields fields at n_scales wavenumbers (Eq. 1 discretised as
 * above; solve of Sect. 2.2.2).
 *
 * fields : n_fields x L doubles, L = ifl_field_length(h), row-major; entries
 *          at dry vertices / inactive cells are ignored. Host or device.
 * k      : host, n_scales wavenumbers (> 0, finite).
 * out    : n_fields x n_scales x L doubles; out[f][s] is field f filtered at
 *          k[s]; dry entries are written as 0. Host or device.
 * stats  : host, n_fields x n_scales entries, or NULL.
 * Errors : IFL_EINVAL (NaN/Inf in a wet entry of a field, bad k, bad sizes),
 *          IFL_ENOTCONV (some column hit max_iter or broke down: out holds
 *          the last iterates and stats say which), IFL_EDEVICE, IFL_ENOMEM.
 * n_fields == 0 or n_scales == 0 is a valid no-op.
 */
ifl_status ifl_filter(ifl_handle* h, int32_t n_fields, const double* fields,
                      int32_t n_scales, const double* k, double* out,
                      ifl_solve_stats* stats);

/*
 * ifl_filter for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solves as ifl_filter with the one-column path (every column
 * solved on its own; bitwise the results of ifl_filter with
 * ifl_options.batch = 1), but the per-call work space (block partial sums
 * and per-column scalars) lives in a static device array of 64 KiB that the
 * library holds on each GPU until the process ends. The call allocates
 * nothing: no hipMalloc / hipFree, no events, no staging buffers.
 *
 * fields : device, n_fields x L doubles on the handle's device.
 * out    : device, n_fields x n_scales x L doubles on the handle's device.
 * k, stats : as ifl_filter (host).
 * Limits : the handle's logical block count G must satisfy 14 G x 8 bytes
 *          <= 65,280 (G <= 582; the default is at most 512); otherwise
 *          IFL_EINVAL with a message naming both sizes. Host pointers for
 *          fields or out are IFL_EINVAL. Profiling (ifl_options.profile)
 *          is ignored, and orders n >= 2 are solved by Jacobi-PCG on S_n
 *          whatever ifl_options.solver says (the shifted solves need work
 *          space of their own).
 * All handles on one GPU share its work space, which keeps the last call's
 * contents (each call clears it first): calls that overlap on one GPU
 * (from several threads, or on several handles' streams) race; serialise
 * them. Calls on one handle are serialised by the handle's lock.
 * Errors : as ifl_filter.
 */
ifl_status ifl_filter_noalloc(ifl_handle* h, int32_t n_fields, const double* fields,
                              int32_t n_scales, const double* k, double* out,
                              ifl_solve_stats* stats);

/*
 * Coarse-graining spectrum of one field (Sect. 2.1, Sect. 4): the filtered
 * energy E(k_j) = (1/2) sum_i M_i phi_bar_i(k_j)^2 / sum_i M_i at each k_j
 * (for vectors phi_bar^2 = u_bar^2 + v_bar^2), and its finite-difference
 * density (E_{j+1} - E_j) / (k_{j+1} - k_j) at k_mid = sqrt(k_j k_{j+1}).
 *
 * field   : L doubles, host or device.
 * k       : host, n_scales > 0 wavenumbers, strictly ascending.
 * energy  : host, n_scales doubles.
 * density : host, n_scales - 1 doubles, or NULL.
 * k_mid   : host, n_scales - 1 doubles, or NULL.
 * Errors  : as ifl_filter; IFL_EINVAL if k is not strictly ascending.
 */
ifl_status ifl_spectrum(ifl_handle* h, const double* field, int32_t n_scales,
                        const double* k, double* energy, double* density,
                        double* k_mid);

/*
 * y = S(k) x in the caller's numbering (the operator of the solve, for
 * checks and for callers that want the residual themselves).
 * x, y : L doubles each, host or device; dry entries of y are 0.
 */
ifl_status ifl_apply(ifl_handle* h, double k, const double* x, double* y);

/*
 * Right-hand side of the vertex vector filter (Sect. 2.1.2): the paper
 * projects cell velocities u_c to vertices by R_vc = integral of N_v over
 * cell c (A_c / 3 for each corner of an active cell, component by
 * component). This writes the vertex field f = M^-1 R_vc u_c, so that
 * ifl_filter(f) solves S u_bar = M f = R_vc u_c (and starts from f).
 * Needs an IFL_VERTEX_VECTOR handle with a device (else IFL_EINVAL /
 * IFL_EDEVICE).
 * cells : 2 n_triangles doubles, (east, north) per triangle, host or device;
 *         entries of inactive triangles are not read; non-finite values
 *         propagate (ifl_filter then rejects the field).
 * out   : L = 2 n_vertices doubles, host or device; 0 at vertices that are
 *         not dofs. Synchronous.
 */
ifl_status ifl_project_cells(ifl_handle* h, const double* cells, double* out);

/*
 * Export the prepared operator to host memory (checks, debugging).
 * Rows are the dofs in the library's internal order. With nnz = the value
 * returned by ifl_operator_nnz:
 *   row_ptr[N+1], col[nnz] (internal dof ids), val[nnz] : K_n in CSR, FP64,
 *   including its diagonal;
 *   mass[N] : lumped mass;
 *   entity[N] : caller-numbering index of each dof (vertex id, or
 *               2*triangle + component for cell vectors).
 * Any pointer may be NULL to skip that array.
 */
int64_t ifl_operator_nnz(const ifl_handle* h);
ifl_status ifl_export_operator(const ifl_handle* h, int64_t* row_ptr, int32_t* col,
                               double* val, double* mass, int64_t* entity);

/*
 * The first-order operator K of a handle (same rows and layout as
 * ifl_export_operator; for order 1 it is K_n itself), which
 * IFL_SOLVER_SHIFTED solves with. nnz = ifl_first_order_nnz(h).
 */
int64_t ifl_first_order_nnz(const ifl_handle* h);
ifl_status ifl_export_first_order(const ifl_handle* h, int64_t* row_ptr, int32_t* col, double* val);

/* Save / load a prepared handle (Sect. 2.2.1: the precomputed arrays can be
 * saved to disk and reused). Versioned little-endian binary. ifl_load
 * uploads to opt->device (NULL opt: defaults). Errors: IFL_EIO. */
ifl_status ifl_save(const ifl_handle* h, const char* path);
ifl_status ifl_load(const char* path, const ifl_options* opt, ifl_handle** out);

/* Thread-local message of the last error ("" if none). */
const char* ifl_last_error(void);

/*
 * SpMV launch timing, for roofline reports (requires opt.profile = 1).
 * Returns the number of timed SpMV launches since the last reset, their
 * summed duration in milliseconds (HIP events on the launch stream), and
 * the algorithmic bytes one launch moves (matrix stream + vector reads and
 * writes, without cache effects). reset != 0 clears the counters.
 */
ifl_status ifl_profile_read(ifl_handle* h, int64_t* launches, double* total_ms,
                            double* bytes_per_launch, int32_t reset);

/*
 * Name of the SpMV kernel of the last timed launch, as a profiler lists it
 * (e.g. "kb_iter<float, 32, true, 6>"), NUL-terminated in buf (len bytes, the
 * name truncated to fit); "" before the first timed launch. IFL_EINVAL for
 * a NULL handle or buffer, IFL_EDEVICE for a host-only handle.
 */
ifl_status ifl_profile_kernel(ifl_handle* h, char* buf, int32_t len);

/*
 * Measured streaming bandwidth of a device, for roofline reports: a plain
 * copy of 'bytes' bytes (rounded down to 16-byte units; at least 16 MiB)
 * between two device buffers the call allocates and frees, each thread
 * moving 16 bytes once (one pass of 256-thread workgroups). Runs 'reps' timed copies (HIP events, after one untimed) and
 * returns the best and the median rate in GB/s (read + write bytes / time).
 * Not part of the filter; IFL_EINVAL on a bad argument, IFL_ENOMEM /
 * IFL_EDEVICE on a device failure.
 */
ifl_status ifl_stream_probe(int32_t device, int64_t bytes, int32_t reps, double* best_gbs, double* median_gbs);

/*
 * Autotuner of the batched engine (the multi-column CG of Sect. 2.2.2 run as
 * one SpMM-like pass per iteration). Times full tiles of pseudo-random
 * columns for tile sizes 16, 32 and 64 and several grid sizes of the
 * gathering and streaming kernels on this handle's matrix in the handle's
 * current precision, and keeps the fastest per column-iteration: the grid
 * sizes per tile size, and the tile size used by ifl_filter when
 * options.batch = 0. Results computed afterwards may differ from untuned
 * ones in the last bits (another reduction order); runs with the same
 * tuning are bitwise reproducible. Takes ~0.1-1 s; needs device memory for
 * one tile of 64 columns. out may be NULL.
 * Errors: IFL_EINVAL (NULL handle), IFL_EDEVICE (host-only handle or a HIP
 * failure), IFL_ENOMEM.
 */
typedef struct ifl_tune {
  int32_t batch;                   /* fastest tile size (columns per tile) */
  int32_t blocks_gather;           /* its blocks of the SpMV / replacement / start / finish kernels */
  int32_t blocks_update;           /* its blocks of the complex tiles' x update (the real tiles'
                                      x update is a one-pass launch, one thread per row and lane) */
  int32_t candidates;              /* configurations timed */
  double us_per_column_iteration;  /* measured cost of the fastest configuration */
} ifl_tune;

ifl_status ifl_autotune(ifl_handle* h, ifl_tune* out);


/* ----------------------------------------------------------- serving API */
typedef struct ifl_server ifl_server;
typedef struct ifl_ticket ifl_ticket;

/*
 * Continuous-batching server over prepared handles (one device).
 * hbm_budget_bytes : device memory the server may use for in-flight work
 *                    (vectors of admitted solves); requests wait until
 *                    their footprint fits.
 * slots            : maximum columns in flight per mesh (tile width), 1..64.
 */
ifl_status ifl_server_create(size_t hbm_budget_bytes, int32_t slots, ifl_server** out);

/* Register a handle (borrowed: it must outlive the server). Handles of the
 * same mesh prepared for n = 1 and n = 2 are separate entries. The handle's
 * options at this call fix how its requests run: in a tile of 'slots'
 * columns (IFL_SOLVER_KN), or, for n >= 2 with IFL_SOLVER_SHIFTED, one
 * column at a time through the shifted first-order solves. IFL_ENOMEM when
 * the work space (tile, or shifted-solve vectors, plus staging) does not fit
 * the budget. */
ifl_status ifl_server_add(ifl_server* s, ifl_handle* h, int32_t* mesh_id);

/*
 * Queue one request: field (host, L doubles) filtered at n_scales
 * wavenumbers into out (host, n_scales x L), or, with out = NULL, into the
 * filtered energies only (the spectrum of Sect. 4, in the stats ifl_wait
 * fills). Returns at once. field and out are borrowed: both must stay
 * valid and unchanged until ifl_wait returns for the ticket (the field is
 * read when the request is admitted). Solves are admitted into the mesh's
 * running tile as slots and memory free up; each result is the same as a
 * standalone ifl_filter within the handle's tolerance. A NaN or Inf at a
 * wet entry of the field fails the request with IFL_EINVAL (reported by
 * ifl_wait). out entries are written only for converged or ENOTCONV
 * columns.
 */
ifl_status ifl_submit(ifl_server* s, int32_t mesh_id, const double* field,
                      int32_t n_scales, const double* k, double* out, ifl_ticket** ticket);

/*
 * Memory accounting and request counters of a server (continuous batching
 * with admission by device-memory footprint). The footprint of a request is
 * its field copy on the device: 8 bytes per dof row, the dofs rounded up to
 * a multiple of 64 (its columns run in the mesh's tile, whose work space is
 * charged once, at ifl_server_add). A request is admitted when
 * tiles + used + its footprint <= budget, or when nothing is in flight, and
 * while fewer than 2 x slots of its mesh's admitted columns wait for a slot
 * (requests of a mesh are admitted in submission order).
 */
typedef struct ifl_server_info {
  size_t budget;          /* hbm_budget_bytes of ifl_server_create */
  size_t tiles;           /* work space of the registered meshes (tiles or shifted solves) */
  size_t used;            /* footprint of the requests in flight now */
  size_t peak_used;       /* largest 'used' so far */
  int64_t submitted;      /* requests accepted by ifl_submit */
  int64_t admitted;       /* requests that got device memory */
  int64_t completed;      /* requests finished (any status) */
  int64_t in_flight;      /* admitted and not finished */
  int64_t peak_in_flight; /* largest 'in_flight' so far */
  int64_t queued;         /* submitted, waiting for admission */
} ifl_server_info;

/* Fill *info (IFL_EINVAL on NULL arguments). Safe while requests run. */
ifl_status ifl_server_query(ifl_server* s, ifl_server_info* info);

/* Block until the request is done; fills stats[n_scales] (may be NULL) and
 * frees the ticket. Returns the request's status. */
ifl_status ifl_wait(ifl_ticket* t, ifl_solve_stats* stats);

/* 1 if done, 0 if not yet (non-blocking). */
int32_t ifl_poll(const ifl_ticket* t);

/* Latency of a finished request (seconds from submit to completion). */
double ifl_ticket_latency(const ifl_ticket* t);

/*
 * Cancel the outstanding work of a server: requests still waiting for
 * admission, and the columns of admitted requests that have not entered a
 * tile slot yet, finish with IFL_ECANCELED (a request with columns already
 * in slots completes those first; its outputs for cancelled columns are
 * not written). Columns already in slots run to their end. Later submits
 * are accepted as usual. For callers that stop serving with a queue
 * (shutdown, a bounded measurement window). IFL_EINVAL on NULL.
 */
ifl_status ifl_server_cancel(ifl_server* s);

/* Drain outstanding work and destroy the server. */
void ifl_server_destroy(ifl_server* s);

#ifdef __cplusplus
}
#endif

#endif /* IFL_H */
