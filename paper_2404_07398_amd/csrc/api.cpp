// C ABI of the implicit-filter library: argument checks, handle lifetime,
// save / load, and dispatch to the prepare and device layers.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

namespace ifl {

static thread_local std::string g_last_error;

ifl_status fail(ifl_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

static ifl_status check_options(const ifl_options& o) {
  if (!(o.gamma > 0) || !std::isfinite(o.gamma)) return fail(IFL_EINVAL, "gamma must be positive and finite");
  if (!(o.rtol > 0) || !(o.rtol < 1)) return fail(IFL_EINVAL, "rtol must be in (0, 1)");
  if (o.max_iter < 1) return fail(IFL_EINVAL, "max_iter must be >= 1");
  if (o.precision != IFL_FP64 && o.precision != IFL_MIXED) return fail(IFL_EINVAL, "unknown precision");
  if (o.batch < 0 || o.batch > 64) return fail(IFL_EINVAL, "batch must be in 0..64");
  if (o.graphs != 0 && o.graphs != 1) return fail(IFL_EINVAL, "graphs must be 0 or 1");
  if (o.solver != IFL_SOLVER_KN && o.solver != IFL_SOLVER_SHIFTED) return fail(IFL_EINVAL, "unknown solver");
  return IFL_OK;
}

static ifl_status check_k(int32_t n_scales, const double* k, bool ascending) {
  if (n_scales < 0) return fail(IFL_EINVAL, "n_scales < 0");
  if (n_scales > 0 && !k) return fail(IFL_EINVAL, "k is NULL");
  for (int32_t j = 0; j < n_scales; ++j) {
    if (!(k[j] > 0) || !std::isfinite(k[j])) return fail(IFL_EINVAL, "wavenumbers must be finite and > 0");
    if (ascending && j > 0 && !(k[j] > k[j - 1])) return fail(IFL_EINVAL, "wavenumbers must be strictly ascending");
  }
  return IFL_OK;
}

}  // namespace ifl

using namespace ifl;

extern "C" {

void ifl_default_options(ifl_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->gamma = 0.5;
  opt->rtol = 1e-12;
  opt->max_iter = 20000;
  opt->precision = IFL_FP64;
  opt->cell_A = std::sqrt(3.0);
  opt->device = 0;
  opt->batch = 0;
  opt->stream = nullptr;
  opt->reorder = 1;
  opt->profile = 0;
  opt->graphs = 1;
}

const char* ifl_last_error(void) { return g_last_error.c_str(); }

ifl_status ifl_prepare(const ifl_mesh* mesh, int32_t placement, int32_t n, const ifl_options* opt,
                       ifl_handle** out) {
  g_last_error.clear();
  if (!mesh || !out) return fail(IFL_EINVAL, "mesh / out is NULL");
  *out = nullptr;
  ifl_options o;
  ifl_default_options(&o);
  if (opt) o = *opt;
  ifl_status st = check_options(o);
  if (st != IFL_OK) return st;
  std::unique_ptr<ifl_handle> h(new (std::nothrow) ifl_handle());
  if (!h) return fail(IFL_ENOMEM, "out of host memory");
  h->opt = o;
  try {
    st = build_operator(*mesh, placement, n, o.cell_A, o.reorder, &h->op);
  } catch (const std::bad_alloc&) {
    return fail(IFL_ENOMEM, "out of host memory during prepare");
  }
  if (st != IFL_OK) return st;
  if (o.device >= 0) {
    st = device_create(h.get());
    if (st != IFL_OK) {
      device_destroy(h.get());
      return st;
    }
  }
  *out = h.release();
  return IFL_OK;
}

void ifl_destroy(ifl_handle* h) {
  if (!h) return;
  device_destroy(h);
  delete h;
}

int64_t ifl_num_dofs(const ifl_handle* h) { return h ? h->op.n : 0; }

int64_t ifl_field_length(const ifl_handle* h) { return h ? h->op.field_len : 0; }

int64_t ifl_num_cells(const ifl_handle* h) { return h ? h->op.n_cells : 0; }

ifl_status ifl_set_options(ifl_handle* h, const ifl_options* opt) {
  if (!h || !opt) return fail(IFL_EINVAL, "handle / options NULL");
  ifl_status st = check_options(*opt);
  if (st != IFL_OK) return st;
  if (opt->device != h->opt.device || opt->reorder != h->opt.reorder ||
      (h->op.placement == IFL_CELL_VECTOR && opt->cell_A != h->opt.cell_A))
    return fail(IFL_EINVAL, "device, reorder and cell_A are fixed at prepare time");
  std::lock_guard<std::mutex> lk(h->mu);
  h->opt = *opt;
  return IFL_OK;
}

ifl_status ifl_get_options(const ifl_handle* h, ifl_options* out) {
  if (!h || !out) return fail(IFL_EINVAL, "handle / out NULL");
  std::lock_guard<std::mutex> lk(const_cast<ifl_handle*>(h)->mu);
  *out = h->opt;
  return IFL_OK;
}

ifl_status ifl_filter(ifl_handle* h, int32_t n_fields, const double* fields, int32_t n_scales, const double* k,
                      double* out, ifl_solve_stats* stats) {
  g_last_error.clear();
  if (!h) return fail(IFL_EINVAL, "handle is NULL");
  if (n_fields < 0) return fail(IFL_EINVAL, "n_fields < 0");
  ifl_status st = check_k(n_scales, k, false);
  if (st != IFL_OK) return st;
  if (n_fields == 0 || n_scales == 0) return IFL_OK;
  if (!fields || !out) return fail(IFL_EINVAL, "fields / out is NULL");
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::lock_guard<std::mutex> lk(h->mu);
  return device_filter(h, n_fields, fields, n_scales, k, out, stats, nullptr);
}

ifl_status ifl_filter_noalloc(ifl_handle* h, int32_t n_fields, const double* fields, int32_t n_scales,
                              const double* k, double* out, ifl_solve_stats* stats) {
  g_last_error.clear();
  if (!h) return fail(IFL_EINVAL, "handle is NULL");
  if (n_fields < 0) return fail(IFL_EINVAL, "n_fields < 0");
  ifl_status st = check_k(n_scales, k, false);
  if (st != IFL_OK) return st;
  if (n_fields == 0 || n_scales == 0) return IFL_OK;
  if (!fields || !out) return fail(IFL_EINVAL, "fields / out is NULL");
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::lock_guard<std::mutex> lk(h->mu);
  return device_filter_noalloc(h, n_fields, fields, n_scales, k, out, stats);
}

ifl_status ifl_spectrum(ifl_handle* h, const double* field, int32_t n_scales, const double* k, double* energy,
                        double* density, double* k_mid) {
  g_last_error.clear();
  if (!h || !field || !energy) return fail(IFL_EINVAL, "handle / field / energy is NULL");
  if (n_scales < 1) return fail(IFL_EINVAL, "n_scales must be >= 1");
  ifl_status st = check_k(n_scales, k, true);
  if (st != IFL_OK) return st;
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::vector<double> e(n_scales);
  {
    std::lock_guard<std::mutex> lk(h->mu);
    st = device_filter(h, 1, field, n_scales, k, nullptr, nullptr, e.data());
  }
  if (st != IFL_OK && st != IFL_ENOTCONV) return st;
  for (int32_t j = 0; j < n_scales; ++j) energy[j] = e[j];
  for (int32_t j = 0; j + 1 < n_scales; ++j) {
    if (density) density[j] = (e[j + 1] - e[j]) / (k[j + 1] - k[j]);
    if (k_mid) k_mid[j] = std::sqrt(k[j] * k[j + 1]);
  }
  return st;
}

ifl_status ifl_apply(ifl_handle* h, double k, const double* x, double* y) {
  g_last_error.clear();
  if (!h || !x || !y) return fail(IFL_EINVAL, "handle / x / y is NULL");
  ifl_status st = check_k(1, &k, false);
  if (st != IFL_OK) return st;
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::lock_guard<std::mutex> lk(h->mu);
  return device_apply(h, k, x, y);
}

ifl_status ifl_project_cells(ifl_handle* h, const double* cells, double* out) {
  g_last_error.clear();
  if (!h || !cells || !out) return fail(IFL_EINVAL, "handle / cells / out is NULL");
  if (h->op.placement != IFL_VERTEX_VECTOR)
    return fail(IFL_EINVAL, "ifl_project_cells needs an IFL_VERTEX_VECTOR handle");
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::lock_guard<std::mutex> lk(h->mu);
  return device_project_cells(h, cells, out);
}

int64_t ifl_operator_nnz(const ifl_handle* h) { return h ? (int64_t)h->op.col.size() : 0; }

int64_t ifl_first_order_nnz(const ifl_handle* h) {
  if (!h) return 0;
  return h->op.order >= 2 ? (int64_t)h->op.k1_col.size() : (int64_t)h->op.col.size();
}

ifl_status ifl_export_first_order(const ifl_handle* h, int64_t* row_ptr, int32_t* col, double* val) {
  if (!h) return fail(IFL_EINVAL, "handle is NULL");
  const HostOperator& op = h->op;
  const bool own = op.order >= 2;
  const auto& rp = own ? op.k1_row_ptr : op.row_ptr;
  const auto& cc = own ? op.k1_col : op.col;
  const auto& vv = own ? op.k1_val : op.val;
  if (row_ptr) std::memcpy(row_ptr, rp.data(), sizeof(int64_t) * rp.size());
  if (col) std::memcpy(col, cc.data(), sizeof(int32_t) * cc.size());
  if (val) std::memcpy(val, vv.data(), sizeof(double) * vv.size());
  return IFL_OK;
}

ifl_status ifl_export_operator(const ifl_handle* h, int64_t* row_ptr, int32_t* col, double* val, double* mass,
                               int64_t* entity) {
  if (!h) return fail(IFL_EINVAL, "handle is NULL");
  const HostOperator& op = h->op;
  if (row_ptr) std::memcpy(row_ptr, op.row_ptr.data(), sizeof(int64_t) * op.row_ptr.size());
  if (col) std::memcpy(col, op.col.data(), sizeof(int32_t) * op.col.size());
  if (val) std::memcpy(val, op.val.data(), sizeof(double) * op.val.size());
  if (mass) std::memcpy(mass, op.mass.data(), sizeof(double) * op.mass.size());
  if (entity) std::memcpy(entity, op.entity.data(), sizeof(int64_t) * op.entity.size());
  return IFL_OK;
}

static const char kMagic[8] = {'I', 'F', 'L', 'H', '0', '0', '0', '2'};

ifl_status ifl_save(const ifl_handle* h, const char* path) {
  if (!h || !path) return fail(IFL_EINVAL, "handle / path is NULL");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(IFL_EIO, std::string("cannot open for writing: ") + path);
  const HostOperator& op = h->op;
  const int64_t nnz = (int64_t)op.col.size();
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8;
  auto w = [&](const void* p, size_t sz) { ok = ok && (sz == 0 || std::fwrite(p, 1, sz, f) == sz); };
  w(&op.placement, 4);
  w(&op.order, 4);
  w(&op.n_components, 4);
  w(&h->opt.reorder, 4);
  w(&op.n, 8);
  w(&op.field_len, 8);
  w(&nnz, 8);
  w(&op.mesh_hash, 8);
  w(&h->opt.cell_A, 8);
  w(op.row_ptr.data(), sizeof(int64_t) * op.row_ptr.size());
  w(op.col.data(), sizeof(int32_t) * op.col.size());
  w(op.val.data(), sizeof(double) * op.val.size());
  w(op.mass.data(), sizeof(double) * op.mass.size());
  w(op.entity.data(), sizeof(int64_t) * op.entity.size());
  if (op.order >= 2) {
    const int64_t nnz1 = (int64_t)op.k1_col.size();
    w(&nnz1, 8);
    w(op.k1_row_ptr.data(), sizeof(int64_t) * op.k1_row_ptr.size());
    w(op.k1_col.data(), sizeof(int32_t) * op.k1_col.size());
    w(op.k1_val.data(), sizeof(double) * op.k1_val.size());
  }
  if (op.placement == IFL_VERTEX_VECTOR) {
    const int64_t pn = (int64_t)op.proj_tri.size();
    w(&op.n_cells, 8);
    w(&pn, 8);
    w(op.proj_ptr.data(), sizeof(int64_t) * op.proj_ptr.size());
    w(op.proj_tri.data(), sizeof(int32_t) * op.proj_tri.size());
    w(op.proj_w.data(), sizeof(double) * op.proj_w.size());
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(IFL_EIO, std::string("write failed: ") + path);
  return IFL_OK;
}

ifl_status ifl_load(const char* path, const ifl_options* opt, ifl_handle** out) {
  g_last_error.clear();
  if (!path || !out) return fail(IFL_EINVAL, "path / out is NULL");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(IFL_EIO, std::string("cannot open: ") + path);
  std::unique_ptr<ifl_handle> h(new ifl_handle());
  ifl_default_options(&h->opt);
  if (opt) h->opt = *opt;
  char magic[8];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0;
  auto r = [&](void* p, size_t sz) { ok = ok && (sz == 0 || std::fread(p, 1, sz, f) == sz); };
  HostOperator& op = h->op;
  int64_t nnz = 0;
  int32_t reorder = 1;
  double cellA = 0;
  r(&op.placement, 4);
  r(&op.order, 4);
  r(&op.n_components, 4);
  r(&reorder, 4);
  r(&op.n, 8);
  r(&op.field_len, 8);
  r(&nnz, 8);
  r(&op.mesh_hash, 8);
  r(&cellA, 8);
  if (ok && (op.n <= 0 || nnz <= 0 || op.n > (1ll << 31) || nnz > (1ll << 40) || op.field_len <= 0)) ok = false;
  if (ok) {
    op.row_ptr.resize(op.n + 1);
    op.col.resize(nnz);
    op.val.resize(nnz);
    op.mass.resize(op.n);
    op.entity.resize(op.n);
    r(op.row_ptr.data(), sizeof(int64_t) * op.row_ptr.size());
    r(op.col.data(), sizeof(int32_t) * op.col.size());
    r(op.val.data(), sizeof(double) * op.val.size());
    r(op.mass.data(), sizeof(double) * op.mass.size());
    r(op.entity.data(), sizeof(int64_t) * op.entity.size());
  }
  if (ok && op.order >= 2) {
    int64_t nnz1 = 0;
    r(&nnz1, 8);
    ok = ok && nnz1 > 0 && nnz1 <= nnz;
    if (ok) {
      op.k1_row_ptr.resize(op.n + 1);
      op.k1_col.resize(nnz1);
      op.k1_val.resize(nnz1);
      r(op.k1_row_ptr.data(), sizeof(int64_t) * op.k1_row_ptr.size());
      r(op.k1_col.data(), sizeof(int32_t) * op.k1_col.size());
      r(op.k1_val.data(), sizeof(double) * op.k1_val.size());
    }
    ok = ok && op.k1_row_ptr[0] == 0 && op.k1_row_ptr[op.n] == nnz1;
    for (int64_t i = 0; ok && i < op.n; ++i) ok = op.k1_row_ptr[i] <= op.k1_row_ptr[i + 1];
    for (int64_t e = 0; ok && e < nnz1; ++e) ok = op.k1_col[e] >= 0 && op.k1_col[e] < op.n;
  }
  if (ok && op.placement == IFL_VERTEX_VECTOR) {
    int64_t pn = 0;
    r(&op.n_cells, 8);
    r(&pn, 8);
    ok = ok && op.n % 2 == 0 && op.n_cells > 0 && op.n_cells < (1ll << 31) && pn > 0 && pn <= 3 * op.n_cells;
    if (ok) {
      op.proj_ptr.resize(op.n / 2 + 1);
      op.proj_tri.resize(pn);
      op.proj_w.resize(pn);
      r(op.proj_ptr.data(), sizeof(int64_t) * op.proj_ptr.size());
      r(op.proj_tri.data(), sizeof(int32_t) * op.proj_tri.size());
      r(op.proj_w.data(), sizeof(double) * op.proj_w.size());
    }
    ok = ok && op.proj_ptr[0] == 0 && op.proj_ptr[op.n / 2] == pn;
    for (int64_t i = 0; ok && i < op.n / 2; ++i) ok = op.proj_ptr[i] <= op.proj_ptr[i + 1];
    for (int64_t e = 0; ok && e < pn; ++e) ok = op.proj_tri[e] >= 0 && op.proj_tri[e] < op.n_cells;
  }
  std::fclose(f);
  if (ok) {
    ok = op.row_ptr[0] == 0 && op.row_ptr[op.n] == nnz;
    for (int64_t i = 0; ok && i < op.n; ++i) ok = op.row_ptr[i] <= op.row_ptr[i + 1];
    for (int64_t e = 0; ok && e < nnz; ++e) ok = op.col[e] >= 0 && op.col[e] < op.n;
    for (int64_t i = 0; ok && i < op.n; ++i) ok = op.entity[i] >= 0 && op.entity[i] < op.field_len;
    if (op.placement == IFL_VERTEX_VECTOR)  // the projection writes (east, north) pairs
      for (int64_t i = 0; ok && i + 1 < op.n; i += 2)
        ok = op.entity[i] % 2 == 0 && op.entity[i + 1] == op.entity[i] + 1;
  }
  if (!ok) return fail(IFL_EIO, std::string("bad or truncated handle file: ") + path);
  h->opt.reorder = reorder;
  h->opt.cell_A = cellA;
  ifl_status st = check_options(h->opt);
  if (st != IFL_OK) return st;
  if (h->opt.device >= 0) {
    st = device_create(h.get());
    if (st != IFL_OK) {
      device_destroy(h.get());
      return st;
    }
  }
  *out = h.release();
  return IFL_OK;
}

ifl_status ifl_profile_read(ifl_handle* h, int64_t* launches, double* total_ms, double* bytes_per_launch,
                            int32_t reset) {
  if (!h) return fail(IFL_EINVAL, "handle is NULL");
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::lock_guard<std::mutex> lk(h->mu);
  return device_profile_read(h, launches, total_ms, bytes_per_launch, reset);
}

ifl_status ifl_profile_kernel(ifl_handle* h, char* buf, int32_t len) {
  if (!h) return fail(IFL_EINVAL, "handle is NULL");
  if (!buf || len < 1) return fail(IFL_EINVAL, "buffer is NULL or empty");
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::lock_guard<std::mutex> lk(h->mu);
  const std::string name = device_profile_kernel(h);
  const size_t n = std::min(name.size(), (size_t)len - 1);
  std::memcpy(buf, name.data(), n);
  buf[n] = '\0';
  return IFL_OK;
}

ifl_status ifl_stream_probe(int32_t device, int64_t bytes, int32_t reps, double* best_gbs, double* median_gbs) {
  if (!best_gbs || !median_gbs) return fail(IFL_EINVAL, "output pointer is NULL");
  if (bytes < (16ll << 20)) return fail(IFL_EINVAL, "the probe copies at least 16 MiB");
  if (reps < 1 || reps > 1000) return fail(IFL_EINVAL, "reps must be in 1..1000");
  return device_stream_probe(device, bytes, reps, best_gbs, median_gbs);
}

ifl_status ifl_autotune(ifl_handle* h, ifl_tune* out) {
  if (!h) return fail(IFL_EINVAL, "handle is NULL");
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::lock_guard<std::mutex> lk(h->mu);
  return device_autotune(h, out);
}

}  // extern "C"
