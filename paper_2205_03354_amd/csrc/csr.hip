// Assembled form of a composed stencil: a CSR matrix over the grid's
// unknowns, multiplied by rocSPARSE. The paper builds its operators this
// way (Sec. 4.5-4.6, Table 3 counting their non-zeros); here it is the
// baseline that the matrix-free sweeps are measured against.
//
// Assembly runs on the device: one thread per row gathers the row's
// (column, weight) pairs, sorts them by column (insertion sort: rows away
// from a wrapped edge arrive sorted, because the taps are ordered by their
// linear offset), sums the pairs of taps that alias to one column on small
// periodic grids, and writes them. A first pass counts the entries of every
// row and a device scan turns the counts into row pointers.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <rocsparse/rocsparse.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "internal.hpp"

struct sc_csr {
  int dim = 0;
  int64_t n[3] = {1, 1, 1};
  int64_t rows = 0;
  int64_t nnz = 0;
  int dtype = SC_F64;
  int alg = SC_CSR_ROWSPLIT;
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  void* val = nullptr;
  rocsparse_spmat_descr mat = nullptr;
  void* work = nullptr;
  size_t work_bytes = 0;
  bool prepared = false;
  int device = 0;
};

namespace sc {

namespace {

constexpr int kMaxCsrTaps = 128;

struct CsrTaps {
  int n;                        // taps in ascending linear offset
  int32_t off[kMaxCsrTaps][3];
  double w[kMaxCsrTaps];
};

// The row's entries in ascending column order, aliased taps summed.
// Returns the entry count; cols / vals receive the entries when non-null.
__device__ inline int row_entries(const CsrTaps& t, int64_t row, int64_t n0, int64_t n1, int64_t n2,
                                  bool periodic, int32_t* cols, double* vals) {
  const int64_t x = row % n0, y = (row / n0) % n1, z = row / (n0 * n1);
  int32_t c[kMaxCsrTaps];
  double v[kMaxCsrTaps];
  int m = 0;
  for (int k = 0; k < t.n; ++k) {
    int64_t xi = x + t.off[k][0], yi = y + t.off[k][1], zi = z + t.off[k][2];
    if (periodic) {
      xi = ((xi % n0) + n0) % n0;
      yi = ((yi % n1) + n1) % n1;
      zi = ((zi % n2) + n2) % n2;
    } else if (xi < 0 || xi >= n0 || yi < 0 || yi >= n1 || zi < 0 || zi >= n2) {
      continue;
    }
    const int32_t cj = (int32_t)(xi + n0 * (yi + n1 * zi));
    const double wk = t.w[k];
    int p = m++;
    while (p > 0 && c[p - 1] > cj) {
      c[p] = c[p - 1];
      v[p] = v[p - 1];
      --p;
    }
    c[p] = cj;
    v[p] = wk;
  }
  int u = 0;
  for (int k = 0; k < m; ++k) {
    if (u > 0 && c[u - 1] == c[k]) {
      v[u - 1] += v[k];
    } else {
      c[u] = c[k];
      v[u] = v[k];
      ++u;
    }
  }
  if (cols)
    for (int k = 0; k < u; ++k) {
      cols[k] = c[k];
      vals[k] = v[k];
    }
  return u;
}

__global__ void csr_count_kernel(CsrTaps t, int64_t n0, int64_t n1, int64_t n2, int periodic, int64_t rows,
                                 int64_t* counts) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  counts[row] = row_entries(t, row, n0, n1, n2, periodic != 0, nullptr, nullptr);
}

template <typename T>
__global__ void csr_fill_kernel(CsrTaps t, int64_t n0, int64_t n1, int64_t n2, int periodic, int64_t rows,
                                const int64_t* row_ptr, int32_t* col, T* val) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  int32_t c[kMaxCsrTaps];
  double v[kMaxCsrTaps];
  const int m = row_entries(t, row, n0, n1, n2, periodic != 0, c, v);
  const int64_t base = row_ptr[row];
  for (int k = 0; k < m; ++k) {
    col[base + k] = c[k];
    val[base + k] = (T)v[k];
  }
}

rocsparse_handle sparse_handle() {
  thread_local std::map<int, rocsparse_handle> handles;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  auto it = handles.find(dev);
  if (it != handles.end()) return it->second;
  rocsparse_handle h = nullptr;
  if (rocsparse_create_handle(&h) != rocsparse_status_success) return nullptr;
  handles[dev] = h;
  return h;
}

sc_status sparse_error(const char* what, rocsparse_status e) {
  set_error("rocSPARSE %s failed (status %d)", what, (int)e);
  return SC_EDEVICE;
}

void release(sc_csr* m) {
  if (!m) return;
  if (m->mat) rocsparse_destroy_spmat_descr(m->mat);
  if (m->work) pool_free(m->work);
  if (m->val) pool_free(m->val);
  if (m->col) pool_free(m->col);
  if (m->row_ptr) pool_free(m->row_ptr);
  delete m;
}

rocsparse_datatype sparse_type(int dtype) {
  return dtype == SC_F64 ? rocsparse_datatype_f64_r : rocsparse_datatype_f32_r;
}

rocsparse_spmv_alg sparse_alg(int alg) {
  return alg == SC_CSR_ADAPTIVE ? rocsparse_spmv_alg_csr_adaptive : rocsparse_spmv_alg_csr_rowsplit;
}

sc_status check_dense(const sc_csr* m, const sc_grid* g, const char* what) {
  sc_status e = check_grid(g, what);
  if (e != SC_OK) return e;
  bool ok = g->dim == m->dim && g->dtype == m->dtype && g->halo == 0 && g->pitch[0] == m->n[0];
  for (int a = 0; a < 3; ++a) ok = ok && g->n[a] == m->n[a];
  if (m->dim == 3) ok = ok && g->pitch[1] == m->n[0] * m->n[1];
  if (!ok) {
    set_error("%s: must match the matrix's grid and dtype, with halo 0 and contiguous rows and planes", what);
    return SC_EINVAL;
  }
  return SC_OK;
}

}  // namespace

sc_status csr_assemble(const sc_stencil* s, double h, int32_t dim, const int64_t* n, int32_t bc, int32_t dtype,
                       int32_t alg, hipStream_t st, sc_csr** out) {
  if (!out || !s || !n) {
    set_error("csr_assemble: NULL argument");
    return SC_EINVAL;
  }
  *out = nullptr;
  if ((dim != 2 && dim != 3) || s->dim != dim) {
    set_error("csr_assemble: dim must be 2 or 3 and match the stencil");
    return SC_EINVAL;
  }
  if (bc != SC_CSR_PERIODIC && bc != SC_CSR_ZERO_RING) {
    set_error("csr_assemble: unknown boundary mode %d", bc);
    return SC_EINVAL;
  }
  if (dtype != SC_F64 && dtype != SC_F32) {
    set_error("csr_assemble: unknown dtype %d", dtype);
    return SC_EINVAL;
  }
  if (alg != SC_CSR_ROWSPLIT && alg != SC_CSR_ADAPTIVE) {
    set_error("csr_assemble: unknown SpMV algorithm %d", alg);
    return SC_EINVAL;
  }
  if (!(h > 0.0) || !std::isfinite(h)) {
    set_error("csr_assemble: invalid grid spacing");
    return SC_EINVAL;
  }
  if (dim == 2 && n[2] != 1) {
    set_error("csr_assemble: n[2] must be 1 in 2D");
    return SC_EINVAL;
  }
  int64_t rows = 1;
  for (int a = 0; a < dim; ++a) {
    if (n[a] < 1 || n[a] >= ((int64_t)1 << 31) || rows * n[a] >= ((int64_t)1 << 31)) {
      set_error("csr_assemble: extent %lld along axis %d is empty or makes 2^31 rows or more", (long long)n[a], a);
      return SC_EINVAL;
    }
    rows *= n[a];
  }
  const int ntaps = (int)s->num.size();
  if (ntaps < 1 || ntaps > kMaxCsrTaps) {
    set_error("csr_assemble: %d taps (1..%d supported)", ntaps, kMaxCsrTaps);
    return SC_EUNSUPPORTED;
  }
  const int64_t n0 = n[0], n1 = n[1], n2 = dim == 3 ? n[2] : 1;

  // weights num / (den h^p), rounded once to double as for the sweeps
  long double hp = 1.0L;
  for (int i = 0; i < std::abs(s->hpow); ++i) hp *= (long double)h;
  if (s->hpow < 0) hp = 1.0L / hp;
  std::vector<int> order(ntaps);
  std::vector<int64_t> lin(ntaps);
  for (int k = 0; k < ntaps; ++k) {
    order[k] = k;
    lin[k] = s->off[k][0] + n0 * (s->off[k][1] + n1 * (int64_t)s->off[k][2]);
  }
  std::sort(order.begin(), order.end(), [&](int a, int b) { return lin[a] < lin[b]; });
  CsrTaps taps{};
  taps.n = ntaps;
  for (int i = 0; i < ntaps; ++i) {
    const int k = order[i];
    for (int a = 0; a < 3; ++a) taps.off[i][a] = s->off[k][a];
    taps.w[i] = (double)((long double)s->num[k] / ((long double)s->den * hp));
  }

  sc_csr* m = new sc_csr();
  m->dim = dim;
  m->n[0] = n0;
  m->n[1] = n1;
  m->n[2] = n2;
  m->rows = rows;
  m->dtype = dtype;
  m->alg = alg;
  SC_HIP_CHECK(hipGetDevice(&m->device));
  const int periodic = bc == SC_CSR_PERIODIC;
  const unsigned threads = 256;
  const unsigned blocks = (unsigned)((rows + threads - 1) / threads);

  m->row_ptr = static_cast<int64_t*>(pool_alloc((size_t)(rows + 1) * sizeof(int64_t)));
  int64_t* counts = static_cast<int64_t*>(pool_alloc((size_t)rows * sizeof(int64_t)));
  if (!m->row_ptr || !counts) {
    if (counts) pool_free(counts);
    release(m);
    set_error("csr_assemble: allocation of row pointers failed");
    return SC_ENOMEM;
  }
  auto fail = [&](sc_status e) {
    if (counts) pool_free(counts);
    release(m);
    return e;
  };
  hipLaunchKernelGGL(csr_count_kernel, dim3(blocks), dim3(threads), 0, st, taps, n0, n1, n2, periodic, rows,
                     counts);
  if (hipGetLastError() != hipSuccess) {
    set_error("csr_assemble: count kernel launch failed");
    return fail(SC_EDEVICE);
  }
  // row_ptr[0] = 0, row_ptr[i + 1] = counts[0] + ... + counts[i]
  if (hipMemsetAsync(m->row_ptr, 0, sizeof(int64_t), st) != hipSuccess) {
    set_error("csr_assemble: row pointer clear failed");
    return fail(SC_EDEVICE);
  }
  size_t scan_bytes = 0;
  if (hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, counts, m->row_ptr + 1, (int)rows, st) !=
      hipSuccess) {
    set_error("csr_assemble: scan size query failed");
    return fail(SC_EDEVICE);
  }
  void* scan_tmp = pool_alloc(std::max<size_t>(scan_bytes, 256));
  if (!scan_tmp) {
    set_error("csr_assemble: scan workspace allocation failed");
    return fail(SC_ENOMEM);
  }
  hipError_t he = hipcub::DeviceScan::InclusiveSum(scan_tmp, scan_bytes, counts, m->row_ptr + 1, (int)rows, st);
  int64_t nnz = 0;
  if (he == hipSuccess) he = hipMemcpyAsync(&nnz, m->row_ptr + rows, sizeof(int64_t), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  pool_free(scan_tmp);
  if (he != hipSuccess) {
    set_error("csr_assemble: row pointer scan failed: %s", hipGetErrorString(he));
    return fail(SC_EDEVICE);
  }
  pool_free(counts);
  counts = nullptr;
  m->nnz = nnz;
  const size_t es = esize(dtype);
  m->col = static_cast<int32_t*>(pool_alloc((size_t)nnz * sizeof(int32_t)));
  m->val = pool_alloc((size_t)nnz * es);
  if (!m->col || !m->val) {
    set_error("csr_assemble: allocation of %lld entries failed", (long long)nnz);
    return fail(SC_ENOMEM);
  }
  if (dtype == SC_F64)
    hipLaunchKernelGGL(csr_fill_kernel<double>, dim3(blocks), dim3(threads), 0, st, taps, n0, n1, n2, periodic,
                       rows, m->row_ptr, m->col, static_cast<double*>(m->val));
  else
    hipLaunchKernelGGL(csr_fill_kernel<float>, dim3(blocks), dim3(threads), 0, st, taps, n0, n1, n2, periodic,
                       rows, m->row_ptr, m->col, static_cast<float*>(m->val));
  he = hipGetLastError();
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) {
    set_error("csr_assemble: fill failed: %s", hipGetErrorString(he));
    return fail(SC_EDEVICE);
  }
  rocsparse_status se = rocsparse_create_csr_descr(&m->mat, rows, rows, nnz, m->row_ptr, m->col, m->val,
                                                   rocsparse_indextype_i64, rocsparse_indextype_i32,
                                                   rocsparse_index_base_zero, sparse_type(dtype));
  if (se != rocsparse_status_success) {
    m->mat = nullptr;
    return fail(sparse_error("matrix descriptor", se));
  }
  *out = m;
  return SC_OK;
}

sc_status csr_info(const sc_csr* m, int64_t* rows, int64_t* nnz, uint64_t* bytes) {
  if (!m) {
    set_error("csr_info: NULL matrix");
    return SC_EINVAL;
  }
  if (rows) *rows = m->rows;
  if (nnz) *nnz = m->nnz;
  if (bytes) *bytes = (uint64_t)(m->rows + 1) * 8 + (uint64_t)m->nnz * (4 + esize(m->dtype));
  return SC_OK;
}

sc_status csr_spmv(sc_csr* m, const sc_grid* x, sc_grid* y, hipStream_t st) {
  if (!m) {
    set_error("csr_spmv: NULL matrix");
    return SC_EINVAL;
  }
  sc_status e;
  if ((e = check_dense(m, x, "csr_spmv x")) != SC_OK) return e;
  if ((e = check_dense(m, y, "csr_spmv y")) != SC_OK) return e;
  const size_t bytes = (size_t)m->rows * esize(m->dtype);
  const char* xa = static_cast<const char*>(x->data);
  const char* ya = static_cast<const char*>(y->data);
  if (xa < ya + bytes && ya < xa + bytes) {
    set_error("csr_spmv: y must not overlap x");
    return SC_EINVAL;
  }
  int dev = 0;
  SC_HIP_CHECK(hipGetDevice(&dev));
  if (dev != m->device) {
    set_error("csr_spmv: the matrix lives on device %d, the current device is %d", m->device, dev);
    return SC_EINVAL;
  }
  rocsparse_handle hs = sparse_handle();
  if (!hs) {
    set_error("csr_spmv: rocSPARSE handle creation failed");
    return SC_EDEVICE;
  }
  rocsparse_status se = rocsparse_set_stream(hs, st);
  if (se != rocsparse_status_success) return sparse_error("stream binding", se);
  rocsparse_dnvec_descr dx = nullptr, dy = nullptr;
  const rocsparse_datatype ty = sparse_type(m->dtype);
  se = rocsparse_create_dnvec_descr(&dx, m->rows, x->data, ty);
  if (se == rocsparse_status_success) se = rocsparse_create_dnvec_descr(&dy, m->rows, y->data, ty);
  if (se != rocsparse_status_success) {
    if (dx) rocsparse_destroy_dnvec_descr(dx);
    return sparse_error("vector descriptor", se);
  }
  const double one64 = 1.0, zero64 = 0.0;
  const float one32 = 1.0f, zero32 = 0.0f;
  const void* alpha = m->dtype == SC_F64 ? (const void*)&one64 : (const void*)&one32;
  const void* beta = m->dtype == SC_F64 ? (const void*)&zero64 : (const void*)&zero32;
  const rocsparse_spmv_alg alg = sparse_alg(m->alg);
  sc_status out = SC_OK;
  if (!m->prepared) {
    size_t wb = 0;
    se = rocsparse_spmv(hs, rocsparse_operation_none, alpha, m->mat, dx, beta, dy, ty, alg,
                        rocsparse_spmv_stage_buffer_size, &wb, nullptr);
    if (se != rocsparse_status_success) {
      out = sparse_error("SpMV buffer size", se);
    } else {
      m->work_bytes = std::max<size_t>(wb, 256);
      m->work = pool_alloc(m->work_bytes);
      if (!m->work) {
        set_error("csr_spmv: SpMV workspace allocation failed");
        out = SC_ENOMEM;
      } else {
        se = rocsparse_spmv(hs, rocsparse_operation_none, alpha, m->mat, dx, beta, dy, ty, alg,
                            rocsparse_spmv_stage_preprocess, &m->work_bytes, m->work);
        if (se != rocsparse_status_success)
          out = sparse_error("SpMV preprocess", se);
        else
          m->prepared = true;
      }
    }
  }
  if (out == SC_OK) {
    se = rocsparse_spmv(hs, rocsparse_operation_none, alpha, m->mat, dx, beta, dy, ty, alg,
                        rocsparse_spmv_stage_compute, &m->work_bytes, m->work);
    if (se != rocsparse_status_success) out = sparse_error("SpMV", se);
  }
  rocsparse_destroy_dnvec_descr(dx);
  rocsparse_destroy_dnvec_descr(dy);
  return out;
}

sc_status csr_export(const sc_csr* m, int64_t* row_ptr, int32_t* col, void* val) {
  if (!m) {
    set_error("csr_export: NULL matrix");
    return SC_EINVAL;
  }
  if (row_ptr) SC_HIP_CHECK(hipMemcpy(row_ptr, m->row_ptr, (size_t)(m->rows + 1) * 8, hipMemcpyDeviceToHost));
  if (col) SC_HIP_CHECK(hipMemcpy(col, m->col, (size_t)m->nnz * 4, hipMemcpyDeviceToHost));
  if (val) SC_HIP_CHECK(hipMemcpy(val, m->val, (size_t)m->nnz * esize(m->dtype), hipMemcpyDeviceToHost));
  return SC_OK;
}

void csr_free(sc_csr* m) {
  if (!m) return;
  int dev = 0;
  const bool swap = hipGetDevice(&dev) == hipSuccess && dev != m->device;
  if (swap) (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  release(m);
  if (swap) (void)hipSetDevice(dev);
}

}  // namespace sc
