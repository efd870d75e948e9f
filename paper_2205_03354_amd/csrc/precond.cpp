// Fast-Poisson preconditioner for the biharmonic boundary-value problem.
//
// The BVP operator (the Laplacian composed with itself, with the unknowns'
// outer ring held at zero) equals L_D^2 plus a non-negative diagonal on the
// layer next to the boundary, L_D being the 5/7-point Dirichlet Laplacian on
// the unknowns (the composition of Sec. 3.3 restricted to the interior).
// L_D is diagonalised by the orthonormal sine transform S (S = S^T = S^-1)
// along every axis, so M^-1 = L_D^-2 = S (Lambda^-2 o (S r)) with Lambda the
// sums of the 1D eigenvalues -(4/h^2) sin^2(pi k / (2(n+1))). Each axis
// transform is a dense product with the n x n matrix S (a GEMM on the
// interior, batched over planes or rows), done by rocBLAS; the scaling is a
// library kernel.
#include <rocblas/rocblas.h>

#include <map>

#include "task.hpp"

namespace sc {

namespace {

rocblas_handle blas_handle() {
  thread_local std::map<int, rocblas_handle> handles;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  auto it = handles.find(dev);
  if (it != handles.end()) return it->second;
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
  handles[dev] = h;
  return h;
}

// C (m x n, ldc) = A (m x k, lda) * B (k x n, ldb), column-major, batched
// with strides (a zero stride reuses the matrix).
sc_status gemm(rocblas_handle hb, int dtype, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, int64_t sa,
               const void* B, int64_t ldb, int64_t sb, void* C, int64_t ldc, int64_t sc_, int64_t batch) {
  rocblas_status e;
  if (dtype == SC_F64) {
    const double one = 1.0, zero = 0.0;
    e = rocblas_dgemm_strided_batched(hb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)m,
                                      (rocblas_int)n, (rocblas_int)k, &one, (const double*)A, (rocblas_int)lda, sa,
                                      (const double*)B, (rocblas_int)ldb, sb, &zero, (double*)C, (rocblas_int)ldc,
                                      sc_, (rocblas_int)batch);
  } else {
    const float one = 1.0f, zero = 0.0f;
    e = rocblas_sgemm_strided_batched(hb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)m,
                                      (rocblas_int)n, (rocblas_int)k, &one, (const float*)A, (rocblas_int)lda, sa,
                                      (const float*)B, (rocblas_int)ldb, sb, &zero, (float*)C, (rocblas_int)ldc, sc_,
                                      (rocblas_int)batch);
  }
  if (e != rocblas_status_success) {
    set_error("rocBLAS GEMM failed: %s", rocblas_status_to_string(e));
    return SC_EDEVICE;
  }
  return SC_OK;
}

}  // namespace

size_t fastpoisson_bytes(int dim, const int64_t* n, int dtype) {
  const size_t es = dtype == SC_F64 ? 8 : 4;
  size_t b = 0;
  for (int a = 0; a < dim; ++a) {
    bool dup = false;
    for (int c = 0; c < a; ++c) dup = dup || n[c] == n[a];
    if (!dup) b += (((size_t)(n[a] * n[a]) * es + 4095) & ~(size_t)4095);
    b += (((size_t)n[a] * 8 + 4095) & ~(size_t)4095);
  }
  return b;
}

FastPoisson::~FastPoisson() {
  for (void* p : allocs_) pool_free(p);
}

sc_status FastPoisson::init(int dim, const int64_t* n, double h, int dtype, hipStream_t st) {
  dim_ = dim;
  dtype_ = dtype;
  for (int a = 0; a < 3; ++a) n_[a] = a < dim ? n[a] : 1;
  const size_t es = dtype == SC_F64 ? 8 : 4;
  for (int a = 0; a < dim; ++a) {
    int same = -1;
    for (int c = 0; c < a; ++c)
      if (n_[c] == n_[a]) same = c;
    const int64_t m = n_[a];
    void* l = pool_alloc((size_t)m * 8);
    void* d = same >= 0 ? S_[same] : pool_alloc((size_t)(m * m) * es);
    if (!l || !d) {
      if (l) pool_free(l);
      set_error("preconditioner allocation failed");
      return SC_ENOMEM;
    }
    allocs_.push_back(l);
    if (same < 0) allocs_.push_back(d);
    S_[a] = d;
    lam_[a] = static_cast<double*>(l);
    // the transform and the 1D eigenvalues are generated on the device
    SC_HIP_CHECK(launch_pc_init(dtype, same >= 0 ? nullptr : d, lam_[a], m, h, st));
  }
  if (!blas_handle()) {
    set_error("rocBLAS handle creation failed");
    return SC_EDEVICE;
  }
  return SC_OK;
}

// z = S (Lambda^-2 o (S r)) on the interior; tmp is scratch of r's layout.
sc_status FastPoisson::apply(const void* r, void* z, void* tmp, const Layout& lay, const DevScalars* s,
                             hipStream_t st) const {
  rocblas_handle hb = blas_handle();
  if (!hb || rocblas_set_stream(hb, st) != rocblas_status_success) {
    set_error("rocBLAS stream binding failed");
    return SC_EDEVICE;
  }
  sc_status e;
  const int64_t n0 = n_[0], n1 = n_[1], n2 = n_[2];
  const int64_t p = lay.pitch, zp = lay.zpitch;
  // one sine transform along every axis, in -> out (in and out distinct)
  auto transform = [&](const void* in, void* out, void* mid) -> sc_status {
    sc_status r2;
    if (dim_ == 2) {
      if ((r2 = gemm(hb, dtype_, n0, n1, n0, S_[0], n0, 0, in, p, 0, mid, p, 0, 1)) != SC_OK) return r2;
      return gemm(hb, dtype_, n0, n1, n1, mid, p, 0, S_[1], n1, 0, out, p, 0, 1);
    }
    // per plane: x (left) then y (right); then z across planes, per row
    if ((r2 = gemm(hb, dtype_, n0, n1, n0, S_[0], n0, 0, in, p, zp, mid, p, zp, n2)) != SC_OK) return r2;
    if ((r2 = gemm(hb, dtype_, n0, n1, n1, mid, p, zp, S_[1], n1, 0, out, p, zp, n2)) != SC_OK) return r2;
    if ((r2 = gemm(hb, dtype_, n0, n2, n2, out, zp, p, S_[2], n2, 0, mid, zp, p, n1)) != SC_OK) return r2;
    return SC_OK;
  };
  if (dim_ == 2) {
    if ((e = transform(r, z, tmp)) != SC_OK) return e;  // S r in z (via tmp)
    SC_HIP_CHECK(launch_pc_scale(dtype_, z, lay, n_, lam_[0], lam_[1], nullptr, s, st));
    return transform(z, z, tmp);  // S (...) back into z
  }
  if ((e = transform(r, z, tmp)) != SC_OK) return e;  // S r in tmp (3 passes)
  SC_HIP_CHECK(launch_pc_scale(dtype_, tmp, lay, n_, lam_[0], lam_[1], lam_[2], s, st));
  if ((e = transform(tmp, tmp, z)) != SC_OK) return e;  // result in z
  return SC_OK;
}

}  // namespace sc
