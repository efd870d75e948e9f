// Fast-Poisson preconditioner for the biharmonic boundary-value problem.
//
// The BVP operator (the Laplacian composed with itself, with the unknowns'
// outer ring held at zero) equals L_D^2 plus a non-negative diagonal on the
// layer next to the boundary, L_D being the 5/7-point Dirichlet Laplacian on
// the unknowns (the composition of Sec. 3.3 restricted to the interior).
// L_D is diagonalised by the orthonormal sine transform S (S = S^T = S^-1)
// along every axis, so M^-1 = L_D^-2 = S (Lambda^-2 o (S r)) with Lambda the
// sums of the 1D eigenvalues -(4/h^2) sin^2(pi k / (2(n+1))). Each axis
// transform is either a dense product with the n x n matrix S (a GEMM on the
// interior, batched over planes or rows, by rocBLAS: 3D grids and small or
// FFT-unfriendly 2D ones) or, on 2D grids of side >= kFftMinSide whose
// n + 1 is a power of two, a real FFT (rocFFT) of each row's odd
// extension, O(n log n) per row and bandwidth-bound, written transposed so
// that the second axis is again a row transform; the extension, extraction
// and scaling are library kernels.
#include <rocblas/rocblas.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <array>
#include <cstdlib>
#include <map>
#include <mutex>

#include "task.hpp"

namespace sc {

namespace {

// Odd extension of each row: e = (0, v_1 .. v_n, 0, -v_n .. -v_1), length
// N = 2 (n + 1); its real FFT at k = 1 .. n is -2i sum_j v_j sin(pi j k / (n + 1)).
template <typename T>
__global__ void __launch_bounds__(256) dst_extend_kernel(const T* __restrict__ v, int64_t pv, int64_t n, int64_t m,
                                                         T* __restrict__ e) {
  const int64_t N = 2 * (n + 1);
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m * N; i += stride) {
    const int64_t r = i / N, j = i - r * N;
    T x = T(0);
    if (j >= 1 && j <= n)
      x = v[r * pv + j - 1];
    else if (j > n + 1)
      x = -v[r * pv + (N - j) - 1];
    e[i] = x;
  }
}

// out[k - 1][r] = -c Im(F[r][k]) / 2 for k = 1 .. n (transposed through a
// 32 x 32 LDS tile so that reads and writes are both coalesced).
template <typename T>
__global__ void __launch_bounds__(256) dst_extract_kernel(const T* __restrict__ F, int64_t n, int64_t m, T* out,
                                                          int64_t pout, T c) {
  __shared__ T tile[32][33];
  const int64_t H = n + 2;  // complex values per row of the half spectrum
  const int64_t k0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t r = r0 + yy, k = k0 + tx + 1;
    tile[yy][tx] = (r < m && k <= n) ? F[2 * (r * H + k) + 1] : T(0);
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t k = k0 + yy + 1, r = r0 + tx;
    if (k <= n && r < m) out[(k - 1) * pout + r] = -T(0.5) * c * tile[tx][yy];
  }
}

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

// C (m x n, ldc) = op(A) (m x k) * op(B) (k x n), column-major (lda, ldb
// describe A and B as stored), batched with strides (a zero stride reuses
// the matrix); ta / tb transpose A / B.
sc_status gemm(rocblas_handle hb, int dtype, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, int64_t sa,
               const void* B, int64_t ldb, int64_t sb, void* C, int64_t ldc, int64_t sc_, int64_t batch,
               bool ta = false, bool tb = false) {
  rocblas_status e;
  const rocblas_operation oa = ta ? rocblas_operation_transpose : rocblas_operation_none;
  const rocblas_operation ob = tb ? rocblas_operation_transpose : rocblas_operation_none;
  if (dtype == SC_F64) {
    const double one = 1.0, zero = 0.0;
    e = rocblas_dgemm_strided_batched(hb, oa, ob, (rocblas_int)m,
                                      (rocblas_int)n, (rocblas_int)k, &one, (const double*)A, (rocblas_int)lda, sa,
                                      (const double*)B, (rocblas_int)ldb, sb, &zero, (double*)C, (rocblas_int)ldc,
                                      sc_, (rocblas_int)batch);
  } else {
    const float one = 1.0f, zero = 0.0f;
    e = rocblas_sgemm_strided_batched(hb, oa, ob, (rocblas_int)m,
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

// The FFT path is taken when both odd-extension lengths 2 (n + 1) are
// powers of two: those have precompiled FFT kernels, so a plan builds in
// milliseconds; other lengths may need kernels compiled at run time (a cost
// a request stream of arbitrary sizes cannot pay), and keep the GEMM
// transforms.
bool fft_sides(int dim, const int64_t* n) {
  if (dim != 2) return false;
  for (int a = 0; a < 2; ++a) {
    const int64_t v = n[a] + 1;
    if (n[a] < kFftMinSide || (v & (v - 1)) != 0) return false;
  }
  return true;
}

// The split GEMM transforms halve the flops but add a butterfly pass and a
// second, half-size GEMM per axis: they pay on large 2D sides (n ~ 2000:
// about 0.6 ms of GEMM saved per apply for 0.07 ms of butterflies), not on
// small grids, where launches dominate (65^2: 1.2 -> 2.0 ms per PCG solve),
// nor in 3D, where the butterflies move as many bytes as the halved GEMMs
// save (255^3: 43 -> 47 ms).
bool split_sides(int dim, const int64_t* n) {
  if (const char* e = std::getenv("SCOMP_PCSPLIT"))  // A/B switch: 0 keeps the full products
    if (e[0] == '0') return false;
  return dim == 2 && !fft_sides(dim, n) && std::min(n[0], n[1]) >= kSplitMinSide;
}

}  // namespace

size_t fastpoisson_bytes(int dim, const int64_t* n, int dtype) {
  const size_t es = dtype == SC_F64 ? 8 : 4;
  size_t b = 0;
  if (fft_sides(dim, n)) {
    // extension, half spectrum and transposed field (the FFT work buffers are
    // small next to these)
    const size_t m = (size_t)std::max(n[0], n[1]);
    const size_t nn = (size_t)std::max(n[0], n[1]);
    b += m * (2 * nn + 2) * es + m * (nn + 2) * 2 * es + (size_t)(n[0] * n[1]) * es + 4 * 1048576;
    for (int a = 0; a < dim; ++a) b += (((size_t)n[a] * 8 + 4095) & ~(size_t)4095);
    return b;
  }
  for (int a = 0; a < dim; ++a) {
    bool dup = false;
    for (int c = 0; c < a; ++c) dup = dup || n[c] == n[a];
    const size_t hp = (size_t)(n[a] + 1) / 2, hm = (size_t)n[a] / 2;  // the split transform's halves
    const size_t mat = split_sides(dim, n) ? hp * hp + hm * hm : (size_t)(n[a] * n[a]);
    if (!dup) b += ((mat * es + 4095) & ~(size_t)4095);
    b += (((size_t)n[a] * 8 + 4095) & ~(size_t)4095);
  }
  return b;
}

FastPoisson::~FastPoisson() {
  for (Dst* d : {&dx_, &dy_})
    if (d->info) rocfft_execution_info_destroy(static_cast<rocfft_execution_info>(d->info));
  for (void* p : allocs_) pool_free(p);
}

sc_status FastPoisson::dst_init(Dst* d, int64_t n, int64_t m, hipStream_t st) {
  // Plans are built once per (device, length, batch, precision) and kept for
  // the life of the process: building one costs milliseconds, more than a
  // whole preconditioned solve on a mid-size grid. Each preconditioner keeps
  // its own execution info (stream) and work buffer.
  static std::mutex mu;
  static std::map<std::array<int64_t, 4>, rocfft_plan> plans;
  static bool setup_done = false;
  int dev = 0;
  SC_HIP_CHECK(hipGetDevice(&dev));
  d->n = n;
  d->m = m;
  rocfft_plan plan = nullptr;
  {
    std::lock_guard<std::mutex> g(mu);
    if (!setup_done) {
      if (rocfft_setup() != rocfft_status_success) {
        set_error("rocFFT setup failed");
        return SC_EDEVICE;
      }
      setup_done = true;
    }
    const std::array<int64_t, 4> key{dev, n, m, dtype_};
    auto it = plans.find(key);
    if (it != plans.end()) {
      plan = it->second;
    } else {
      const size_t len = (size_t)(2 * (n + 1));
      const rocfft_status e =
          rocfft_plan_create(&plan, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                             dtype_ == SC_F64 ? rocfft_precision_double : rocfft_precision_single, 1, &len,
                             (size_t)m, nullptr);
      if (e != rocfft_status_success) {
        set_error("rocFFT plan creation failed (status %d)", (int)e);
        return SC_EDEVICE;
      }
      plans[key] = plan;
    }
  }
  d->plan = plan;
  rocfft_execution_info info = nullptr;
  if (rocfft_execution_info_create(&info) != rocfft_status_success) {
    set_error("rocFFT execution info creation failed");
    return SC_EDEVICE;
  }
  d->info = info;
  size_t wb = 0;
  if (rocfft_plan_get_work_buffer_size(plan, &wb) != rocfft_status_success) {
    set_error("rocFFT work buffer query failed");
    return SC_EDEVICE;
  }
  if (wb > 0) {
    void* w = pool_alloc(wb);
    if (!w) {
      set_error("rocFFT work buffer allocation failed");
      return SC_ENOMEM;
    }
    allocs_.push_back(w);
    d->work = w;
    d->work_bytes = wb;
    if (rocfft_execution_info_set_work_buffer(info, w, wb) != rocfft_status_success) {
      set_error("rocFFT work buffer binding failed");
      return SC_EDEVICE;
    }
  }
  (void)st;
  return SC_OK;
}

sc_status FastPoisson::dst_rows(const Dst& d, const void* in, int64_t pin, void* out, int64_t pout,
                                hipStream_t st) const {
  const int64_t n = d.n, m = d.m, N = 2 * (n + 1);
  const int64_t total = m * N;
  const unsigned eb = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  const double c = std::sqrt(2.0 / (double)(n + 1));
  const dim3 tgrid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
  if (dtype_ == SC_F64)
    hipLaunchKernelGGL(dst_extend_kernel<double>, dim3(eb), dim3(256), 0, st, static_cast<const double*>(in), pin, n,
                       m, static_cast<double*>(ext_));
  else
    hipLaunchKernelGGL(dst_extend_kernel<float>, dim3(eb), dim3(256), 0, st, static_cast<const float*>(in), pin, n,
                       m, static_cast<float*>(ext_));
  SC_HIP_CHECK(hipGetLastError());
  auto info = static_cast<rocfft_execution_info>(d.info);
  if (rocfft_execution_info_set_stream(info, st) != rocfft_status_success) {
    set_error("rocFFT stream binding failed");
    return SC_EDEVICE;
  }
  void* ib[1] = {ext_};
  void* ob[1] = {spec_};
  const rocfft_status e = rocfft_execute(static_cast<rocfft_plan>(d.plan), ib, ob, info);
  if (e != rocfft_status_success) {
    set_error("rocFFT execution failed (status %d)", (int)e);
    return SC_EDEVICE;
  }
  if (dtype_ == SC_F64)
    hipLaunchKernelGGL(dst_extract_kernel<double>, tgrid, dim3(256), 0, st, static_cast<const double*>(spec_), n, m,
                       static_cast<double*>(out), pout, c);
  else
    hipLaunchKernelGGL(dst_extract_kernel<float>, tgrid, dim3(256), 0, st, static_cast<const float*>(spec_), n, m,
                       static_cast<float*>(out), pout, (float)c);
  SC_HIP_CHECK(hipGetLastError());
  return SC_OK;
}

sc_status FastPoisson::init(int dim, const int64_t* n, double h, int dtype, hipStream_t st) {
  dim_ = dim;
  dtype_ = dtype;
  for (int a = 0; a < 3; ++a) n_[a] = a < dim ? n[a] : 1;
  const size_t es = dtype == SC_F64 ? 8 : 4;
  fft_ = fft_sides(dim, n_);
  if (fft_) {
    sc_status e;
    const int64_t mx = std::max(n_[0], n_[1]);
    ext_ = pool_alloc((size_t)(mx * (2 * mx + 2)) * es);
    spec_ = pool_alloc((size_t)(mx * (mx + 2)) * 2 * es);
    tr_ = pool_alloc((size_t)(n_[0] * n_[1]) * es);
    for (void* q : {ext_, spec_, tr_})
      if (q) allocs_.push_back(q);
    if (!ext_ || !spec_ || !tr_) {
      set_error("preconditioner allocation failed");
      return SC_ENOMEM;
    }
    if ((e = dst_init(&dx_, n_[0], n_[1], st)) != SC_OK || (e = dst_init(&dy_, n_[1], n_[0], st)) != SC_OK) return e;
    for (int a = 0; a < 2; ++a) {
      void* l = pool_alloc((size_t)n_[a] * 8);
      if (!l) {
        set_error("preconditioner allocation failed");
        return SC_ENOMEM;
      }
      allocs_.push_back(l);
      lam_[a] = static_cast<double*>(l);
      SC_HIP_CHECK(launch_pc_init(dtype, nullptr, lam_[a], n_[a], h, st));
    }
    return SC_OK;
  }
  split_ = split_sides(dim, n_);
  for (int a = 0; a < dim; ++a) {
    int same = -1;
    for (int c = 0; c < a; ++c)
      if (n_[c] == n_[a]) same = c;
    const int64_t m = n_[a];
    void* l = pool_alloc((size_t)m * 8);
    const int64_t hp = (m + 1) / 2, hm = m / 2;
    const int64_t mat = split_ ? hp * hp + hm * hm : m * m;
    void* d = same >= 0 ? S_[same] : pool_alloc((size_t)mat * es);
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
    if (split_)
      SC_HIP_CHECK(launch_pc_init_split(dtype, same >= 0 ? nullptr : d, lam_[a], m, h, st));
    else
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
  if (fft_) {
    // along x (rows of r) into tr (transposed), along y back into tmp; scale;
    // the same two transforms again into z
    if ((e = dst_rows(dx_, r, p, tr_, n1, st)) != SC_OK || (e = dst_rows(dy_, tr_, n1, tmp, p, st)) != SC_OK)
      return e;
    SC_HIP_CHECK(launch_pc_scale(dtype_, tmp, lay, n_, lam_[0], lam_[1], nullptr, s, st));
    if ((e = dst_rows(dx_, tmp, p, tr_, n1, st)) != SC_OK) return e;
    return dst_rows(dy_, tr_, n1, z, p, st);
  }
  if (!split_) {
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
  // Sine transforms split by the transform's even/odd symmetry (half the
  // flops of the full product; see launch_pc_init_split): along an axis of
  // n points, a butterfly folds the data into sums (first ceil(n/2)) and
  // reversed differences (last floor(n/2)), and two half-size GEMMs give
  // the transform with its even rows first and its odd rows after (the
  // order lam is stored in); the transposed half products followed by the
  // same butterfly bring such data back to natural order.
  const size_t es = dtype_ == SC_F64 ? 8 : 4;
  const int64_t N[3] = {n0, n1, n2};
  auto hpf = [&](int a) { return (N[a] + 1) / 2; };
  auto hmf = [&](int a) { return N[a] / 2; };
  auto Fo = [&](int a) { return static_cast<const void*>(S_[a]); };
  auto FeR = [&](int a) {
    return static_cast<const void*>(static_cast<const char*>(S_[a]) + (size_t)(hpf(a) * hpf(a)) * es);
  };
  auto off = [&](const void* q, int64_t elems) { return static_cast<const char*>(q) + elems * (int64_t)es; };
  auto offm = [&](void* q, int64_t elems) { return static_cast<char*>(q) + elems * (int64_t)es; };
  // along x (left products, per plane): out[0:hp] = Fo U[0:hp],
  // out[hp:n0] = FeR U[hp:n0]; inverse: the transposes
  auto along_x = [&](const void* U, void* out, bool inv) -> sc_status {
    sc_status r2;
    const int64_t hp = hpf(0), hm = hmf(0), zb = dim_ == 3 ? zp : 0;
    if ((r2 = gemm(hb, dtype_, hp, n1, hp, Fo(0), hp, 0, U, p, zb, out, p, zb, n2, inv, false)) != SC_OK) return r2;
    if (hm == 0) return SC_OK;
    return gemm(hb, dtype_, hm, n1, hm, FeR(0), hm, 0, off(U, hp), p, zb, offm(out, hp), p, zb, n2, inv, false);
  };
  // along y (right products, per plane) and along z (right products on
  // the x-z view of each y row): out[:, 0:hp] = U[:, 0:hp] Fo^T, ...
  auto along_yz = [&](int a, const void* U, void* out, bool inv) -> sc_status {
    sc_status r2;
    const int64_t hp = hpf(a), hm = hmf(a);
    const int64_t ld = a == 1 ? p : zp, bs = a == 1 ? (dim_ == 3 ? zp : 0) : p, nb = a == 1 ? n2 : n1;
    if ((r2 = gemm(hb, dtype_, n0, hp, hp, U, ld, bs, Fo(a), hp, 0, out, ld, bs, nb, false, !inv)) != SC_OK)
      return r2;
    if (hm == 0) return SC_OK;
    return gemm(hb, dtype_, n0, hm, hm, off(U, hp * ld), ld, bs, FeR(a), hm, 0, offm(out, hp * ld), ld, bs, nb, false,
                !inv);
  };
  auto fly = [&](const void* in, void* out, int a) -> sc_status {
    SC_HIP_CHECK(launch_butterfly(dtype_, in, out, lay, n_, a, st));
    return SC_OK;
  };
  if (dim_ == 2) {
    if ((e = fly(r, tmp, 0)) != SC_OK || (e = along_x(tmp, z, false)) != SC_OK || (e = fly(z, z, 1)) != SC_OK ||
        (e = along_yz(1, z, tmp, false)) != SC_OK)
      return e;
    SC_HIP_CHECK(launch_pc_scale(dtype_, tmp, lay, n_, lam_[0], lam_[1], nullptr, s, st));
    if ((e = along_x(tmp, z, true)) != SC_OK || (e = fly(z, z, 0)) != SC_OK ||
        (e = along_yz(1, z, tmp, true)) != SC_OK)
      return e;
    return fly(tmp, z, 1);
  }
  if ((e = fly(r, tmp, 0)) != SC_OK || (e = along_x(tmp, z, false)) != SC_OK || (e = fly(z, z, 1)) != SC_OK ||
      (e = along_yz(1, z, tmp, false)) != SC_OK || (e = fly(tmp, tmp, 2)) != SC_OK ||
      (e = along_yz(2, tmp, z, false)) != SC_OK)
    return e;
  SC_HIP_CHECK(launch_pc_scale(dtype_, z, lay, n_, lam_[0], lam_[1], lam_[2], s, st));
  if ((e = along_yz(2, z, tmp, true)) != SC_OK || (e = fly(tmp, tmp, 2)) != SC_OK ||
      (e = along_yz(1, tmp, z, true)) != SC_OK || (e = fly(z, z, 1)) != SC_OK || (e = along_x(z, tmp, true)) != SC_OK)
    return e;
  return fly(tmp, z, 0);
}

}  // namespace sc
