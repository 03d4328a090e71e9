// Gradient of sigma = PPL(L, X) with respect to the Cholesky vectors.
//
// For a real loss with upstream gradient G (PyTorch's complex convention),
//   Lbar^P = 2 sum_m G_m conj(L^P) X_m^H,
// with G_m, X_m the full antisymmetric v x v matrices of row m = (r, ij).
// Taking the complex conjugate, Lbar = 2 conj(Z) with
//   Z^P_ac = sum_{b,d} R[(a,c),(b,d)] L^P_bd,
//   R[(a,c),(b,d)] = sum_m conj(G_m^ab) X_m^cd,
// where R (v^2 x v^2) plays the role of the recomputed integral tile: it is
// never stored whole.  For a panel of virtual indices a:
//   1. R_panel: one strided-batched GEMM per a over the rows m (batch over c),
//      written directly in (a,c) x (b,d) order;
//   2. Z[:, (a,c)] = L (nchol x v^2) . R_panel^T, one GEMM with K = v^2.
// Both are plain dense GEMMs and go to rocBLAS; unpacking the packed doubles
// to full antisymmetric matrices and the final conjugation are HIP kernels.
#include <rocblas/rocblas.h>

#include <algorithm>

#include "internal.hpp"

namespace lrcc {

namespace {

template <typename C> struct Real;
template <> struct Real<double2> { typedef double t; };
template <> struct Real<float2> { typedef float t; };

__device__ inline long pidx(long p, long q, long n) { return p * (2 * n - p - 1) / 2 + (q - p - 1); }

// packed [M][npo? no: rows m][npv] -> full antisymmetric [M][v][v]
template <typename C>
__global__ void k_unpack_full(const C* __restrict__ Xp, long M, int v, long npv,
                              C* __restrict__ Xf) {
  const long total = M * v * v;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e % v, a = (e / v) % v;
    const long m = e / ((long)v * v);
    C z;
    z.x = 0;
    z.y = 0;
    if (a < b) {
      z = Xp[m * npv + pidx(a, b, v)];
    } else if (a > b) {
      z = Xp[m * npv + pidx(b, a, v)];
      z.x = -z.x;
      z.y = -z.y;
    }
    Xf[e] = z;
  }
}

template <typename C>
__global__ void k_conj_scale(long n, typename Real<C>::t s, C* __restrict__ p) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x) {
    C z = p[i];
    z.x = s * z.x;
    z.y = -s * z.y;
    p[i] = z;
  }
}

inline int grid_for(long n) {
  long g = (n + 255) / 256;
  return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

rocblas_status gemm_sb(rocblas_handle rb, bool c128, rocblas_operation ta, rocblas_operation tb,
                       int m, int n, int k, const void* A, long lda, long sa, const void* B,
                       long ldb, long sb, void* Cm, long ldc, long sc, int batch) {
  if (c128) {
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    return rocblas_zgemm_strided_batched(
        rb, ta, tb, m, n, k, &one, static_cast<const rocblas_double_complex*>(A), lda, sa,
        static_cast<const rocblas_double_complex*>(B), ldb, sb, &zero,
        static_cast<rocblas_double_complex*>(Cm), ldc, sc, batch);
  }
  const rocblas_float_complex one{1.0f, 0.0f}, zero{0.0f, 0.0f};
  return rocblas_cgemm_strided_batched(
      rb, ta, tb, m, n, k, &one, static_cast<const rocblas_float_complex*>(A), lda, sa,
      static_cast<const rocblas_float_complex*>(B), ldb, sb, &zero,
      static_cast<rocblas_float_complex*>(Cm), ldc, sc, batch);
}

rocblas_status gemm(rocblas_handle rb, bool c128, rocblas_operation ta, rocblas_operation tb,
                    int m, int n, int k, const void* A, long lda, const void* B, long ldb,
                    void* Cm, long ldc) {
  if (c128) {
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    return rocblas_zgemm(rb, ta, tb, m, n, k, &one,
                         static_cast<const rocblas_double_complex*>(A), lda,
                         static_cast<const rocblas_double_complex*>(B), ldb, &zero,
                         static_cast<rocblas_double_complex*>(Cm), ldc);
  }
  const rocblas_float_complex one{1.0f, 0.0f}, zero{0.0f, 0.0f};
  return rocblas_cgemm(rb, ta, tb, m, n, k, &one, static_cast<const rocblas_float_complex*>(A),
                       lda, static_cast<const rocblas_float_complex*>(B), ldb, &zero,
                       static_cast<rocblas_float_complex*>(Cm), ldc);
}

}  // namespace

lrcc_status grad_L(lrcc_handle h, const Geom& g, const void* L, const void* X, const void* G,
                   void* dL, lrcc_dtype dt) {
  const bool c128 = dt == LRCC_C128;
  const size_t es = c128 ? 16 : 8;
  const long v = g.v, v2 = v * v, M = g.M;
  const size_t nl = (size_t)g.nchol * v2;
  if (nl == 0) return LRCC_OK;
  if (M == 0 || g.npv == 0) {  // sigma does not depend on L: zero gradient
    LRCC_HIP(h, hipMemsetAsync(dL, 0, nl * es, h->stream));
    return LRCC_OK;
  }
  if (!h->rb) {
    if (rocblas_create_handle(reinterpret_cast<rocblas_handle*>(&h->rb)) !=
        rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_create_handle failed");
  }
  rocblas_handle rb = static_cast<rocblas_handle>(h->rb);
  if (rocblas_set_stream(rb, h->stream) != rocblas_status_success)
    return fail(h, LRCC_ERR_DEVICE, "rocblas_set_stream failed");
  // full antisymmetric G and X: [M][v][v]
  const size_t nf = (size_t)M * v2 * es;
  LRCC_HIP(h, h->gb.ensure(2 * nf));
  char* Gf = h->gb.as<char>();
  char* Xf = Gf + nf;
  if (c128) {
    hipLaunchKernelGGL(k_unpack_full<double2>, dim3(grid_for(M * v2)), dim3(256), 0, h->stream,
                       static_cast<const double2*>(G), M, (int)v, g.npv,
                       reinterpret_cast<double2*>(Gf));
    hipLaunchKernelGGL(k_unpack_full<double2>, dim3(grid_for(M * v2)), dim3(256), 0, h->stream,
                       static_cast<const double2*>(X), M, (int)v, g.npv,
                       reinterpret_cast<double2*>(Xf));
  } else {
    hipLaunchKernelGGL(k_unpack_full<float2>, dim3(grid_for(M * v2)), dim3(256), 0, h->stream,
                       static_cast<const float2*>(G), M, (int)v, g.npv,
                       reinterpret_cast<float2*>(Gf));
    hipLaunchKernelGGL(k_unpack_full<float2>, dim3(grid_for(M * v2)), dim3(256), 0, h->stream,
                       static_cast<const float2*>(X), M, (int)v, g.npv,
                       reinterpret_cast<float2*>(Xf));
  }
  LRCC_HIP(h, hipGetLastError());
  // R panel: na virtual indices a at a time, na * v * v^2 elements
  const size_t per_a = (size_t)v * v2 * es;
  const size_t cap = (size_t)4 << 30;
  const long na = std::max<long>(1, std::min<long>(v, (long)(cap / per_a)));
  LRCC_HIP(h, h->vws.ensure(na * per_a));
  char* R = h->vws.as<char>();
  for (long a0 = 0; a0 < v; a0 += na) {
    const long n = std::min(na, v - a0);
    for (long al = 0; al < n; ++al) {
      const long a = a0 + al;
      // column-major: R_ac (d x b) = X_c^T (d x m) . conj(G_a) (m x b), batch over c
      rocblas_status s = gemm_sb(rb, c128, rocblas_operation_none,
                                 rocblas_operation_conjugate_transpose, (int)v, (int)v, (int)M,
                                 Xf, v2, v, Gf + a * v * es, v2, 0, R + al * v * v2 * es, v, v2,
                                 (int)v);
      if (s != rocblas_status_success) return fail(h, LRCC_ERR_DEVICE, "rocBLAS batched GEMM failed");
    }
    // column-major: Z^T[(a,c), P] = R_panel (n v x v^2) . L^T (v^2 x nchol)
    rocblas_status s = gemm(rb, c128, rocblas_operation_transpose, rocblas_operation_none,
                            (int)(n * v), g.nchol, (int)v2, R, v2, L, v2,
                            static_cast<char*>(dL) + a0 * v * es, v2);
    if (s != rocblas_status_success) return fail(h, LRCC_ERR_DEVICE, "rocBLAS GEMM failed");
  }
  // Lbar = 2 conj(Z)
  if (c128)
    hipLaunchKernelGGL(k_conj_scale<double2>, dim3(grid_for((long)nl)), dim3(256), 0, h->stream,
                       (long)nl, 2.0, static_cast<double2*>(dL));
  else
    hipLaunchKernelGGL(k_conj_scale<float2>, dim3(grid_for((long)nl)), dim3(256), 0, h->stream,
                       (long)nl, 2.0f, static_cast<float2*>(dL));
  LRCC_HIP(h, hipGetLastError());
  return LRCC_OK;
}

}  // namespace lrcc
