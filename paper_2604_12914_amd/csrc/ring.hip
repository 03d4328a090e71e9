// Ring (particle-hole) term of the doubles-doubles Jacobian at zero
// ground-state amplitudes (Sec. 2.2), with the integrals from the Cholesky
// vectors of Sec. 3:
//   <kb||cj> = sum_P L^P_kc L^P_bj - sum_P L^P_kj L^P_bc
//   r_ij^ab  = sum_{k,c} <kb||cj> X_ik^ac,   sigma = P(ij) P(ab) r.
// The particle-hole integral matrix M[(kc)][(jb)] = <kb||cj> is formed
// explicitly (two GEMMs over the vectors and one transposing combine, (ov)^2
// entries: no more than two particle indices), then per right-hand side
// the unpacked amplitudes Xt[(ia)][(kc)] = X_ik^ac multiply it (one GEMM for
// all right-hand sides) and the four permutations are gathered into the
// packed output.
//
//   A' [(kc)][(bj)] = sum_P Lov[P][k][c] Lvo[P][b][j]     (rocBLAS zgemm)
//   B2 [(bc)][(kj)] = sum_P Lvv[P][b][c] Loo[P][k][j]     (rocBLAS zgemm)
//   k_ring_m:   M[(kc)][(jb)] = A'[(kc)][(bj)] - B2[(bc)][(kj)], 32 x 32 LDS
//               tiles over (b, j) so that reads and writes are both whole rows
//   k_ring_x:   Xt from the packed doubles
//   R = Xt M    (rocBLAS zgemm, nrhs ov x ov x ov)
//   k_ring_out: sigma[r][(i<j)][(a<b)] (+)= R_ij^ab - R_ji^ab - R_ij^ba + R_ji^ba
#include <rocblas/rocblas.h>

#include <algorithm>

#include "internal.hpp"

namespace lrcc {

namespace {

constexpr int RT = 32;

// Grid: x = (b-tile, j-tile), y = (k, c).  Block RT x 8 threads.
__global__ __launch_bounds__(RT * 8) void k_ring_m(int o, int v, const double2* __restrict__ Ap,
                                                  const double2* __restrict__ B2,
                                                  double2* __restrict__ M) {
  __shared__ double2 tile[RT][RT + 1];  // [b][j]
  const int ntj = (o + RT - 1) / RT;
  const int b0 = (blockIdx.x / ntj) * RT, j0 = (blockIdx.x % ntj) * RT;
  const int kc = blockIdx.y, k = kc / v, c = kc % v;
  const long ov = (long)o * v, o2 = (long)o * o;
  const int tx = threadIdx.x % RT, ty = threadIdx.x / RT;
  for (int r = ty; r < RT; r += 8) {
    const int b = b0 + r, j = j0 + tx;
    double2 val = make_double2(0.0, 0.0);
    if (b < v && j < o) {
      const double2 x = Ap[(long)kc * ov + (long)b * o + j];
      const double2 y = B2[((long)b * v + c) * o2 + (long)k * o + j];
      val = make_double2(x.x - y.x, x.y - y.y);
    }
    tile[r][tx] = val;
  }
  __syncthreads();
  for (int r = ty; r < RT; r += 8) {
    const int j = j0 + r, b = b0 + tx;
    if (j < o && b < v) M[(long)kc * ov + (long)j * v + b] = tile[tx][r];
  }
}

__device__ inline long pair_index(int p, int q, int n) {  // p < q
  return (long)p * (2 * n - p - 1) / 2 + (q - p - 1);
}

// Xt[((r o + i) v + a)][(k v + c)] = X_ik^ac (antisymmetric unpacking).
__global__ void k_ring_x(int o, int v, int nrhs, const double2* __restrict__ X,
                         double2* __restrict__ Xt) {
  const long ov = (long)o * v;
  const long total = (long)nrhs * ov * ov;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long row = e / ov, col = e % ov;
  const int r = (int)(row / ov), i = (int)(row % ov / v), a = (int)(row % v);
  const int k = (int)(col / v), c = (int)(col % v);
  double2 x = make_double2(0.0, 0.0);
  if (i != k && a != c) {
    const long npo = (long)o * (o - 1) / 2, npv = (long)v * (v - 1) / 2;
    const long p = pair_index(min(i, k), max(i, k), o), q = pair_index(min(a, c), max(a, c), v);
    x = X[((long)r * npo + p) * npv + q];
    if ((i > k) != (a > c)) x = make_double2(-x.x, -x.y);
  }
  Xt[e] = x;
}

// One thread per packed output element.
__global__ void k_ring_out(int o, int v, int nrhs, const double2* __restrict__ R, int accumulate,
                           double2* __restrict__ S) {
  const long npo = (long)o * (o - 1) / 2, npv = (long)v * (v - 1) / 2;
  const long total = (long)nrhs * npo * npv;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long q = e % npv, rp = e / npv;
  const long p = rp % npo;
  const int r = (int)(rp / npo);
  // decode the pairs (p over o, q over v): row-major upper triangles
  int i = 0;
  while (pair_index(i, o - 1, o) < p) ++i;
  const int j = (int)(p - pair_index(i, i + 1, o)) + i + 1;
  int a = 0;
  while (pair_index(a, v - 1, v) < q) ++a;
  const int b = (int)(q - pair_index(a, a + 1, v)) + a + 1;
  const long ov = (long)o * v;
  auto Rv = [&](int ii, int aa, int jj, int bb) {
    return R[(((long)r * o + ii) * v + aa) * ov + (long)jj * v + bb];
  };
  const double2 t1 = Rv(i, a, j, b), t2 = Rv(j, a, i, b), t3 = Rv(i, b, j, a), t4 = Rv(j, b, i, a);
  double2 y = make_double2(t1.x - t2.x - t3.x + t4.x, t1.y - t2.y - t3.y + t4.y);
  if (accumulate) {
    y.x += S[e].x;
    y.y += S[e].y;
  }
  S[e] = y;
}

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

rocblas_status zgemm(rocblas_handle rb, rocblas_operation ta, rocblas_operation tb, long m,
                     long n, long k, const double2* A, long lda, const double2* B, long ldb,
                     double2* C, long ldc) {
  const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
  return rocblas_zgemm(rb, ta, tb, (rocblas_int)m, (rocblas_int)n, (rocblas_int)k, &one,
                       reinterpret_cast<const rocblas_double_complex*>(A), (rocblas_int)lda,
                       reinterpret_cast<const rocblas_double_complex*>(B), (rocblas_int)ldb,
                       &zero, reinterpret_cast<rocblas_double_complex*>(C), (rocblas_int)ldc);
}

// out[P][j][i] = in[P][i][j] for [n0][n1][n2] complex arrays.
__global__ void k_tr3(long n0, int n1, int n2, const double2* __restrict__ in,
                      double2* __restrict__ out) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n0 * n1 * n2) return;
  const long P = e / ((long)n1 * n2);
  const int r = (int)(e % ((long)n1 * n2));
  const int i = r / n2, j = r % n2;
  out[(P * n2 + j) * n1 + i] = in[e];
}

hipError_t transpose3(long n0, int n1, int n2, const void* in, void* out, hipStream_t st) {
  const long n = n0 * n1 * n2;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tr3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n0, n1, n2,
                     static_cast<const double2*>(in), static_cast<double2*>(out));
  return hipGetLastError();
}

lrcc_status get_blas(lrcc_handle h, rocblas_handle* rb) {
  if (!h->rb) {
    if (rocblas_create_handle(reinterpret_cast<rocblas_handle*>(&h->rb)) !=
        rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_create_handle failed");
  }
  *rb = static_cast<rocblas_handle>(h->rb);
  if (rocblas_set_stream(*rb, h->stream) != rocblas_status_success)
    return fail(h, LRCC_ERR_DEVICE, "rocblas_set_stream failed");
  return LRCC_OK;
}

}  // namespace

size_t ring_m_bytes(int o, int v) { return al256((size_t)o * v * o * v * 16); }

size_t ring_build_ws_bytes(int o, int v, int nchol, bool transposed) {
  const size_t ov2 = (size_t)o * v * o * v;
  size_t b = 2 * al256(ov2 * 16);
  if (transposed) b += al256((size_t)nchol * (o + v) * (o + v) * 16);
  return b;
}

size_t ring_apply_ws_bytes(int o, int v, int nrhs) {
  return 2 * al256((size_t)nrhs * o * v * o * v * 16);
}

size_t ring_ws_bytes(int o, int v, int nrhs) {
  return ring_m_bytes(o, v) + std::max(ring_build_ws_bytes(o, v, 0, false),
                                       ring_apply_ws_bytes(o, v, nrhs));
}

lrcc_status ring_build_m(lrcc_handle h, int o, int v, int nchol, const void* Loo,
                         const void* Lov, const void* Lvo, const void* Lvv, bool transposed,
                         double2* M, void* ws) {
  hipStream_t st = h->stream;
  const long ov = (long)o * v, o2 = (long)o * o, v2 = (long)v * v;
  const size_t ov2 = (size_t)ov * ov;
  if (ov2 == 0) return LRCC_OK;
  char* p = static_cast<char*>(ws);
  double2* Ap = reinterpret_cast<double2*>(p);
  p += al256(ov2 * 16);
  double2* B2 = reinterpret_cast<double2*>(p);
  p += al256(ov2 * 16);
  if (nchol > 0) {
    if (transposed) {
      // the blocks of (L^P)^T: oo and vv transposed, ov and vo swapped and transposed
      double2* t = reinterpret_cast<double2*>(p);
      double2 *too = t, *tov = too + nchol * o2, *tvo = tov + nchol * ov, *tvv = tvo + nchol * ov;
      LRCC_HIP(h, transpose3(nchol, o, o, Loo, too, st));
      LRCC_HIP(h, transpose3(nchol, v, o, Lvo, tov, st));
      LRCC_HIP(h, transpose3(nchol, o, v, Lov, tvo, st));
      LRCC_HIP(h, transpose3(nchol, v, v, Lvv, tvv, st));
      Loo = too;
      Lov = tov;
      Lvo = tvo;
      Lvv = tvv;
    }
    rocblas_handle rb;
    lrcc_status s = get_blas(h, &rb);
    if (s != LRCC_OK) return s;
    const rocblas_operation N = rocblas_operation_none, T = rocblas_operation_transpose;
    // A'^c((bj), (kc)) = sum_P Lvo^c((bj), P) Lov^c((kc), P)
    if (zgemm(rb, N, T, ov, ov, nchol, static_cast<const double2*>(Lvo), ov,
              static_cast<const double2*>(Lov), ov, Ap, ov) != rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_zgemm failed");
    // B2^c((kj), (bc)) = sum_P Loo^c((kj), P) Lvv^c((bc), P)
    if (zgemm(rb, N, T, o2, v2, nchol, static_cast<const double2*>(Loo), o2,
              static_cast<const double2*>(Lvv), v2, B2, o2) != rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_zgemm failed");
  } else {
    LRCC_HIP(h, fill_zero(Ap, ov2 * 16, st));
    LRCC_HIP(h, fill_zero(B2, ov2 * 16, st));
  }
  const int ntb = (v + RT - 1) / RT, ntj = (o + RT - 1) / RT;
  hipLaunchKernelGGL(k_ring_m, dim3(ntb * ntj, (unsigned)ov), dim3(RT * 8), 0, st, o, v, Ap, B2,
                     M);
  LRCC_HIP(h, hipGetLastError());
  return LRCC_OK;
}

lrcc_status ring_apply(lrcc_handle h, int o, int v, int nrhs, const double2* M, const void* X,
                       void* S, bool accumulate, void* ws) {
  hipStream_t st = h->stream;
  const long ov = (long)o * v;
  const size_t ov2 = (size_t)ov * ov;
  const long npo = (long)o * (o - 1) / 2, npv = (long)v * (v - 1) / 2;
  const long nout = (long)nrhs * npo * npv;
  if (nout == 0) return LRCC_OK;
  double2* Xt = static_cast<double2*>(ws);
  double2* R = reinterpret_cast<double2*>(static_cast<char*>(ws) +
                                          al256((size_t)nrhs * ov2 * 16));
  const long nx = (long)nrhs * (long)ov2;
  hipLaunchKernelGGL(k_ring_x, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, o, v, nrhs,
                     static_cast<const double2*>(X), Xt);
  LRCC_HIP(h, hipGetLastError());
  rocblas_handle rb;
  lrcc_status s = get_blas(h, &rb);
  if (s != LRCC_OK) return s;
  // R^c((jb), (ria)) = sum_(kc) M^c((jb), (kc)) Xt^c((kc), (ria))
  if (zgemm(rb, rocblas_operation_none, rocblas_operation_none, ov, (long)nrhs * ov, ov, M, ov,
            Xt, ov, R, ov) != rocblas_status_success)
    return fail(h, LRCC_ERR_DEVICE, "rocblas_zgemm failed");
  hipLaunchKernelGGL(k_ring_out, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, st, o, v,
                     nrhs, R, accumulate ? 1 : 0, static_cast<double2*>(S));
  LRCC_HIP(h, hipGetLastError());
  return LRCC_OK;
}

lrcc_status ring_run(lrcc_handle h, int o, int v, int nchol, int nrhs, const void* Loo,
                     const void* Lov, const void* Lvo, const void* Lvv, const void* X, void* S,
                     bool accumulate, void* ws) {
  const long npo = (long)o * (o - 1) / 2, npv = (long)v * (v - 1) / 2;
  if ((long)nrhs * npo * npv == 0) return LRCC_OK;
  double2* M = static_cast<double2*>(ws);
  void* rest = static_cast<char*>(ws) + ring_m_bytes(o, v);
  lrcc_status s = ring_build_m(h, o, v, nchol, Loo, Lov, Lvo, Lvv, false, M, rest);
  if (s != LRCC_OK) return s;
  return ring_apply(h, o, v, nrhs, M, X, S, accumulate, rest);
}

}  // namespace lrcc
