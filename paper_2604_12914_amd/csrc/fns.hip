// Perturbation-sensitive natural spinors (FNS++) of the virtual space,
// Sec. 2.4, with the diagonalisation, Fock transform, semicanonicalisation
// and basis change of Sec. 2.3, for a canonical reference (diagonal Fock
// matrix, spinor energies eps).
//
// Pipeline on the handle's stream (o occupied, v virtual spinors, npo =
// o(o-1)/2 occupied pairs; all complex128, row-major):
//   1. G = L^T L over the occupied-virtual Cholesky vectors, G[(ia)][(jb)] =
//      <ij|ab>, for the blocks i < j only (one zgemm per i, (o-1-i) v x v x
//      nchol: half of the full product)
//   2. k_fns_t: t_ij^ab = (G[ia][jb] - G[ib][ja]) / (e_i + e_j - e_a - e_b)
//      for i < j, t_ji = -t_ij, zero for i = j or a = b; the transposed read
//      goes through LDS tiles
//   3. k_fns_hbar: Hb_ii = e_i + 1/2 sum_{jab} |t_ij^ab|^2 D_ij^ab and
//      Hb_aa = e_a - 1/2 sum_{mnf} |t_mn^af|^2 D_mn^af (t conj<||> = |t|^2 D,
//      the second sum taken over the antisymmetric partner t_mn^af), each
//      index's range cut into fixed segments, summed in a fixed order
//   per perturbation component x:
//   4. X'[(ijc)][a] = sum_e t_ij^ce A_ae for i < j (one zgemm per i); by the
//      antisymmetry of t the vv term of the perturbed doubles,
//      P(a,c) sum_e t_ij^ec A_ae, is X'[(ija)][c] - X'[(ijc)][a]
//   5. Y[i][(jac)] = sum_m A_mi t_mj^ac (one zgemm, o v^2 x o x o)
//   6. k_fns_pert: Q[a][(i<j)][c] = (X'_ij,ac - X'_ij,ca - Y_ij,ac + Y_ji,ac)
//      / (Hb_aa + Hb_cc - Hb_ii - Hb_jj + w), the perturbed doubles for
//      i < j only, laid out so that the density is one product;
//      k_fns_t1: T1[a][i] = A_ia / (Hb_aa - Hb_ii + w)
//   7. G_ab += (1/ncomp) (sum_{i<j,c} Q[a]..Q[b]^* + sum_i T1[a][i] T1[b][i]^*)
//      (the restriction to i < j absorbs the factor 1/2; the long pair sum
//      is split into chunks whose partial products are added in order)
//   then:
//   8. Jacobi eigensolver on G, occupations ordered by descending magnitude;
//      keep = number with |n| > threshold (read back to the host)
//   9. Vt = the kept columns, S = diag(e_v) Vt (one gather)
//  10. Ft = Vt^H S (zgemm), its eigenpairs in ascending order (Jacobi)
//  11. B = Vt Z (zgemm)
// Plain GEMMs go to rocBLAS; the elementwise and transposing steps, the
// reductions and the eigensolver are the kernels below and in heev.hip.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace lrcc {

namespace {

constexpr int TT = 32;  // transpose tile edge
constexpr int TR = 8;   // rows per thread pass (block = TT x TR threads)

// Step 2.  Grid: x = tile (a-tile, b-tile), y = i * o + j.  Only the blocks
// i < j of G are formed; t_ij = -t_ji gives the rest (i > j reads block
// (j, i)), and t_ii = 0.
__global__ __launch_bounds__(TT * TR) void k_fns_t(int o, int v, const double2* __restrict__ G,
                                                  const double* __restrict__ eps,
                                                  double2* __restrict__ t) {
  __shared__ double2 tr[TT][TT + 1];
  const int ntb = (v + TT - 1) / TT;
  const int a0 = (blockIdx.x / ntb) * TT, b0 = (blockIdx.x % ntb) * TT;
  const int i = blockIdx.y / o, j = blockIdx.y % o;
  const int lo = min(i, j), hi = max(i, j);
  const double sg = i < j ? 1.0 : -1.0;
  const long ov = (long)o * v;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  // tr[bl][al] = G[(lo, b0+bl)][(hi, a0+al)]
  if (i != j) {
    for (int r = ty; r < TT; r += TR) {
      const int b = b0 + r, a = a0 + tx;
      tr[r][tx] = (b < v && a < v) ? G[((long)lo * v + b) * ov + (long)hi * v + a]
                                   : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  const double eij = eps[i] + eps[j];
  for (int r = ty; r < TT; r += TR) {
    const int a = a0 + r, b = b0 + tx;
    if (a >= v || b >= v) continue;
    double2 y = make_double2(0.0, 0.0);
    if (i != j && a != b) {
      const double2 g1 = G[((long)lo * v + a) * ov + (long)hi * v + b];
      const double2 g2 = tr[tx][r];
      const double inv = sg / (eij - eps[o + a] - eps[o + b]);
      y = make_double2((g1.x - g2.x) * inv, (g1.y - g2.y) * inv);
    }
    t[(((long)i * o + j) * v + a) * v + b] = y;
  }
}

constexpr int HB = 256;
__device__ inline double block_sum(double x, double* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int w = HB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

// Step 3.  Grid (o + v, NSEG): blockIdx.x < o sums segment blockIdx.y of the
// (j, a, b) range of occupied i; otherwise segment blockIdx.y of the
// (m, n, f) range of virtual a.  part[idx][seg] holds the segment sums,
// k_fns_hbar_fin adds them in segment order (deterministic).
constexpr int NSEG = 32;
__global__ __launch_bounds__(HB) void k_fns_hbar(int o, int v, const double2* __restrict__ t,
                                                 const double* __restrict__ eps,
                                                 double* __restrict__ part) {
  __shared__ double sh[HB];
  const long v2 = (long)v * v;
  const int seg = blockIdx.y;
  double acc = 0.0;
  if ((int)blockIdx.x < o) {
    const int i = blockIdx.x;
    const long n = (long)o * v2, e0 = n * seg / NSEG, e1 = n * (seg + 1) / NSEG;
    const double2* ti = t + (long)i * n;
    for (long e = e0 + threadIdx.x; e < e1; e += HB) {
      const int j = (int)(e / v2), a = (int)(e / v % v), b = (int)(e % v);
      const double2 x = ti[e];
      acc += (x.x * x.x + x.y * x.y) * (eps[i] + eps[j] - eps[o + a] - eps[o + b]);
    }
  } else {
    const int a = blockIdx.x - o;
    const long n = (long)o * o * v, e0 = n * seg / NSEG, e1 = n * (seg + 1) / NSEG;
    for (long e = e0 + threadIdx.x; e < e1; e += HB) {
      const long mn = e / v;
      const int f = (int)(e % v), m = (int)(mn / o), nn = (int)(mn % o);
      const double2 x = t[(mn * v + a) * v + f];
      acc += (x.x * x.x + x.y * x.y) * (eps[m] + eps[nn] - eps[o + a] - eps[o + f]);
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(long)blockIdx.x * NSEG + seg] = s;
}

__global__ void k_fns_hbar_fin(int o, int v, const double* __restrict__ part,
                               const double* __restrict__ eps, double* __restrict__ hbar) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= o + v) return;
  double s = 0.0;
  for (int k = 0; k < NSEG; ++k) s += part[(long)idx * NSEG + k];
  hbar[idx] = eps[idx] + (idx < o ? 0.5 : -0.5) * s;
}

// Gm += w * sum_s P[s] (fixed order).
__global__ void k_sum_parts(long n, int ns, const double2* __restrict__ P, double wgt,
                            double2* __restrict__ Gm) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < ns; ++k) {
    const double2 x = P[(long)k * n + e];
    acc.x += x.x;
    acc.y += x.y;
  }
  Gm[e].x += wgt * acc.x;
  Gm[e].y += wgt * acc.y;
}

// Step 6.  Grid: x = tile (a-tile, c-tile), y = occupied pair p (i < j).
// Xp = X' [o][o][v][v] (X'_ij[c][a] in row (i, j, c), column a), Y [o][o][v][v].
__global__ __launch_bounds__(TT * TR) void k_fns_pert(int o, int v, const int* __restrict__ otab,
                                                     const double2* __restrict__ Xp,
                                                     const double2* __restrict__ Y,
                                                     const double* __restrict__ hbar, double w,
                                                     double2* __restrict__ Q) {
  __shared__ double2 tr[TT][TT + 1];
  const int ntc = (v + TT - 1) / TT;
  const int a0 = (blockIdx.x / ntc) * TT, c0 = (blockIdx.x % ntc) * TT;
  const int p = blockIdx.y;
  const int npo = o * (o - 1) / 2;
  const int i = otab[p] >> 16, j = otab[p] & 0xffff;
  const long v2 = (long)v * v;
  const double2* xij = Xp + ((long)i * o + j) * v2;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  // tr[cl][al] = X'_ij[c0+cl][a0+al]
  for (int r = ty; r < TT; r += TR) {
    const int c = c0 + r, a = a0 + tx;
    tr[r][tx] = (c < v && a < v) ? xij[(long)c * v + a] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double hij = hbar[i] + hbar[j];
  const double2* yij = Y + ((long)i * o + j) * v2;
  const double2* yji = Y + ((long)j * o + i) * v2;
  for (int r = ty; r < TT; r += TR) {
    const int a = a0 + r, c = c0 + tx;
    if (a >= v || c >= v) continue;
    const double2 x1 = xij[(long)a * v + c];  // X'_ij[a][c]
    const double2 x2 = tr[tx][r];             // X'_ij[c][a]
    const double2 y1 = yij[(long)a * v + c], y2 = yji[(long)a * v + c];
    const double inv = 1.0 / (hbar[o + a] + hbar[o + c] - hij + w);
    Q[((long)a * npo + p) * v + c] =
        make_double2((x1.x - x2.x - y1.x + y2.x) * inv, (x1.y - x2.y - y1.y + y2.y) * inv);
  }
}

// Step 6, singles: T1[a][i] = A_ov[i][a] / (Hb_aa - Hb_ii + w).
__global__ void k_fns_t1(int o, int v, const double2* __restrict__ Aov,
                         const double* __restrict__ hbar, double w, double2* __restrict__ T1) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= o * v) return;
  const int a = e / o, i = e % o;
  const double2 x = Aov[(long)i * v + a];
  const double inv = 1.0 / (hbar[o + a] - hbar[i] + w);
  T1[e] = make_double2(x.x * inv, x.y * inv);
}

__global__ void k_conj_copy(long n, const double2* __restrict__ in, double2* __restrict__ out) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < n) out[e] = make_double2(in[e].x, -in[e].y);
}

__global__ void k_tr_small(int o, const double2* __restrict__ in, double2* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < o * o) out[(e % o) * o + e / o] = in[e];
}

__global__ void k_fns_pairs(int o, int* __restrict__ otab) {
  const int i = blockIdx.x;
  for (int j = i + 1 + threadIdx.x; j < o; j += blockDim.x) {
    const int p = i * (2 * o - i - 1) / 2 + (j - i - 1);
    otab[p] = (i << 16) | j;
  }
}

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

rocblas_status zgemm(rocblas_handle rb, rocblas_operation ta, rocblas_operation tb, long m,
                     long n, long k, double2 alpha, const double2* A, long lda, const double2* B,
                     long ldb, double2 beta, double2* C, long ldc) {
  const rocblas_double_complex al{alpha.x, alpha.y}, be{beta.x, beta.y};
  return rocblas_zgemm(rb, ta, tb, (rocblas_int)m, (rocblas_int)n, (rocblas_int)k, &al,
                       reinterpret_cast<const rocblas_double_complex*>(A), (rocblas_int)lda,
                       reinterpret_cast<const rocblas_double_complex*>(B), (rocblas_int)ldb, &be,
                       reinterpret_cast<rocblas_double_complex*>(C), (rocblas_int)ldc);
}

rocblas_status zgemm_sb(rocblas_handle rb, rocblas_operation ta, rocblas_operation tb, long m,
                        long n, long k, double2 alpha, const double2* A, long lda, long sa,
                        const double2* B, long ldb, long sb, double2 beta, double2* C, long ldc,
                        long sc, long batch) {
  const rocblas_double_complex al{alpha.x, alpha.y}, be{beta.x, beta.y};
  return rocblas_zgemm_strided_batched(
      rb, ta, tb, (rocblas_int)m, (rocblas_int)n, (rocblas_int)k, &al,
      reinterpret_cast<const rocblas_double_complex*>(A), (rocblas_int)lda, sa,
      reinterpret_cast<const rocblas_double_complex*>(B), (rocblas_int)ldb, sb, &be,
      reinterpret_cast<rocblas_double_complex*>(C), (rocblas_int)ldc, sc, (rocblas_int)batch);
}

// Split of the density product's K = npo v range: enough chunks to fill
// the chip with 64 x 64 output tiles, each chunk at least 1024 long.
int density_splits(int v, long K) {
  const long tiles = ((v + 63) / 64) * (long)((v + 63) / 64);
  long ns = (1024 + tiles - 1) / tiles;
  ns = std::min(ns, std::max(1L, K / 1024));
  return (int)std::min(ns, 64L);
}

}  // namespace

size_t fns_ws_bytes(int o, int v, int ncomp) {
  const size_t o2v2 = (size_t)o * o * v * v, npo = (size_t)o * (o - 1) / 2;
  size_t b = 0;
  b += al256(o2v2 * 16);                  // G, then X'
  b += al256(o2v2 * 16);                  // t
  b += ncomp ? al256(o2v2 * 16) : 0;      // Y
  b += ncomp ? al256(npo * v * v * 16) : 0;  // Q
  b += al256((size_t)o * v * 16);         // T1
  b += al256((size_t)v * v * 16);         // gamma
  b += al256((size_t)(o + v) * 8);        // hbar
  b += al256((size_t)v * 8);              // occupations
  b += al256(npo * 4 + 4);                // pair table
  b += al256((size_t)v * 4);              // eigen permutation
  b += al256((size_t)v * v * 16) * 4;     // Vt, S, Ft, Z
  b += al256((size_t)(o + v) * NSEG * 8);  // hbar segment sums
  b += al256((size_t)o * o * 16);           // transposed A_oo
  b += al256((size_t)density_splits(v, (long)npo * v) * v * v * 16);  // density partials
  b += heev_ws_bytes(v);
  return b;
}

lrcc_status fns_run(lrcc_handle h, int o, int v, int nchol, const double* eps, const void* Lov,
                    int ncomp, const void* Aov, const void* Avv, const void* Aoo, double omega,
                    double threshold, double* occ, void* B, double* eps_new, int* keep,
                    void* gamma, double* hbar_out, void* ws, lrcc_fns_info* info) {
  hipStream_t st = h->stream;
  const size_t o2v2 = (size_t)o * o * v * v, npo = (size_t)o * (o - 1) / 2;
  const long ov = (long)o * v, v2 = (long)v * v;
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += al256(bytes);
    return q;
  };
  double2* G = reinterpret_cast<double2*>(take(o2v2 * 16));
  double2* t = reinterpret_cast<double2*>(take(o2v2 * 16));
  double2* Y = ncomp ? reinterpret_cast<double2*>(take(o2v2 * 16)) : nullptr;
  double2* Q = ncomp ? reinterpret_cast<double2*>(take(npo * v2 * 16)) : nullptr;
  double2* T1 = reinterpret_cast<double2*>(take((size_t)ov * 16));
  double2* Gm = reinterpret_cast<double2*>(take((size_t)v2 * 16));
  double* hb = reinterpret_cast<double*>(take((size_t)(o + v) * 8));
  double* nocc = reinterpret_cast<double*>(take((size_t)v * 8));
  int* otab = reinterpret_cast<int*>(take(npo * 4 + 4));
  int* perm = reinterpret_cast<int*>(take((size_t)v * 4));
  double2* Vt = reinterpret_cast<double2*>(take((size_t)v2 * 16));
  double2* S = reinterpret_cast<double2*>(take((size_t)v2 * 16));
  double2* Ft = reinterpret_cast<double2*>(take((size_t)v2 * 16));
  double2* Z = reinterpret_cast<double2*>(take((size_t)v2 * 16));
  void* hws = take(heev_ws_bytes(v));
  double* hpart = reinterpret_cast<double*>(take((size_t)(o + v) * NSEG * 8));
  const long Kd = (long)npo * v;
  const int nsplit = density_splits(v, Kd);
  double2* Pd = reinterpret_cast<double2*>(take((size_t)nsplit * v2 * 16));
  double2* Atr = reinterpret_cast<double2*>(take((size_t)o * o * 16));

  if (!h->rb) {
    if (rocblas_create_handle(reinterpret_cast<rocblas_handle*>(&h->rb)) !=
        rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_create_handle failed");
  }
  rocblas_handle rb = static_cast<rocblas_handle>(h->rb);
  if (rocblas_set_stream(rb, st) != rocblas_status_success)
    return fail(h, LRCC_ERR_DEVICE, "rocblas_set_stream failed");
  const rocblas_operation N = rocblas_operation_none, T = rocblas_operation_transpose,
                          C = rocblas_operation_conjugate_transpose;
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  auto blas = [&](rocblas_status s) -> lrcc_status {
    return s == rocblas_status_success ? LRCC_OK
                                       : fail(h, LRCC_ERR_DEVICE, "rocblas_zgemm failed");
  };
  lrcc_status s;
  const dim3 tb(TT * TR);
  const int ntile = (v + TT - 1) / TT;

  // 1-3: amplitudes and dressed diagonals
  if (o == 0) {
    // no occupied spinors: no amplitudes, hbar = eps, a zero density
  } else if (nchol > 0) {
    // blocks i < j only: row block i against column blocks j > i, column-major
    // C^c((jb), a) = sum_P L^c((jb), P) L^c((ia), P) with L^c (ov x nchol, ld ov)
    const double2* L = static_cast<const double2*>(Lov);
    for (int i = 0; i + 1 < o; ++i) {
      s = blas(zgemm(rb, N, T, (long)(o - 1 - i) * v, v, nchol, one, L + (long)(i + 1) * v, ov,
                     L + (long)i * v, ov, zero, G + (long)i * v * ov + (long)(i + 1) * v, ov));
      if (s != LRCC_OK) return s;
    }
  } else {
    LRCC_HIP(h, fill_zero(G, o2v2 * 16, st));
  }
  if (o > 0) {
    hipLaunchKernelGGL(k_fns_t, dim3(ntile * ntile, o * o), tb, 0, st, o, v, G, eps, t);
    LRCC_HIP(h, hipGetLastError());
  }
  hipLaunchKernelGGL(k_fns_hbar, dim3(o + v, NSEG), dim3(HB), 0, st, o, v, t, eps, hpart);
  LRCC_HIP(h, hipGetLastError());
  hipLaunchKernelGGL(k_fns_hbar_fin, dim3((o + v + 255) / 256), dim3(256), 0, st, o, v, hpart,
                     eps, hb);
  LRCC_HIP(h, hipGetLastError());
  if (npo > 0) {
    hipLaunchKernelGGL(k_fns_pairs, dim3(o), dim3(64), 0, st, o, otab);
    LRCC_HIP(h, hipGetLastError());
  }

  // 4-7: perturbed amplitudes and the averaged density
  LRCC_HIP(h, fill_zero(Gm, (size_t)v2 * 16, st));
  const double2 wgt = make_double2(1.0 / (ncomp > 0 ? ncomp : 1), 0.0);
  double2* Xp = G;  // G is dead once t is formed
  for (int x = 0; x < (o > 0 ? ncomp : 0); ++x) {
    const double2* avv = static_cast<const double2*>(Avv) + (size_t)x * v2;
    const double2* aoo = static_cast<const double2*>(Aoo) + (size_t)x * o * o;
    const double2* aov = static_cast<const double2*>(Aov) + (size_t)x * ov;
    // column-major X'^c (v x o^2 v): X'^c(a, (ijc)) = sum_e A^c(e, a) t^c(e, (ijc)),
    // for the rows i < j only (per i, the rows (i, j > i, c) are contiguous)
    for (int i = 0; i + 1 < o; ++i) {
      const long r0 = ((long)i * o + i + 1) * v;
      s = blas(zgemm(rb, T, N, v, (long)(o - 1 - i) * v, v, one, avv, v, t + r0 * v, v, zero,
                     Xp + r0 * v, v));
      if (s != LRCC_OK) return s;
    }
    // Y^c (o v^2 x o) = t^c (o v^2 x o) * A_oo (o x o), A_oo through a
    // transposed copy (a plain NN product)
    hipLaunchKernelGGL(k_tr_small, dim3((o * o + 255) / 256), dim3(256), 0, st, o, aoo, Atr);
    LRCC_HIP(h, hipGetLastError());
    s = blas(zgemm(rb, N, N, (long)o * v2, o, o, one, t, (long)o * v2, Atr, o, zero, Y,
                   (long)o * v2));
    if (s != LRCC_OK) return s;
    if (npo > 0) {
      hipLaunchKernelGGL(k_fns_pert, dim3(ntile * ntile, (int)npo), tb, 0, st, o, v, otab, Xp, Y,
                         hb, omega, Q);
      LRCC_HIP(h, hipGetLastError());
      // Gm^c += Q^c^H Q^c with Q^c (npo v x v, ld npo v), K split into
      // nsplit chunks (partials Pd, summed in order)
      const long Kc = (Kd + nsplit - 1) / nsplit, Kl = Kd - (nsplit - 1) * Kc;
      if (nsplit > 1) {
        s = blas(zgemm_sb(rb, C, N, v, v, Kc, one, Q, Kd, Kc, Q, Kd, Kc, zero, Pd, v, v2,
                          nsplit - 1));
        if (s != LRCC_OK) return s;
      }
      s = blas(zgemm(rb, C, N, v, v, Kl, one, Q + (nsplit - 1) * Kc, Kd, Q + (nsplit - 1) * Kc,
                     Kd, zero, Pd + (long)(nsplit - 1) * v2, v));
      if (s != LRCC_OK) return s;
      hipLaunchKernelGGL(k_sum_parts, dim3((int)((v2 + 255) / 256)), dim3(256), 0, st, v2,
                         nsplit, Pd, wgt.x, Gm);
      LRCC_HIP(h, hipGetLastError());
    }
    hipLaunchKernelGGL(k_fns_t1, dim3((int)((ov + 255) / 256)), dim3(256), 0, st, o, v, aov, hb,
                       omega, T1);
    LRCC_HIP(h, hipGetLastError());
    s = blas(zgemm(rb, C, N, v, v, o, wgt, T1, o, T1, o, one, Gm, v));
    if (s != LRCC_OK) return s;
  }

  // 8: natural spinors, ordered by descending |n|
  int sweeps1 = 0, sweeps2 = 0;
  LRCC_HIP(h, heev_run(v, Gm, 1, nocc, nullptr, 0, hws, perm, &sweeps1, st));
  std::vector<double> hn(v);
  LRCC_HIP(h, hipMemcpyAsync(hn.data(), nocc, (size_t)v * 8, hipMemcpyDeviceToHost, st));
  LRCC_HIP(h, hipStreamSynchronize(st));
  int k = 0;
  while (k < v && std::fabs(hn[k]) > threshold) ++k;
  *keep = k;
  if (occ) LRCC_HIP(h, hipMemcpyAsync(occ, nocc, (size_t)v * 8, hipMemcpyDeviceToDevice, st));
  if (gamma) LRCC_HIP(h, hipMemcpyAsync(gamma, Gm, (size_t)v2 * 16, hipMemcpyDeviceToDevice, st));
  if (hbar_out)
    LRCC_HIP(h, hipMemcpyAsync(hbar_out, hb, (size_t)(o + v) * 8, hipMemcpyDeviceToDevice, st));

  // 9-11: truncated, semicanonical basis
  if (k > 0) {
    LRCC_HIP(h, gather_cols(v, k, heev_vectors(hws, v), perm, Vt, eps + o, S, st));
    // Ft^c (k x k) = S^c Vt^c^H, with S^c, Vt^c (k x v, ld k)
    s = blas(zgemm(rb, N, C, k, k, v, one, S, k, Vt, k, zero, Ft, k));
    if (s != LRCC_OK) return s;
    LRCC_HIP(h, heev_run(k, Ft, 0, eps_new, Z, k, hws, nullptr, &sweeps2, st));
    // B^c (k x v) = Z^c (k x k) Vt^c (k x v)
    s = blas(zgemm(rb, N, N, k, v, k, one, Z, k, Vt, k, zero, static_cast<double2*>(B), k));
    if (s != LRCC_OK) return s;
  }
  if (info) {
    info->sweeps_density = sweeps1;
    info->sweeps_fock = sweeps2;
  }
  LRCC_HIP(h, hipStreamSynchronize(st));
  return LRCC_OK;
}

// Vectors and dipole block in the kept basis: Lt^P = B^H L^P B (one product
// T = L B over all P, then a strided-batched B^H T^P) and
// mu_t = mu conj(B) (the dipole's virtual index is a bra index).
size_t fns_transform_ws_bytes(int v, int k, int nchol) {
  return al256((size_t)nchol * v * k * 16) + al256((size_t)v * k * 16);
}

lrcc_status fns_transform(lrcc_handle h, int v, int k, int nchol, int nrow, const void* B,
                          const void* L, const void* mu, void* Lt, void* mut, void* ws) {
  if (v == 0 || k == 0) return LRCC_OK;
  if (!h->rb) {
    if (rocblas_create_handle(reinterpret_cast<rocblas_handle*>(&h->rb)) !=
        rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_create_handle failed");
  }
  rocblas_handle rb = static_cast<rocblas_handle>(h->rb);
  if (rocblas_set_stream(rb, h->stream) != rocblas_status_success)
    return fail(h, LRCC_ERR_DEVICE, "rocblas_set_stream failed");
  const rocblas_operation N = rocblas_operation_none, C = rocblas_operation_conjugate_transpose;
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  const double2* Bp = static_cast<const double2*>(B);
  if (nchol > 0 && L && Lt) {
    double2* T = static_cast<double2*>(ws);
    // T = L B for all P at once: rows (P, a) of L times B; column-major
    // T^c (k x nchol v) = B^c (k x v) L^c (v x nchol v)
    if (zgemm(rb, N, N, k, (long)nchol * v, v, one, Bp, k, static_cast<const double2*>(L), v,
              zero, T, k) != rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_zgemm failed");
    // Lt^c (k x k) = T^c (k x v) (B^c)^H (v x k), per P
    if (zgemm_sb(rb, N, C, k, k, v, one, T, k, (long)v * k, Bp, k, 0, zero,
                 static_cast<double2*>(Lt), k, (long)k * k, nchol) != rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_zgemm_strided_batched failed");
  }
  if (nrow > 0 && mu && mut) {
    double2* Bc = reinterpret_cast<double2*>(static_cast<char*>(ws) +
                                             al256((size_t)nchol * v * k * 16));
    const long nb = (long)v * k;
    hipLaunchKernelGGL(k_conj_copy, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, h->stream,
                       nb, Bp, Bc);
    LRCC_HIP(h, hipGetLastError());
    // mu_t^c (k x nrow) = conj(B)^c (k x v) mu^c (v x nrow)
    if (zgemm(rb, N, N, k, nrow, v, one, Bc, k, static_cast<const double2*>(mu), v, zero,
              static_cast<double2*>(mut), k) != rocblas_status_success)
      return fail(h, LRCC_ERR_DEVICE, "rocblas_zgemm failed");
  }
  return LRCC_OK;
}

}  // namespace lrcc
