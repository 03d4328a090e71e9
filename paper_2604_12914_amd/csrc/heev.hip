// Hermitian eigensolver by two-sided Jacobi rotations in parallel
// round-robin order, for the natural-spinor diagonalisation and the
// semicanonicalisation of the truncated Fock block (Sec. 2.3).
//
// A sweep visits every index pair once in m - 1 rounds (m = n rounded up to
// even; the circle method: in round k index m-1 pairs with k and every other
// r pairs with (2k - r) mod (m-1)).  The pairs of one round are disjoint, so
// their 2x2 rotations combine into one unitary J and a round is one launch,
// A <- J^H A J and V <- V J, out of place: a thread updates one 2x2 block
// of A (its row pair by its column pair, every element read once) or one
// row of V on a column pair, recomputing the two rotations it needs from
// the old A (a handful of flops), so no separate parameter pass is needed.
//
// For the pair p < q with a = A_pp, d = A_qq, b = A_pq = |b| e^{i phi}:
//   tau = (d - a) / (2|b|),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2),   s = t c,
//   J_pp = J_qq = c,  J_pq = s e^{i phi},  J_qp = -s e^{-i phi},
// the complex form of the classical Jacobi rotation (a phase that makes the
// coupling real, the real rotation, the phase undone); it zeroes A_pq.
//
// After each sweep one block sums the squared off-diagonal and total
// magnitudes; the host stops one sweep after the off-diagonal part falls
// below 1e-14 of the matrix in Frobenius norm (the extra sweep takes it to
// rounding level), or after a sweep cap.  Eigenvalues are the final
// diagonal; a sort kernel orders them (ascending, or by descending
// magnitude) and a gather kernel permutes the eigenvector columns.
#include <cmath>
#include <utility>

#include "internal.hpp"

namespace lrcc {

namespace {

// Pair s of round k (0 <= s < m/2), returned ordered lo < hi.
__device__ inline void rr_pair(int s, int k, int m, int& lo, int& hi) {
  const int mm = m - 1;
  int p, q;
  if (s == 0) {
    p = k;
    q = mm;
  } else {
    p = (k + s) % mm;
    q = (k - s + mm) % mm;
  }
  lo = min(p, q);
  hi = max(p, q);
}

// The rotation of pair (lo, hi) as a 2x2 block in (lo, hi) coordinates:
// J = [[c, s e^{i phi}], [-s e^{-i phi}, c]]; the identity when hi is the
// padding index or the coupling vanishes.
struct Rot2 {
  double c;
  double2 up;  // J_lo,hi
  double2 dn;  // J_hi,lo
};

__device__ inline Rot2 rotation(const double2* __restrict__ A, int n, int lo, int hi) {
  Rot2 r{1.0, make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  if (hi >= n) return r;
  const double a = A[(long)lo * n + lo].x, d = A[(long)hi * n + hi].x;
  const double2 b = A[(long)lo * n + hi];
  const double ab = hypot(b.x, b.y);
  if (!(ab > 0.0)) return r;
  const double tau = (d - a) / (2.0 * ab);
  double t;
  if (fabs(tau) > 1e150)
    t = 0.5 / tau;
  else
    t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
  const double px = b.x / ab, py = b.y / ab;  // e^{i phi}
  r.c = c;
  r.up = make_double2(s * px, s * py);
  r.dn = make_double2(-s * px, s * py);  // -s e^{-i phi}
  return r;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 rscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

// One round.  Threads [0, P^2): the 2x2 block of A on row pair sr and column
// pair sc, A2 = J_r^H A J_c (each element of A read once); threads
// [P^2, P^2 + n P): row r of V on column pair sc, V2 = V J_c.  P = m / 2.
__global__ __launch_bounds__(256) void k_jac_round(int n, int m, int k,
                                                   const double2* __restrict__ A,
                                                   double2* __restrict__ A2,
                                                   const double2* __restrict__ V,
                                                   double2* __restrict__ V2) {
  const int P = m / 2;
  const long na = (long)P * P;
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= na + (long)n * P) return;
  int sr, sc, r = -1;
  if (e < na) {
    sr = (int)(e / P);
    sc = (int)(e % P);
  } else {
    e -= na;
    r = (int)(e / P);
    sc = (int)(e % P);
    sr = 0;
  }
  int lc, hc;
  rr_pair(sc, k, m, lc, hc);
  const Rot2 jc = rotation(A, n, lc, hc);
  const bool hcv = hc < n;
  if (r >= 0) {  // V2[r][lc, hc] = V[r][lc, hc] J_c
    const double2 x0 = V[(long)r * n + lc];
    const double2 x1 = hcv ? V[(long)r * n + hc] : make_double2(0.0, 0.0);
    V2[(long)r * n + lc] = cadd(rscale(jc.c, x0), cmul(x1, jc.dn));
    if (hcv) V2[(long)r * n + hc] = cadd(cmul(x0, jc.up), rscale(jc.c, x1));
    return;
  }
  int lr, hr;
  rr_pair(sr, k, m, lr, hr);
  const Rot2 jr = rotation(A, n, lr, hr);
  const bool hrv = hr < n;
  const double2 zero = make_double2(0.0, 0.0);
  const double2 a00 = A[(long)lr * n + lc];
  const double2 a01 = hcv ? A[(long)lr * n + hc] : zero;
  const double2 a10 = hrv ? A[(long)hr * n + lc] : zero;
  const double2 a11 = (hrv && hcv) ? A[(long)hr * n + hc] : zero;
  // B = A_blk J_c
  const double2 b00 = cadd(rscale(jc.c, a00), cmul(a01, jc.dn));
  const double2 b01 = cadd(cmul(a00, jc.up), rscale(jc.c, a01));
  const double2 b10 = cadd(rscale(jc.c, a10), cmul(a11, jc.dn));
  const double2 b11 = cadd(cmul(a10, jc.up), rscale(jc.c, a11));
  // A2 = J_r^H B: row lo = c B0 + conj(J_hi,lo) B1, row hi = conj(J_lo,hi) B0 + c B1
  A2[(long)lr * n + lc] = cadd(rscale(jr.c, b00), cmulc(jr.dn, b10));
  if (hcv) A2[(long)lr * n + hc] = cadd(rscale(jr.c, b01), cmulc(jr.dn, b11));
  if (hrv) {
    A2[(long)hr * n + lc] = cadd(cmulc(jr.up, b00), rscale(jr.c, b10));
    if (hcv) A2[(long)hr * n + hc] = cadd(cmulc(jr.up, b01), rscale(jr.c, b11));
  }
}

__global__ void k_jac_eye(int n, double2* __restrict__ V) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  V[e] = make_double2((e / n) == (e % n) ? 1.0 : 0.0, 0.0);
}

constexpr int RB = 1024;
// red[0] = sum_{r != c} |A_rc|^2, red[1] = sum |A_rc|^2 (fixed order).
__global__ __launch_bounds__(RB) void k_jac_norms(int n, const double2* __restrict__ A,
                                                  double* __restrict__ red) {
  __shared__ double so[RB], st[RB];
  double off = 0.0, tot = 0.0;
  const long nn = (long)n * n;
  for (long e = threadIdx.x; e < nn; e += RB) {
    const double2 x = A[e];
    const double q = x.x * x.x + x.y * x.y;
    tot += q;
    if (e / n != e % n) off += q;
  }
  so[threadIdx.x] = off;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      st[threadIdx.x] += st[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[0] = so[0];
    red[1] = st[0];
  }
}

// Sort key: ascending value (mode 0) or descending magnitude (mode 1); a
// value that is not a number sorts last, so the keys are totally ordered
// and every rank below is taken exactly once.
__device__ inline double sort_key(double x, int mode) {
  if (x != x) return INFINITY;
  return mode ? -fabs(x) : x;
}

// rank of each diagonal value; w[rank] = value, perm[rank] = index.
// Ties keep index order.
__global__ void k_jac_sort(int n, const double2* __restrict__ A, int mode,
                           double* __restrict__ w, int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double vi = A[(long)i * n + i].x;
  const double ki = sort_key(vi, mode);
  int rank = 0;
  for (int j = 0; j < n; ++j) {
    const double kj = sort_key(A[(long)j * n + j].x, mode);
    rank += (kj < ki) || (kj == ki && j < i);
  }
  w[rank] = vi;
  perm[rank] = i;
}

// Out[r][k] = V[r][perm[k]] for k < ncol (row stride ncol); when scale is
// given, Sout[r][k] = scale[r] * Out[r][k] as well.
__global__ void k_gather_cols(int n, int ncol, const double2* __restrict__ V,
                              const int* __restrict__ perm, double2* __restrict__ Out,
                              const double* __restrict__ scale, double2* __restrict__ Sout) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * ncol) return;
  const int r = (int)(e / ncol), k = (int)(e % ncol);
  const double2 x = V[(long)r * n + perm[k]];
  Out[e] = x;
  if (Sout) Sout[e] = make_double2(scale[r] * x.x, scale[r] * x.y);
}

}  // namespace

size_t heev_ws_bytes(int n) {
  const size_t nn = (size_t)n * n;
  return 4 * nn * sizeof(double2) + 256 + ((size_t)n * sizeof(int) + 255) / 256 * 256;
}

hipError_t heev_run(int n, const void* A, int mode, double* w, void* Vout, int ncol_out,
                    void* ws, int* perm_out, int* sweeps, hipStream_t st) {
  if (sweeps) *sweeps = 0;
  if (n <= 0) return hipSuccess;
  const size_t nn = (size_t)n * n;
  double2* a0 = static_cast<double2*>(ws);
  double2* a1 = a0 + nn;
  double2* v0 = a1 + nn;
  double2* v1 = v0 + nn;
  double* red = reinterpret_cast<double*>(v1 + nn);
  int* perm = reinterpret_cast<int*>(reinterpret_cast<char*>(red) + 256);
  hipError_t e = hipMemcpyAsync(a0, A, nn * sizeof(double2), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  const int gb = (int)((nn + 255) / 256);
  hipLaunchKernelGGL(k_jac_eye, dim3(gb), dim3(256), 0, st, n, v0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int m = n + (n & 1);
  const long nthr = (long)(m / 2) * (m / 2) + (long)n * (m / 2);
  const int g2 = (int)((nthr + 255) / 256);
  constexpr int MAX_SWEEPS = 60;
  bool last = false;
  int sw = 0;
  for (; sw < MAX_SWEEPS; ++sw) {
    if (n > 1) {
      for (int k = 0; k < m - 1; ++k) {
        hipLaunchKernelGGL(k_jac_round, dim3(g2), dim3(256), 0, st, n, m, k, a0, a1, v0, v1);
        std::swap(a0, a1);
        std::swap(v0, v1);
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (last) break;
    hipLaunchKernelGGL(k_jac_norms, dim3(1), dim3(RB), 0, st, n, a0, red);
    double hr[2];
    if ((e = hipMemcpyAsync(hr, red, sizeof hr, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (!(hr[0] > 1e-28 * hr[1])) last = true;  // converged (or not a number): one more sweep
    if (!(hr[1] > 0.0) || n == 1) break;        // zero matrix or a single element
  }
  if (sweeps) *sweeps = sw + 1;
  hipLaunchKernelGGL(k_jac_sort, dim3((n + 255) / 256), dim3(256), 0, st, n, a0, mode, w, perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (perm_out) {
    e = hipMemcpyAsync(perm_out, perm, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  // the final eigenvectors go to the front of the workspace's vector slot
  double2* vfin = static_cast<double2*>(ws) + 2 * nn;
  if (v0 != vfin) {
    e = hipMemcpyAsync(vfin, v0, nn * sizeof(double2), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  if (Vout && ncol_out > 0) return gather_cols(n, ncol_out, vfin, perm, Vout, nullptr, nullptr, st);
  return hipSuccess;
}

const void* heev_vectors(const void* ws, int n) {
  return static_cast<const double2*>(ws) + 2 * (size_t)n * n;
}

hipError_t gather_cols(int n, int ncol, const void* V, const int* perm, void* Out,
                       const double* scale, void* Sout, hipStream_t st) {
  const long ne = (long)n * ncol;
  if (ne <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_cols, dim3((int)((ne + 255) / 256)), dim3(256), 0, st, n, ncol,
                     static_cast<const double2*>(V), perm, static_cast<double2*>(Out), scale,
                     static_cast<double2*>(Sout));
  return hipGetLastError();
}

}  // namespace lrcc
