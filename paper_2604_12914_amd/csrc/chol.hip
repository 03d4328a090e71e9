// Pivoted (single-step) Cholesky decomposition of a Hermitian positive
// semi-definite two-electron matrix M (n x n, complex128, row-major), Sec. 3:
// vectors are added one at a time at the pivot of the largest remaining
// diagonal element until that element is at or below tau.
//
// Per vector four launches on the handle's stream, with all decisions on
// the device (nothing returns to the host until the end):
//   k_chol_pivot   one workgroup: argmax of the remaining diagonal d (the
//                  first index among equal maxima); sets `done` when the
//                  maximum is <= tau (or not a number) or the cap is reached
//   k_chol_dot     the sum over earlier vectors, sum_{q<k} L_q,i conj(L_q,p),
//                  split into vector segments (row blocks x segments fill the
//                  chip even for small n); partial sums per segment
//   k_chol_column  l_i = (M_ip - the segment sums, in order) / sqrt(d_p) and
//                  d_i -= |l_i|^2, one thread per row i
//   k_chol_advance k += 1 unless done
// Every kernel returns at once when `done` is set, so the host can launch a
// fixed number of steps and read the flag now and then.  The work is
// latency-bound: n-element passes per vector plus the O(k n) column update.
#include <algorithm>

#include "internal.hpp"

namespace lrcc {

namespace {

struct CholState {
  int count;  // vectors so far
  int done;   // nonzero: stop
  int piv;    // pivot of the vector being formed
  int pad;
  double dp;  // remaining diagonal at the pivot
};

__global__ void k_chol_init(long n, const double2* __restrict__ M, int maxv,
                            double* __restrict__ d, CholState* __restrict__ s) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) d[i] = M[i * n + i].x;
  if (i == 0) {
    s->count = 0;
    s->done = maxv <= 0;
    s->piv = -1;
    s->dp = 0;
  }
}

constexpr int PB = 1024;
__global__ __launch_bounds__(PB) void k_chol_pivot(long n, const double* __restrict__ d,
                                                   double tau, int maxv,
                                                   CholState* __restrict__ s,
                                                   int* __restrict__ pivots) {
  if (s->done) return;
  __shared__ double bv[PB];
  __shared__ long bi[PB];
  double best = -1.0;
  long bidx = -1;
  for (long i = threadIdx.x; i < n; i += PB) {
    const double x = d[i];
    if (x > best) {  // ascending i per thread: the first of equal values stays
      best = x;
      bidx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int w = PB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double ov = bv[threadIdx.x + w];
      const long oi = bi[threadIdx.x + w];
      if (oi >= 0 && (ov > bv[threadIdx.x] ||
                      (ov == bv[threadIdx.x] && (bi[threadIdx.x] < 0 || oi < bi[threadIdx.x])))) {
        bv[threadIdx.x] = ov;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = bv[0];
    if (s->count >= maxv || bi[0] < 0 || !(m > tau)) {
      s->done = 1;
    } else {
      s->piv = (int)bi[0];
      s->dp = m;
      if (pivots) pivots[s->count] = (int)bi[0];
    }
  }
}

// part[seg][i] = sum over this segment's q of L_q,i conj(L_q,p): the earlier
// vectors' contribution to the new column, split over the vectors so that
// small n still fills the chip (grid: row blocks x segments).
__global__ void k_chol_dot(long n, int nseg, const double2* __restrict__ L,
                           const CholState* __restrict__ s, double2* __restrict__ part) {
  if (s->done) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = s->count, seg = blockIdx.y;
  const long p = s->piv;
  const int q0 = (int)((long)k * seg / nseg), q1 = (int)((long)k * (seg + 1) / nseg);
  double2 acc = make_double2(0.0, 0.0);
  for (int q = q0; q < q1; ++q) {
    const double2 a = L[(size_t)q * n + i], b = L[(size_t)q * n + p];
    acc.x += a.x * b.x + a.y * b.y;  // a conj(b)
    acc.y += a.y * b.x - a.x * b.y;
  }
  part[(size_t)seg * n + i] = acc;
}

__global__ void k_chol_column(long n, int nseg, const double2* __restrict__ M,
                              const double2* __restrict__ part, double2* __restrict__ L,
                              double* __restrict__ d, const CholState* __restrict__ s) {
  if (s->done) return;
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = s->count;
  const long p = s->piv;
  double2 acc = M[i * n + p];
  for (int seg = 0; seg < nseg; ++seg) {  // fixed order
    const double2 x = part[(size_t)seg * n + i];
    acc.x -= x.x;
    acc.y -= x.y;
  }
  const double r = sqrt(s->dp);
  const double2 l = make_double2(acc.x / r, acc.y / r);
  L[(size_t)k * n + i] = l;
  d[i] -= l.x * l.x + l.y * l.y;
}

__global__ void k_chol_advance(CholState* s) {
  if (!s->done) s->count += 1;
}

}  // namespace

// Vector segments of the column update: enough row-block x segment
// workgroups to fill the chip, at most 32.
int chol_segments(long n) {
  const long rb = (n + 255) / 256;
  return (int)std::max(1L, std::min(32L, (1024 + rb - 1) / std::max(rb, 1L)));
}

size_t chol_state_bytes(long n) {
  return roundup(n * 8, 256) + roundup(sizeof(CholState), 256) +
         (size_t)chol_segments(n) * n * sizeof(double2);
}

// Launch-and-check loop: `step` vectors per batch, the flag read between
// batches.  ws: chol_state_bytes(n) bytes of device workspace.
hipError_t chol_run(long n, const void* M, double tau, int maxv, void* L, int* pivots, void* ws,
                    int* nvec, hipStream_t st) {
  double* d = static_cast<double*>(ws);
  CholState* s = reinterpret_cast<CholState*>(static_cast<char*>(ws) + roundup(n * 8, 256));
  double2* part = reinterpret_cast<double2*>(static_cast<char*>(ws) + roundup(n * 8, 256) +
                                             roundup(sizeof(CholState), 256));
  const int nseg = chol_segments(n);
  const double2* Mc = static_cast<const double2*>(M);
  double2* Lc = static_cast<double2*>(L);
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_chol_init, dim3(g), dim3(256), 0, st, n, Mc, maxv, d, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  CholState h{0, maxv <= 0, -1, 0, 0};
  constexpr int STEP = 32;
  for (int k0 = 0; k0 < maxv && !h.done; k0 += STEP) {
    for (int k = k0; k < std::min(maxv, k0 + STEP); ++k) {
      hipLaunchKernelGGL(k_chol_pivot, dim3(1), dim3(PB), 0, st, n, d, tau, maxv, s, pivots);
      hipLaunchKernelGGL(k_chol_dot, dim3(g, nseg), dim3(256), 0, st, n, nseg, Lc, s, part);
      hipLaunchKernelGGL(k_chol_column, dim3(g), dim3(256), 0, st, n, nseg, Mc, part, Lc, d, s);
      hipLaunchKernelGGL(k_chol_advance, dim3(1), dim3(1), 0, st, s);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&h, s, sizeof(CholState), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
  }
  *nvec = h.count;
  return hipSuccess;
}

}  // namespace lrcc
