// Hole-hole ladder of the doubles-doubles Jacobian (model extension):
//   sigma_ij^ab += sum_{k,l} <kl||ij> X_kl^ab,   <kl|ij> = sum_P L^P_ki L^P_lj
// over occupied-occupied Cholesky vectors, the unrestricted k, l sum taken
// literally as for the particle-particle ladder.  The integral has no
// particle index, so it is formed explicitly (the paper builds integrals with
// at most two particle indices, Sec. 3) as the packed-pair matrix
//   W[(ij), (kl)] = 2 <kl||ij>   (npo x npo complex, the 2 for k < l only),
// and applied per block pair and right-hand side as a small complex GEMM on
// the block layout: sigma[bp][r npo + ij][s] += sum_kl W[ij][kl] X[bp][r npo + kl][s].
// Its cost is npo^2 npv per right-hand side against the ladder's npo npv^2.
#include "internal.hpp"

namespace lrcc {

namespace {

__device__ inline double2 load_c(const void* p, lrcc_dtype dt, size_t i) {
  if (dt == LRCC_C128) return static_cast<const double2*>(p)[i];
  const float2 f = static_cast<const float2*>(p)[i];
  return make_double2(f.x, f.y);
}

// One thread per (ij, kl).  form L_TRANS builds W from the transposed
// vectors (L^P)^T, which gives W^T (the left-hand solve's operator).
__global__ void k_hh_w(const void* __restrict__ Loo, lrcc_dtype dt, int o, int nchol, long npo,
                       const int* __restrict__ otab, int form, double scale,
                       double2* __restrict__ W) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= npo * npo) return;
  const int ij = (int)(e / npo), kl = (int)(e % npo);
  const int i = otab[ij] >> 16, j = otab[ij] & 0xffff;
  const int k = otab[kl] >> 16, l = otab[kl] & 0xffff;
  // element (p, q) of (L^P) or its transpose
  auto el = [&](int P, int p, int q) {
    const size_t idx = form == L_TRANS ? ((size_t)P * o + q) * o + p : ((size_t)P * o + p) * o + q;
    return load_c(Loo, dt, idx);
  };
  double re = 0, im = 0;
  for (int P = 0; P < nchol; ++P) {
    const double2 ki = el(P, k, i), lj = el(P, l, j), kj = el(P, k, j), li = el(P, l, i);
    re += (ki.x * lj.x - ki.y * lj.y) - (kj.x * li.x - kj.y * li.y);
    im += (ki.x * lj.y + ki.y * lj.x) - (kj.x * li.y + kj.y * li.x);
  }
  W[e] = make_double2(scale * re, scale * im);
}

// Sb += W X on the block layout.  Workgroup: (block pair, right-hand side,
// 16 rows ij); thread: slot s = tid % 64 and rows 16 tile + 4 (tid / 64) + t.
// K (the pair kl) in steps of 16 through LDS.
constexpr int HT = 16;
__global__ __launch_bounds__(256) void k_hh_apply(const double2* __restrict__ W, long npo,
                                                  long Mp, long plane,
                                                  const double* __restrict__ Xb,
                                                  double* __restrict__ Sb) {
  __shared__ double2 wt[HT][HT + 1];
  __shared__ double2 xt[HT][NS];
  const int bp = blockIdx.x, r = blockIdx.y, tile = blockIdx.z;
  const int s = threadIdx.x % NS, g = threadIdx.x / NS;
  const size_t base = ((size_t)bp * Mp + (size_t)r * npo) * NS;
  double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  for (long k0 = 0; k0 < npo; k0 += HT) {
    __syncthreads();
    {  // W tile: rows 16 tile .. +15, columns k0 .. k0+15 (zero outside)
      const int rr = threadIdx.x / HT, cc = threadIdx.x % HT;
      const long row = (long)tile * HT + rr, col = k0 + cc;
      wt[rr][cc] = row < npo && col < npo ? W[row * npo + col] : make_double2(0, 0);
    }
#pragma unroll
    for (int q = 0; q < HT * NS / 256; ++q) {  // X tile: rows kl = k0 .. k0+15
      const int e = q * 256 + threadIdx.x, kk = e / NS, ss = e % NS;
      double xr = 0, xi = 0;
      if (k0 + kk < npo) {
        const size_t a = base + (size_t)(k0 + kk) * NS + ss;
        xr = Xb[a];
        xi = Xb[a + plane];
      }
      xt[kk][ss] = make_double2(xr, xi);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < HT; ++kk) {
      const double2 x = xt[kk][s];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 w = wt[4 * g + t][kk];
        ar[t] += w.x * x.x - w.y * x.y;
        ai[t] += w.x * x.y + w.y * x.x;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const long ij = (long)tile * HT + 4 * g + t;
    if (ij >= npo) continue;
    const size_t a = base + (size_t)ij * NS + s;
    Sb[a] += ar[t];
    Sb[a + plane] += ai[t];
  }
}

// otab[p] = (i << 16) | j for the packed occupied pair p = (i, j), i < j.
__global__ void k_pair_table(int o, int* __restrict__ otab) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= o * o) return;
  const int i = e / o, j = e % o;
  if (i < j) otab[i * (2 * o - i - 1) / 2 + (j - i - 1)] = (i << 16) | j;
}

}  // namespace

hipError_t hh_pair_table(int o, int* otab, hipStream_t st) {
  if (o < 2) return hipSuccess;
  hipLaunchKernelGGL(k_pair_table, dim3((unsigned)((o * o + 255) / 256)), dim3(256), 0, st, o,
                     otab);
  return hipGetLastError();
}

hipError_t hh_build_w(const void* Loo, lrcc_dtype dt, int o, int nchol, const int* otab,
                      LForm form, double scale, double2* W, hipStream_t st) {
  const long npo = npair(o), n = npo * npo;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hh_w, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Loo, dt, o,
                     nchol, npo, otab, (int)form, scale, W);
  return hipGetLastError();
}

hipError_t hh_apply(const double2* W, const Geom& g, const double* Xb, double* Sb,
                    hipStream_t st) {
  if (g.npo == 0 || g.nbp == 0 || g.nrhs == 0) return hipSuccess;
  if (g.nrhs > 65535 || (g.npo + HT - 1) / HT > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)g.nbp, (unsigned)g.nrhs, (unsigned)((g.npo + HT - 1) / HT));
  hipLaunchKernelGGL(k_hh_apply, grid, dim3(256), 0, st, W, g.npo, g.Mp, g.xb_plane(), Xb, Sb);
  return hipGetLastError();
}

}  // namespace lrcc
