// Model LR-CCSD response solve on the device (paper Sec. 2.2):
//   (A - w) X = -xi,  (A X) = D o X + sigma(X),  D_ij^ab = e_a + e_b - e_i - e_j,
//   xi_ij^ab = mu_ia mu_jb - mu_ib mu_ja,  alpha_xy(w) = -<xi_x | X_y(w)>.
//
// Everything between the ladder launches stays on the device in FP64 and in
// the block-pair layout of the ladder kernel (no packing per iteration):
//   k_resid   one streaming pass per iteration: R = b - (D - w) X - sigma,
//             e = R / (D - w) (denominators rebuilt from the orbital
//             energies, never stored), X~ = X + e into the DIIS ring, and per
//             right-hand side the partial sums |R|^2, |b|^2 and <e_j|e>;
//   k_diis    one workgroup per right-hand side: fixed-order reduction of the
//             partials, convergence test, DIIS matrix update, bordered solve;
//   k_extrap  X = sum_k c_k X~_k.
// The host reads back only the per-RHS active flags and residuals.
//
// Reduced precision (FP32 / BF16X3 ladder): iterative refinement.  The outer
// residual r = -xi - (A - w) x uses the FP64 ladder; the correction solves
// (A - w) d = r with the reduced-precision ladder by the same Jacobi + DIIS
// to a loose relative tolerance; x += d.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <memory>
#include <vector>

#include "internal.hpp"

namespace lrcc {

namespace {

constexpr int MAXD = 12;  // largest DIIS subspace
constexpr int RB = 256;   // threads of the streaming kernels

struct Dims {
  long Mp, npo, plane;  // padded rows, occupied pairs, elements per plane
  int nbp, v, o;
  long per_rhs;         // elements of one RHS over all block pairs: nbp*npo*64
};

// Element f of right-hand side r -> global index in the block layout; also
// its virtual pair (a, b) and occupied pair (i, j).
struct Elem {
  long g;
  int a, b, i, j;
  bool live;
};

__device__ __forceinline__ Elem locate(const Dims& d, int r, long f, const int* tab,
                                       const int* otab) {
  Elem e;
  const int s = f & 63;
  const long ml = (f >> 6) % d.npo;
  const int bp = (int)((f >> 6) / d.npo);
  e.g = (((long)bp * d.Mp) + (long)r * d.npo + ml) * 64 + s;
  const int AB = tab[bp], IJ = otab[ml];
  e.a = (AB >> 16) * TB + (s >> 3);
  e.b = (AB & 0xffff) * TB + (s & 7);
  e.i = IJ >> 16;
  e.j = IJ & 0xffff;
  e.live = e.a < e.b && e.b < d.v;
  return e;
}

// Sum over the 64 lanes of a wavefront by lane exchanges (a fixed butterfly:
// the same order on every run); every lane receives the sum.
__device__ __forceinline__ double2 wave_sum(double2 x) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    x.x += __shfl_xor(x.x, m, 64);
    x.y += __shfl_xor(x.y, m, 64);
  }
  return x;
}

// Sum over the workgroup: wavefront sums, then one combine of the NT / 64
// wave sums through LDS (sh: at least NT / 64 entries).  Every thread
// receives the sum.
template <int NT>
__device__ __forceinline__ double2 block_sum(double2 x, double2* sh) {
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  double2 r = sh[0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) {
    r.x += sh[k].x;
    r.y += sh[k].y;
  }
  __syncthreads();
  return r;
}

// xi in block layout for every RHS r = w * ncomp + x (conj: its complex
// conjugate, the left-hand right-hand side eta).
__global__ void k_xi(Dims d, int ncomp, const double2* __restrict__ mu, const int* tab,
                     const int* otab, int conj, double* __restrict__ xi) {
  const int r = blockIdx.y;
  const double2* m = mu + (size_t)(r % ncomp) * d.o * d.v;
  for (long f = blockIdx.x * (long)RB + threadIdx.x; f < d.per_rhs; f += (long)gridDim.x * RB) {
    Elem e = locate(d, r, f, tab, otab);
    double re = 0, im = 0;
    if (e.live) {
      const double2 ia = m[e.i * d.v + e.a], jb = m[e.j * d.v + e.b];
      const double2 ib = m[e.i * d.v + e.b], ja = m[e.j * d.v + e.a];
      re = (ia.x * jb.x - ia.y * jb.y) - (ib.x * ja.x - ib.y * ja.y);
      im = (ia.x * jb.y + ia.y * jb.x) - (ib.x * ja.y + ib.y * ja.x);
    }
    xi[e.g] = re;
    xi[e.g + d.plane] = conj ? -im : im;
  }
}

__device__ __forceinline__ double denom(const Dims& d, const Elem& e, const double* eps, double w) {
  return (eps[d.o + e.a] + eps[d.o + e.b]) - (eps[e.i] + eps[e.j]) - w;
}

// x = b / (D - w), or x = 0 when zero_start.
__global__ void k_start(Dims d, const double* __restrict__ eps, const double* __restrict__ omega,
                        const int* tab, const int* otab, const int* __restrict__ active,
                        const double* __restrict__ b, double* __restrict__ x) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  const double w = omega[r];
  for (long f = blockIdx.x * (long)RB + threadIdx.x; f < d.per_rhs; f += (long)gridDim.x * RB) {
    Elem e = locate(d, r, f, tab, otab);
    double re = 0, im = 0;
    if (e.live) {
      const double D = denom(d, e, eps, w);
      re = b[e.g] / D;
      im = b[e.g + d.plane] / D;
    }
    x[e.g] = re;
    x[e.g + d.plane] = im;
  }
}

// One Jacobi + DIIS residual pass.  part layout: [r][q][chunk] double2 with
// q = 0: (|R|^2, |b|^2), q = 1 + j: <e_j | e_new> for ring slot j.
__global__ __launch_bounds__(RB) void k_resid(Dims d, const double* __restrict__ eps,
                                              const double* __restrict__ omega, const int* tab,
                                              const int* otab, const int* __restrict__ active,
                                              const unsigned* __restrict__ valid,
                                              const int* __restrict__ itp, int mdim,
                                              const double* __restrict__ b,
                                              const double* __restrict__ x,
                                              const double* __restrict__ s,
                                              double* __restrict__ xt, double* __restrict__ ev,
                                              double2* __restrict__ part) {
  __shared__ double2 sh[RB];
  const int r = blockIdx.y;
  if (!active[r]) return;
  const double w = omega[r];
  const int slot = *itp % mdim;
  const unsigned vmask = valid[r] | (1u << slot);
  const size_t hs = (size_t)2 * d.plane;  // stride between ring slots
  double rr = 0, bb = 0;
  double2 dots[MAXD];
#pragma unroll
  for (int j = 0; j < MAXD; ++j) dots[j] = make_double2(0, 0);
  for (long f = blockIdx.x * (long)RB + threadIdx.x; f < d.per_rhs; f += (long)gridDim.x * RB) {
    Elem e = locate(d, r, f, tab, otab);
    if (!e.live) {
      // dead slots of the ring stay zero (a ring shared by several
      // instances may hold another layout's values there)
      xt[slot * hs + e.g] = 0;
      xt[slot * hs + e.g + d.plane] = 0;
      ev[slot * hs + e.g] = 0;
      ev[slot * hs + e.g + d.plane] = 0;
      continue;
    }
    const double D = denom(d, e, eps, w);
    const double br = b[e.g], bi = b[e.g + d.plane];
    const double xr = x[e.g], xi = x[e.g + d.plane];
    const double Rr = br - D * xr - s[e.g], Ri = bi - D * xi - s[e.g + d.plane];
    const double er = Rr / D, ei = Ri / D;
    xt[slot * hs + e.g] = xr + er;
    xt[slot * hs + e.g + d.plane] = xi + ei;
    ev[slot * hs + e.g] = er;
    ev[slot * hs + e.g + d.plane] = ei;
    rr += Rr * Rr + Ri * Ri;
    bb += br * br + bi * bi;
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
      if (j >= mdim || !((vmask >> j) & 1u)) continue;
      double ur = er, ui = ei;
      if (j != slot) {
        ur = ev[j * hs + e.g];
        ui = ev[j * hs + e.g + d.plane];
      }
      // conj(e_j) * e_new
      dots[j].x += ur * er + ui * ei;
      dots[j].y += ur * ei - ui * er;
    }
  }
  // all 1 + mdim sums at once: wavefront sums by lane exchanges, the wave
  // sums through LDS, one barrier, then thread q adds up quantity q
  const int nq = mdim + 1;
  constexpr int NW = RB / 64;
  double2* pr = part + ((size_t)r * nq) * gridDim.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double2 t = wave_sum(make_double2(rr, bb));
  if (lane == 0) sh[wv] = t;
#pragma unroll
  for (int j = 0; j < MAXD; ++j) {
    if (j >= mdim || !((vmask >> j) & 1u)) continue;  // uniform
    t = wave_sum(dots[j]);
    if (lane == 0) sh[(1 + j) * NW + wv] = t;
  }
  __syncthreads();
  const int q = threadIdx.x;
  if (q < nq && (q == 0 || ((vmask >> (q - 1)) & 1u))) {
    double2 acc = sh[q * NW];
#pragma unroll
    for (int k = 1; k < NW; ++k) {
      acc.x += sh[q * NW + k].x;
      acc.y += sh[q * NW + k].y;
    }
    pr[(size_t)q * gridDim.x + blockIdx.x] = acc;
  }
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cdiv(double2 a, double2 b) {
  const double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

// Per RHS: reduce partials, test convergence, update the DIIS matrix and
// solve for the extrapolation coefficients.  Bmat: [r][MAXD][MAXD] double2.
__global__ void k_diis(int nchunk, int mdim, const int* __restrict__ itp, int max_iter, double tol,
                       const double2* __restrict__ part, int* __restrict__ active,
                       unsigned* __restrict__ valid, double2* __restrict__ Bmat,
                       double2* __restrict__ coef, double* __restrict__ relres) {
  __shared__ double2 sh[64];
  __shared__ double2 q[MAXD + 1];
  const int r = blockIdx.x;
  if (!active[r]) return;
  const int it = *itp, slot = it % mdim;
  const int nq = mdim + 1;
  const unsigned vmask = valid[r] | (1u << slot);
  for (int k = 0; k < nq; ++k) {
    if (k > 0 && !((vmask >> (k - 1)) & 1u)) continue;  // uniform over the block
    double2 acc = make_double2(0, 0);
    const double2* p = part + ((size_t)r * nq + k) * nchunk;
    for (int c = threadIdx.x; c < nchunk; c += 64) {
      acc.x += p[c].x;
      acc.y += p[c].y;
    }
    acc = block_sum<64>(acc, sh);
    if (threadIdx.x == 0) q[k] = acc;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double rel = sqrt(q[0].x / q[0].y);
  relres[r] = rel;
  if (rel < tol || it >= max_iter || !isfinite(rel)) {
    active[r] = 0;
    return;
  }
  double2* B = Bmat + (size_t)r * MAXD * MAXD;
  for (int j = 0; j < mdim; ++j) {
    if (!((vmask >> j) & 1u)) continue;
    B[slot * MAXD + j] = make_double2(q[1 + j].x, -q[1 + j].y);  // <e_new|e_j>
    B[j * MAXD + slot] = q[1 + j];                                // <e_j|e_new>
  }
  int idx[MAXD], k = 0;
  for (int j = 0; j < mdim; ++j)
    if ((vmask >> j) & 1u) idx[k++] = j;
  double2* c = coef + (size_t)r * MAXD;
  for (int j = 0; j < MAXD; ++j) c[j] = make_double2(0, 0);
  bool singular = false;
  double2 sol[MAXD + 1];
  if (k > 1) {
    // singularity test: Cholesky of the unit-diagonal form of B
    double dg[MAXD], G[MAXD][MAXD][2];
    double dmax = 0;
    for (int u = 0; u < k; ++u) {
      dg[u] = sqrt(B[idx[u] * MAXD + idx[u]].x);
      dmax = fmax(dmax, dg[u]);
    }
    for (int u = 0; u < k; ++u)
      for (int t = 0; t < k; ++t) {
        const double2 z = B[idx[u] * MAXD + idx[t]];
        G[u][t][0] = z.x / (dg[u] * dg[t]);
        G[u][t][1] = z.y / (dg[u] * dg[t]);
      }
    for (int u = 0; u < k && !singular; ++u) {
      double piv = G[u][u][0];
      for (int t = 0; t < u; ++t) piv -= G[u][t][0] * G[u][t][0] + G[u][t][1] * G[u][t][1];
      if (!(piv > 1e-14)) {
        singular = true;
        break;
      }
      const double l = sqrt(piv);
      G[u][u][0] = l;
      G[u][u][1] = 0;
      for (int t = u + 1; t < k; ++t) {
        // L[t][u] = (G[t][u] - sum_s L[t][s] conj(L[u][s])) / l
        double zr = G[t][u][0], zi = G[t][u][1];
        for (int s2 = 0; s2 < u; ++s2) {
          zr -= G[t][s2][0] * G[u][s2][0] + G[t][s2][1] * G[u][s2][1];
          zi -= G[t][s2][1] * G[u][s2][0] - G[t][s2][0] * G[u][s2][1];
        }
        G[t][u][0] = zr / l;
        G[t][u][1] = zi / l;
      }
    }
    if (!singular) {
      // bordered system [[B / dmax^2, 1], [1^T, 0]] [c; l] = [0; 1],
      // Gaussian elimination with partial pivoting
      const int n = k + 1;
      double2 Aa[MAXD + 1][MAXD + 2];
      for (int u = 0; u < n; ++u)
        for (int t = 0; t <= n; ++t) Aa[u][t] = make_double2(0, 0);
      for (int u = 0; u < k; ++u) {
        for (int t = 0; t < k; ++t) {
          const double2 z = B[idx[u] * MAXD + idx[t]];
          Aa[u][t] = make_double2(z.x / (dmax * dmax), z.y / (dmax * dmax));
        }
        Aa[u][k] = make_double2(1, 0);
        Aa[k][u] = make_double2(1, 0);
      }
      Aa[k][n] = make_double2(1, 0);
      for (int col = 0; col < n; ++col) {
        int p = col;
        double best = hypot(Aa[col][col].x, Aa[col][col].y);
        for (int u = col + 1; u < n; ++u) {
          const double m2 = hypot(Aa[u][col].x, Aa[u][col].y);
          if (m2 > best) {
            best = m2;
            p = u;
          }
        }
        if (!(best > 0)) {
          singular = true;
          break;
        }
        if (p != col)
          for (int t = 0; t <= n; ++t) {
            double2 tmp = Aa[col][t];
            Aa[col][t] = Aa[p][t];
            Aa[p][t] = tmp;
          }
        for (int u = col + 1; u < n; ++u) {
          const double2 f = cdiv(Aa[u][col], Aa[col][col]);
          for (int t = col; t <= n; ++t) {
            const double2 z = cmul(f, Aa[col][t]);
            Aa[u][t].x -= z.x;
            Aa[u][t].y -= z.y;
          }
        }
      }
      if (!singular) {
        for (int u = n - 1; u >= 0; --u) {
          double2 z = Aa[u][n];
          for (int t = u + 1; t < n; ++t) {
            const double2 y = cmul(Aa[u][t], sol[t]);
            z.x -= y.x;
            z.y -= y.y;
          }
          sol[u] = cdiv(z, Aa[u][u]);
        }
      }
    }
  }
  if (k <= 1 || singular) {
    c[slot] = make_double2(1, 0);
    valid[r] = 1u << slot;
  } else {
    for (int u = 0; u < k; ++u) c[idx[u]] = sol[u];
    valid[r] = vmask;
  }
}

__global__ void k_extrap(Dims d, int mdim, const int* __restrict__ active,
                         const unsigned* __restrict__ valid, const double2* __restrict__ coef,
                         const double* __restrict__ xt, double* __restrict__ x) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  const unsigned vm = valid[r];
  const double2* c = coef + (size_t)r * MAXD;
  const size_t hs = (size_t)2 * d.plane;
  for (long f = blockIdx.x * (long)RB + threadIdx.x; f < d.per_rhs; f += (long)gridDim.x * RB) {
    const int s = f & 63;
    const long ml = (f >> 6) % d.npo;
    const int bp = (int)((f >> 6) / d.npo);
    const long g = (((long)bp * d.Mp) + (long)r * d.npo + ml) * 64 + s;
    double re = 0, im = 0;
    for (int j = 0; j < mdim; ++j) {
      if (!((vm >> j) & 1u)) continue;
      const double ar = xt[j * hs + g], ai = xt[j * hs + g + d.plane];
      re += c[j].x * ar - c[j].y * ai;
      im += c[j].x * ai + c[j].y * ar;
    }
    x[g] = re;
    x[g + d.plane] = im;
  }
}

// Outer residual of the refinement: r = b0 - (D - w) x - s, and per RHS
// partial (|r|^2, |b0|^2).  x += d beforehand when add_d.
__global__ __launch_bounds__(RB) void k_outer(Dims d, const double* __restrict__ eps,
                                              const double* __restrict__ omega, const int* tab,
                                              const int* otab, const int* __restrict__ active,
                                              const double* __restrict__ b0,
                                              const double* __restrict__ x,
                                              const double* __restrict__ s,
                                              double* __restrict__ rk, double2* __restrict__ part) {
  __shared__ double2 sh[RB];
  const int r = blockIdx.y;
  if (!active[r]) return;
  const double w = omega[r];
  double rr = 0, bb = 0;
  for (long f = blockIdx.x * (long)RB + threadIdx.x; f < d.per_rhs; f += (long)gridDim.x * RB) {
    Elem e = locate(d, r, f, tab, otab);
    double Rr = 0, Ri = 0;
    if (e.live) {
      const double D = denom(d, e, eps, w);
      const double br = b0[e.g], bi = b0[e.g + d.plane];
      Rr = br - D * x[e.g] - s[e.g];
      Ri = bi - D * x[e.g + d.plane] - s[e.g + d.plane];
      rr += Rr * Rr + Ri * Ri;
      bb += br * br + bi * bi;
    }
    rk[e.g] = Rr;
    rk[e.g + d.plane] = Ri;
  }
  double2 t = block_sum<RB>(make_double2(rr, bb), sh);
  if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = t;
}

// x += d for the active right-hand sides.
__global__ void k_add(Dims d, const int* __restrict__ active, const double* __restrict__ dlt,
                      double* __restrict__ x) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  for (long f = blockIdx.x * (long)RB + threadIdx.x; f < d.per_rhs; f += (long)gridDim.x * RB) {
    const int s = f & 63;
    const long ml = (f >> 6) % d.npo;
    const int bp = (int)((f >> 6) / d.npo);
    const long g = (((long)bp * d.Mp) + (long)r * d.npo + ml) * 64 + s;
    x[g] += dlt[g];
    x[g + d.plane] += dlt[g + d.plane];
  }
}

// Partial sums of <u_r1 | w_r2> for the pairs (r1, r2) = (xi of (w, x), X of (w, y)).
__global__ __launch_bounds__(RB) void k_alpha(Dims d, int ncomp, const double* __restrict__ xi,
                                              const double* __restrict__ x,
                                              double2* __restrict__ part) {
  __shared__ double2 sh[RB];
  const int p = blockIdx.y;  // (w, xc, yc)
  const int yc = p % ncomp, xc = (p / ncomp) % ncomp, w = p / (ncomp * ncomp);
  const int r1 = w * ncomp + xc, r2 = w * ncomp + yc;
  double2 acc = make_double2(0, 0);
  for (long f = blockIdx.x * (long)RB + threadIdx.x; f < d.per_rhs; f += (long)gridDim.x * RB) {
    const int s = f & 63;
    const long ml = (f >> 6) % d.npo;
    const int bp = (int)((f >> 6) / d.npo);
    const long base = ((long)bp * d.Mp + ml) * 64 + s;
    const long g1 = base + (long)r1 * d.npo * 64, g2 = base + (long)r2 * d.npo * 64;
    const double ur = xi[g1], ui = xi[g1 + d.plane];
    const double wr = x[g2], wi = x[g2 + d.plane];
    acc.x += ur * wr + ui * wi;
    acc.y += ur * wi - ui * wr;
  }
  double2 t = block_sum<RB>(acc, sh);
  if (threadIdx.x == 0) part[(size_t)p * gridDim.x + blockIdx.x] = t;
}

// acc += s for the active right-hand sides (the reduced-precision ladder of
// a refinement correction added to the ladder of the iterate).
__global__ void k_acc(Dims d, const int* __restrict__ active, const double* __restrict__ s,
                      double* __restrict__ acc) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  for (long f = blockIdx.x * (long)RB + threadIdx.x; f < d.per_rhs; f += (long)gridDim.x * RB) {
    const int sl = f & 63;
    const long ml = (f >> 6) % d.npo;
    const int bp = (int)((f >> 6) / d.npo);
    const long g = (((long)bp * d.Mp) + (long)r * d.npo + ml) * 64 + sl;
    acc[g] += s[g];
    acc[g + d.plane] += s[g + d.plane];
  }
}

// y += x over n doubles (the ring image added to the ladder's).
__global__ void k_axpy1(long n, const double* __restrict__ x, double* __restrict__ y) {
  for (long e = blockIdx.x * (long)RB + threadIdx.x; e < n; e += (long)gridDim.x * RB)
    y[e] += x[e];
}

// x *= a over n doubles.
__global__ void k_scale(long n, double a, double* __restrict__ x) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    x[e] *= a;
}

// Advance the device-resident iteration counter (one thread).
__global__ void k_inc(int* itp) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *itp += 1;
}

// b = -a elementwise.
__global__ void k_neg(long n, const double* __restrict__ a, double* __restrict__ b) {
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB) b[i] = -a[i];
}

// Convert the two FP64 planes of the doubles to float for the reduced-
// precision ladder.
__global__ void k_to_f32(long n, const double* __restrict__ a, float* __restrict__ b) {
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB)
    b[i] = (float)a[i];
}

// The FP32 ladder's float sums back to the FP64 planes.
__global__ void k_to_f64(long n, const float* __restrict__ a, double* __restrict__ b) {
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < n; i += (long)gridDim.x * RB)
    b[i] = (double)a[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// Host driver

namespace {

// Workspace slots of one solve: 0 xi, 1 x, 2 s, 3 ring X~, 4 ring e, 5 b,
// 6 x2 (refined iterate), 7 rk, 8 small device state, 9 partials, 10 x32 and s32,
// 11 sx (ladder of the refined iterate), 12 staged FP64 vectors, 13 block-pair
// table, 14 tile order (the last three only for batched instances).
constexpr int NBUF = 15;

struct Solver {
  lrcc_handle h = nullptr;
  Buf* buf[NBUF] = {};
  Geom g;
  Dims d;
  int n = 0, ncomp = 0, nomega = 0, mdim = 0, nchunk = 0;
  const int* tab = nullptr;
  // device buffers
  double *xi = nullptr, *x = nullptr, *s = nullptr, *xt = nullptr, *ev = nullptr, *b = nullptr;
  double *omega = nullptr, *eps = nullptr, *x2 = nullptr, *rk = nullptr, *sx = nullptr;
  float* x32 = nullptr;
  float* s32 = nullptr;  // float sums of the FP32 ladder
  int *otab = nullptr, *active = nullptr, *itp = nullptr;
  int* nonherm = nullptr;  // Hermiticity flag of L (herm_check)
  const double2* W = nullptr;  // hole-hole ladder matrix (optional)
  const double2* ringM = nullptr;  // particle-hole integral matrix of the ring term (optional)
  double2 *rx = nullptr, *rs = nullptr;  // packed iterate and ring image
  double* rb = nullptr;                  // ring image in the block layout
  void* rws = nullptr;                   // ring application workspace
  unsigned* valid = nullptr;
  double2 *Bm = nullptr, *coef = nullptr, *part = nullptr;
  double* relres = nullptr;
  // host mirrors (pinned)
  int* h_active = nullptr;
  double* h_relres = nullptr;
  double2* h_part = nullptr;
  int n_sigma64 = 0, n_sigma_lp = 0, iters_max = 0;
  std::vector<int> act;  // host view of the active flags
  // per-iteration metrics (one JSON line per iteration; null: off)
  FILE* metrics = nullptr;
  const char* side = "right";
  const char* phase = "fp64";
  int sweep = 0;
  std::chrono::steady_clock::time_point t0;
  ~Solver() {
    if (h_active) (void)hipHostFree(h_active);
    if (h_relres) (void)hipHostFree(h_relres);
    if (h_part) (void)hipHostFree(h_part);
  }
};

dim3 grid_rhs(const Solver& S, int nr) { return dim3(S.nchunk, nr); }

// Geometry, workspace, right-hand sides and zeroed iterates of one solve.
// tab: the block-pair table for this nbv (device).  `ir`: reduced precision.
lrcc_status setup(Solver& S, lrcc_handle h, int o, int v, int nchol, const double* eps,
                  int ncomp, const void* mu, int nomega, const double* omegas, int mdim,
                  bool ir, const int* tab, bool conj_rhs, hipStream_t st) {
  S.h = h;
  S.n = nomega * ncomp;
  S.ncomp = ncomp;
  S.nomega = nomega;
  S.mdim = mdim;
  S.tab = tab;
  S.g = make_geom(o, v, nchol, S.n, 1);
  const Geom& g = S.g;
  S.d = Dims{g.Mp, g.npo, g.xb_plane(), g.nbp, v, o, (long)g.nbp * g.npo * 64};
  S.nchunk = (int)std::max<long>(1, std::min<long>(256, (S.d.per_rhs + 4 * RB - 1) / (4 * RB)));
  const size_t vb = (size_t)2 * S.d.plane * 8;
  size_t need[12] = {vb, vb, vb, vb * mdim, vb * mdim, vb, ir ? vb : 16, ir ? vb : 16, 0, 0,
                     ir ? vb : 16,  // x32 (f32 planes, or 4 bf16 planes: same bytes), s32
                     ir ? vb : 16};
  const size_t np_alpha = (size_t)nomega * ncomp * ncomp;
  const size_t npart = std::max((size_t)S.n * (mdim + 1), np_alpha) * S.nchunk;
  need[9] = npart * sizeof(double2);
  // small state: omega[n], eps[o+v], otab[npo], active[n], valid[n], relres[n],
  // B, coef, iteration counter
  const size_t off_om = 0, off_eps = off_om + roundup(S.n * 8, 256),
               off_ot = off_eps + roundup((o + v) * 8, 256),
               off_act = off_ot + roundup(g.npo * 4, 256), off_val = off_act + roundup(S.n * 4, 256),
               off_rel = off_val + roundup(S.n * 4, 256), off_B = off_rel + roundup(S.n * 8, 256),
               off_c = off_B + roundup((long)S.n * MAXD * MAXD * 16, 256),
               off_it = off_c + roundup((long)S.n * MAXD * 16, 256), off_nh = off_it + 256,
               end = off_nh + 256;
  need[8] = end;
  for (int k = 0; k < 12; ++k) LRCC_HIP(h, S.buf[k]->ensure(need[k]));
  S.xi = S.buf[0]->as<double>();
  S.x = S.buf[1]->as<double>();
  S.s = S.buf[2]->as<double>();
  S.xt = S.buf[3]->as<double>();
  S.ev = S.buf[4]->as<double>();
  S.b = S.buf[5]->as<double>();
  S.x2 = S.buf[6]->as<double>();
  S.rk = S.buf[7]->as<double>();
  char* sm = S.buf[8]->as<char>();
  S.omega = reinterpret_cast<double*>(sm + off_om);
  S.eps = reinterpret_cast<double*>(sm + off_eps);
  S.otab = reinterpret_cast<int*>(sm + off_ot);
  S.active = reinterpret_cast<int*>(sm + off_act);
  S.valid = reinterpret_cast<unsigned*>(sm + off_val);
  S.relres = reinterpret_cast<double*>(sm + off_rel);
  S.Bm = reinterpret_cast<double2*>(sm + off_B);
  S.coef = reinterpret_cast<double2*>(sm + off_c);
  S.itp = reinterpret_cast<int*>(sm + off_it);
  S.nonherm = reinterpret_cast<int*>(sm + off_nh);
  S.part = S.buf[9]->as<double2>();
  S.x32 = S.buf[10]->as<float>();
  S.s32 = ir ? S.x32 + S.d.plane * 2 : nullptr;
  S.sx = S.buf[11]->as<double>();

  std::vector<double> om(S.n);
  for (int w = 0; w < nomega; ++w)
    for (int x = 0; x < ncomp; ++x) om[w * ncomp + x] = omegas[w];
  std::vector<int> ot(g.npo);
  for (int i = 0, k = 0; i < o; ++i)
    for (int j = i + 1; j < o; ++j) ot[k++] = (i << 16) | j;
  LRCC_HIP(h, hipHostMalloc((void**)&S.h_active, S.n * sizeof(int), hipHostMallocDefault));
  LRCC_HIP(h, hipHostMalloc((void**)&S.h_relres, S.n * sizeof(double), hipHostMallocDefault));
  LRCC_HIP(h, hipHostMalloc((void**)&S.h_part, std::max((size_t)S.n, np_alpha) * S.nchunk *
                                                   sizeof(double2),
                            hipHostMallocDefault));
  LRCC_HIP(h, hipMemcpyAsync(S.omega, om.data(), S.n * 8, hipMemcpyHostToDevice, st));
  LRCC_HIP(h, hipMemcpyAsync(S.eps, eps, (o + v) * 8, hipMemcpyDeviceToDevice, st));
  LRCC_HIP(h, hipMemcpyAsync(S.otab, ot.data(), g.npo * 4, hipMemcpyHostToDevice, st));
  LRCC_HIP(h, hipStreamSynchronize(st));  // host vectors go out of scope below

  hipLaunchKernelGGL(k_xi, grid_rhs(S, S.n), dim3(RB), 0, st, S.d, ncomp,
                     static_cast<const double2*>(mu), tab, S.otab, (int)conj_rhs, S.xi);
  LRCC_HIP(h, hipGetLastError());
  // zero the iterates and the DIIS ring once so dead slots and pad rows hold
  // zeros (the ladder kernel reads whole block-pair rows)
  LRCC_HIP(h, fill_zero(S.x, vb, st));
  LRCC_HIP(h, fill_zero(S.xt, vb * mdim, st));
  LRCC_HIP(h, fill_zero(S.ev, vb * mdim, st));
  hipLaunchKernelGGL(k_neg, dim3((unsigned)std::min<long>((2 * S.d.plane + RB - 1) / RB, 8192)),
                     dim3(RB), 0, st, 2 * S.d.plane, (const double*)S.xi, S.b);
  LRCC_HIP(h, hipGetLastError());
  return LRCC_OK;
}

// Stage L (in the form `form`) for a ladder of precision `prec` into dst.
lrcc_status stage_for(Solver& S, const void* L, lrcc_prec prec, lrcc_cmul cmul, Buf& dst,
                      LForm form) {
  lrcc_handle h = S.h;
  Geom g = S.g;
  if (prec == LRCC_BF16X3) {
    g.ncp = (int)roundup(g.nchol, bf16x3_chunk());
    LRCC_HIP(h, dst.ensure(bf16x3_ls_bytes(g)));
    if (g.nchol > 0) LRCC_HIP(h, bf16x3_stage_L(L, LRCC_C128, g, form, dst.p, h->stream));
    return LRCC_OK;
  }
  g.ncp = (int)roundup(g.nchol, ppl_chunk(prec, cmul));
  LRCC_HIP(h, dst.ensure(ppl_ls_bytes(prec, cmul, g)));
  if (g.nchol > 0) {
    if (prec == LRCC_FP64)
      LRCC_HIP(h, stage_L<double>(L, LRCC_C128, g, form, dst.as<double>(), h->stream));
    else
      LRCC_HIP(h, stage_L<float>(L, LRCC_C128, g, form, dst.as<float>(), h->stream));
  }
  return LRCC_OK;
}

// s = ladder(xin) for all rows (block layout, FP64 accumulation), with the
// Cholesky vectors staged for `prec` in ls.
lrcc_status apply_ppl(Solver& S, const double* xin, lrcc_prec prec, lrcc_cmul cmul,
                      const void* ls) {
  lrcc_handle h = S.h;
  Geom g = S.g;
  g.ncp = (int)roundup(g.nchol, ppl_chunk(prec, cmul));
  LRCC_HIP(h, fill_zero(S.s, (size_t)2 * S.d.plane * 8, h->stream));
  if (g.nchol == 0) return LRCC_OK;
  if (prec == LRCC_BF16X3) {
    g.ncp = (int)roundup(g.nchol, bf16x3_chunk());
    LRCC_HIP(h, bf16x3_split_x(xin, g, S.x32, h->stream));
    lrcc_status st = bf16x3_apply(h, g, ls, S.x32, S.s, true, S.nonherm);
    if (st != LRCC_OK) return st;
    ++S.n_sigma_lp;
    return LRCC_OK;
  }
  if (prec == LRCC_FP64) {
    lrcc_status st = ppl_run(h, prec, cmul, true, g, ls, xin, S.s, S.nonherm);
    if (st != LRCC_OK) return st;
    ++S.n_sigma64;
    return LRCC_OK;
  }
  // FP32: float operands and float sums across tiles (the atomic additions
  // of the partial sums cost half the memory traffic of FP64 ones), widened
  // to the FP64 planes afterwards
  const long n = 2 * S.d.plane;
  const dim3 grid((unsigned)std::min<long>((n + RB - 1) / RB, 8192));
  hipLaunchKernelGGL(k_to_f32, grid, dim3(RB), 0, h->stream, n, xin, S.x32);
  LRCC_HIP(h, hipGetLastError());
  LRCC_HIP(h, fill_zero(S.s32, (size_t)n * 4, h->stream));
  lrcc_status st = ppl_run(h, prec, cmul, false, g, ls, S.x32, S.s32, S.nonherm);
  if (st != LRCC_OK) return st;
  hipLaunchKernelGGL(k_to_f64, grid, dim3(RB), 0, h->stream, n, S.s32, S.s);
  LRCC_HIP(h, hipGetLastError());
  ++S.n_sigma_lp;
  return LRCC_OK;
}

// s = the two-electron part of the Jacobian applied to xin: the particle-
// particle ladder in `prec` alone or, when the model includes the hole-hole
// ladder (and the ring term), the T = 0 doubles-doubles block of the
// two-electron operator, 1/2 PPL + 1/2 HHL (+ RING) in the ladders' doubled
// convention (the hole-hole ladder in FP64: its npo^2 npv cost per
// right-hand side is small beside the ladder's; S.W holds the half).
lrcc_status apply_sigma(Solver& S, const double* xin, lrcc_prec prec, lrcc_cmul cmul,
                        const void* ls) {
  lrcc_status st = apply_ppl(S, xin, prec, cmul, ls);
  if (st != LRCC_OK || !S.W || S.g.nchol == 0) return st;
  {
    const long n = 2 * S.d.plane;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)std::min<long>((n + RB - 1) / RB, 8192)), dim3(RB),
                       0, S.h->stream, n, 0.5, S.s);
    LRCC_HIP(S.h, hipGetLastError());
  }
  LRCC_HIP(S.h, hh_apply(S.W, S.g, xin, S.s, S.h->stream));
  if (!S.ringM) return LRCC_OK;
  // the ring term on packed doubles: block -> packed, ring, packed -> block, add
  hipStream_t s = S.h->stream;
  const int nrhs = S.ncomp * S.nomega;
  LRCC_HIP(S.h, block_to_pack<double>(xin, S.g, S.tab, S.rx, LRCC_C128, s));
  st = ring_apply(S.h, S.g.o, S.g.v, nrhs, S.ringM, S.rx, S.rs, false, S.rws);
  if (st != LRCC_OK) return st;
  LRCC_HIP(S.h, pack_to_block<double>(S.rs, LRCC_C128, S.g, S.tab, S.rb, s));
  const long n = 2 * S.d.plane;
  hipLaunchKernelGGL(k_axpy1, dim3((unsigned)std::min<long>((n + RB - 1) / RB, 8192)), dim3(RB),
                     0, s, n, S.rb, S.s);
  LRCC_HIP(S.h, hipGetLastError());
  return LRCC_OK;
}

// Start of a Jacobi + DIIS run: active flags, empty subspace, iteration 0,
// x = b / (D - w).
lrcc_status start_iteration(Solver& S, const double* b, double* x, const int* h_active_in,
                            hipStream_t st, bool keep_x = false) {
  lrcc_handle h = S.h;
  LRCC_HIP(h, hipMemcpyAsync(S.active, h_active_in, S.n * sizeof(int), hipMemcpyHostToDevice, st));
  LRCC_HIP(h, fill_zero(S.valid, roundup((long)S.n * 4, 16), st));
  LRCC_HIP(h, fill_zero(S.itp, 16, st));
  if (!keep_x) {  // else x holds the caller's initial amplitudes
    hipLaunchKernelGGL(k_start, grid_rhs(S, S.n), dim3(RB), 0, st, S.d, S.eps, S.omega, S.tab,
                       S.otab, S.active, b, x);
    LRCC_HIP(h, hipGetLastError());
  }
  S.act.assign(h_active_in, h_active_in + S.n);
  return LRCC_OK;
}

// The vector part of one iteration after the ladder: residual pass, DIIS,
// extrapolation, counter.  All launches on `st` (capturable).
lrcc_status iterate_vectors(Solver& S, const double* b, double* x, double tol, int max_iter,
                            hipStream_t st) {
  lrcc_handle h = S.h;
  hipLaunchKernelGGL(k_resid, grid_rhs(S, S.n), dim3(RB), 0, st, S.d, S.eps, S.omega, S.tab,
                     S.otab, S.active, S.valid, (const int*)S.itp, S.mdim, b, x, S.s, S.xt, S.ev,
                     S.part);
  LRCC_HIP(h, hipGetLastError());
  hipLaunchKernelGGL(k_diis, dim3(S.n), dim3(64), 0, st, S.nchunk, S.mdim, (const int*)S.itp,
                     max_iter, tol, S.part, S.active, S.valid, S.Bm, S.coef, S.relres);
  LRCC_HIP(h, hipGetLastError());
  hipLaunchKernelGGL(k_extrap, grid_rhs(S, S.n), dim3(RB), 0, st, S.d, S.mdim, S.active,
                     S.valid, S.coef, S.xt, x);
  LRCC_HIP(h, hipGetLastError());
  hipLaunchKernelGGL(k_inc, dim3(1), dim3(64), 0, st, S.itp);
  LRCC_HIP(h, hipGetLastError());
  return LRCC_OK;
}

// After an iteration: copy flags and residuals to the host (async on st).
lrcc_status fetch_flags(Solver& S, hipStream_t st) {
  lrcc_handle h = S.h;
  LRCC_HIP(h, hipMemcpyAsync(S.h_active, S.active, S.n * sizeof(int), hipMemcpyDeviceToHost, st));
  LRCC_HIP(h, hipMemcpyAsync(S.h_relres, S.relres, S.n * sizeof(double), hipMemcpyDeviceToHost,
                             st));
  return LRCC_OK;
}

// Host bookkeeping after fetch_flags completed; returns the number of RHS
// still active and updates *result.
int absorb_flags(Solver& S, int it, double tol, lrcc_status* result) {
  int nact = 0;
  for (int r = 0; r < S.n; ++r) {
    if (!S.act[r]) continue;
    if (!std::isfinite(S.h_relres[r])) *result = LRCC_ERR_NONFINITE;
    if (S.h_active[r]) {
      ++nact;
    } else {
      S.act[r] = 0;
      if (S.h_relres[r] >= tol && *result == LRCC_OK) *result = LRCC_ERR_NOT_CONVERGED;
    }
  }
  S.iters_max = std::max(S.iters_max, it);
  return nact;
}

// One metrics line: the solve side, the phase (fp64: the FP64 solve;
// inner: a reduced-precision inner iteration; outer: a refinement sweep's
// FP64 residual), the sweep, the iteration, the active count, every right-
// hand side's relative residual and the milliseconds since the call began.
void write_metrics(Solver& S, int it, int nact, const double* rel) {
  if (!S.metrics) return;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                              S.t0).count();
  std::fprintf(S.metrics, "{\"side\": \"%s\", \"phase\": \"%s\", \"sweep\": %d, \"iter\": %d, "
               "\"active\": %d, \"ms\": %.3f, \"relres\": [", S.side, S.phase, S.sweep, it, nact, ms);
  for (int r = 0; r < S.n; ++r) std::fprintf(S.metrics, r ? ", %.6e" : "%.6e", rel[r]);
  std::fprintf(S.metrics, "]}\n");
  std::fflush(S.metrics);
}

// Jacobi + DIIS for (A - w) x = b on the RHS whose active flag is set on
// entry.  x receives the solution.  Returns LRCC_ERR_NOT_CONVERGED if any
// RHS stopped at max_iter, LRCC_ERR_NONFINITE on NaN/Inf.
lrcc_status jacobi_diis(Solver& S, const double* b, double* x, lrcc_prec prec, lrcc_cmul cmul,
                        const void* ls, double tol, int max_iter, const int* h_active_in,
                        bool keep_x = false) {
  lrcc_handle h = S.h;
  lrcc_status st = start_iteration(S, b, x, h_active_in, h->stream, keep_x);
  if (st != LRCC_OK) return st;
  lrcc_status result = LRCC_OK;
  for (int it = 0;; ++it) {
    st = apply_sigma(S, x, prec, cmul, ls);
    if (st != LRCC_OK) return st;
    st = iterate_vectors(S, b, x, tol, max_iter, h->stream);
    if (st != LRCC_OK) return st;
    st = fetch_flags(S, h->stream);
    if (st != LRCC_OK) return st;
    LRCC_HIP(h, hipStreamSynchronize(h->stream));
    const int nact = absorb_flags(S, it, tol, &result);
    write_metrics(S, it, nact, S.h_relres);
    if (nact == 0 || result == LRCC_ERR_NONFINITE) break;
  }
  return result;
}

lrcc_status finish_alpha(Solver& S, const double* x, double* alpha, hipStream_t st) {
  lrcc_handle h = S.h;
  const int np = S.nomega * S.ncomp * S.ncomp;
  hipLaunchKernelGGL(k_alpha, dim3(S.nchunk, np), dim3(RB), 0, st, S.d, S.ncomp, S.xi, x, S.part);
  LRCC_HIP(h, hipGetLastError());
  LRCC_HIP(h, hipMemcpyAsync(S.h_part, S.part, (size_t)np * S.nchunk * sizeof(double2),
                             hipMemcpyDeviceToHost, st));
  LRCC_HIP(h, hipStreamSynchronize(st));
  for (int p = 0; p < np; ++p) {
    double re = 0, im = 0;
    for (int c = 0; c < S.nchunk; ++c) {
      re += S.h_part[(size_t)p * S.nchunk + c].x;
      im += S.h_part[(size_t)p * S.nchunk + c].y;
    }
    alpha[2 * p] = -re;  // alpha_xy = -<xi_x | X_y>
    alpha[2 * p + 1] = -im;
  }
  return LRCC_OK;
}

struct Opts {
  double tol, inner_tol;
  int max_iter, mdim, max_outer;
};

// Refinement residual: rk = b - (D - w) x2 - sx for the active right-hand
// sides (device flags); the relative residual norms of those flagged in
// `flags` into rel.  Synchronises `st`.
lrcc_status refine_residual(Solver& S, const std::vector<int>& flags, std::vector<double>& rel,
                            hipStream_t st) {
  lrcc_handle h = S.h;
  hipLaunchKernelGGL(k_outer, grid_rhs(S, S.n), dim3(RB), 0, st, S.d, S.eps, S.omega, S.tab,
                     S.otab, S.active, S.b, S.x2, S.sx, S.rk, S.part);
  LRCC_HIP(h, hipGetLastError());
  LRCC_HIP(h, hipMemcpyAsync(S.h_part, S.part, (size_t)S.n * S.nchunk * sizeof(double2),
                             hipMemcpyDeviceToHost, st));
  LRCC_HIP(h, hipStreamSynchronize(st));
  for (int r = 0; r < S.n; ++r) {
    if (!flags[r]) continue;
    double rr = 0, bb = 0;
    for (int c = 0; c < S.nchunk; ++c) {
      rr += S.h_part[(size_t)r * S.nchunk + c].x;
      bb += S.h_part[(size_t)r * S.nchunk + c].y;
    }
    rel[r] = std::sqrt(rr / bb);
    if (!std::isfinite(rel[r])) return fail(h, LRCC_ERR_NONFINITE, "non-finite residual");
  }
  return LRCC_OK;
}

lrcc_status read_opts(lrcc_handle h, const lrcc_solve_opts* in, lrcc_solve_opts* op, Opts* o) {
  *op = lrcc_solve_opts{};
  if (in) *op = *in;
  o->tol = op->tol > 0 ? op->tol : 1e-8;
  o->max_iter = op->max_iter > 0 ? op->max_iter : 100;
  o->mdim = op->diis_dim > 0 ? op->diis_dim : 8;
  o->inner_tol = op->inner_tol > 0 ? op->inner_tol : 1e-5;
  o->max_outer = op->max_outer > 0 ? op->max_outer : 6;
  if (o->mdim > MAXD) return fail(h, LRCC_ERR_ARG, "diis_dim exceeds 12");
  if (op->prec != LRCC_FP64 && op->prec != LRCC_FP32 && op->prec != LRCC_BF16X3)
    return fail(h, LRCC_ERR_ARG, "unknown precision");
  if (op->cmul != LRCC_CMUL_4M && op->cmul != LRCC_CMUL_3M)
    return fail(h, LRCC_ERR_ARG, "unknown complex-multiply form");

  if ((op->L_ov != nullptr) != (op->L_vo != nullptr))
    return fail(h, LRCC_ERR_ARG, "L_ov and L_vo come together");
  if (op->L_ov && !op->L_oo)
    return fail(h, LRCC_ERR_ARG, "the ring term needs L_oo as well");
  if ((uintptr_t)op->x0 % 16 || (uintptr_t)op->x_out % 16)
    return fail(h, LRCC_ERR_ARG, "x0/x_out not 16-byte aligned");
  const void* ps[] = {op->L_oo, op->L_ov, op->L_vo};
  for (const void* q : ps)
    if (q && (uintptr_t)q % 16) return fail(h, LRCC_ERR_ARG, "L_oo/L_ov/L_vo not 16-byte aligned");
  return LRCC_OK;
}

}  // namespace

namespace {

// One response solve: (A' - w) X = -b for every (w, component), with
// A' X = D o X + K(L') X, L' = L or L^T (form) and b = xi or its conjugate
// (conj_rhs); alpha receives -<b_x | X_y> per w.  Counts go into *tally.
// Returns LRCC_OK, LRCC_ERR_NOT_CONVERGED (alpha filled) or an error.
lrcc_status solve_side(lrcc_handle h, int o, int v, int nchol, const double* eps, const void* L,
                       int ncomp, const void* mu, int nomega, const double* omegas,
                       const lrcc_solve_opts& op, const Opts& O, LForm form, bool conj_rhs,
                       double* alpha, lrcc_solve_info* tally, FILE* metrics,
                       std::chrono::steady_clock::time_point t0) {
  lrcc_status st;
  const bool ir = op.prec != LRCC_FP64;
  Solver S;
  for (int k = 0; k < 12; ++k) S.buf[k] = &h->sv[k];
  st = setup(S, h, o, v, nchol, eps, ncomp, mu, nomega, omegas, O.mdim, ir, h->tab.as<int>(),
             conj_rhs, h->stream);
  if (st != LRCC_OK) return st;
  // staged vectors: h->ls for the FP64 ladder (or the refinement's anchor
  // ladder), h->ls2 for the reduced-precision inner ladder
  const lrcc_prec anchor = ir ? op.anchor_prec : LRCC_FP64;
  if (anchor != LRCC_FP64 && anchor != LRCC_FP32)
    return fail(h, LRCC_ERR_ARG, "anchor_prec must be FP64 or FP32");
  LRCC_HIP(h, herm_check(L, LRCC_C128, v, nchol, S.nonherm, h->stream));
  if (op.L_oo && nchol > 0) {  // the hole-hole ladder: W (or W^T for L^T)
    const size_t wbytes = (size_t)S.g.npo * S.g.npo * 16;
    LRCC_HIP(h, h->hw.ensure(wbytes));
    LRCC_HIP(h, hh_build_w(op.L_oo, LRCC_C128, o, nchol, S.otab, form, 1.0,
                           h->hw.as<double2>(), h->stream));
    S.W = h->hw.as<double2>();
    if (op.L_ov) {  // the ring term: M from the blocks of L (or of L^T)
      const int nrhs = S.ncomp * S.nomega;
      if ((long)o * v > 65535 || (long)nrhs * o * v >= (1L << 31))
        return fail(h, LRCC_ERR_SHAPE, "ring term: o v exceeds 65535 or nrhs o v reaches 2^31");
      const size_t mb = ring_m_bytes(o, v);
      const size_t bb = ring_build_ws_bytes(o, v, nchol, form == L_TRANS);
      const size_t ab = ring_apply_ws_bytes(o, v, nrhs);
      const size_t pk = ((size_t)nrhs * S.g.npo * S.g.npv * 16 + 255) / 256 * 256;
      const size_t bl = ((size_t)2 * S.d.plane * 8 + 255) / 256 * 256;
      LRCC_HIP(h, h->rw.ensure(mb + std::max(bb, ab + 2 * pk + bl)));
      char* base = h->rw.as<char>();
      double2* M = reinterpret_cast<double2*>(base);
      st = ring_build_m(h, o, v, nchol, op.L_oo, op.L_ov, op.L_vo, L, form == L_TRANS, M,
                        base + mb);
      if (st != LRCC_OK) return st;
      S.ringM = M;
      S.rws = base + mb;
      S.rx = reinterpret_cast<double2*>(base + mb + ab);
      S.rs = reinterpret_cast<double2*>(base + mb + ab + pk);
      S.rb = reinterpret_cast<double*>(base + mb + ab + 2 * pk);
    }
  }
  st = stage_for(S, L, anchor, op.cmul, h->ls, form);
  if (st != LRCC_OK) return st;
  if (ir) {
    st = stage_for(S, L, op.prec, op.cmul, h->ls2, form);
    if (st != LRCC_OK) return st;
  }
  const size_t vb = (size_t)2 * S.d.plane * 8;
  std::vector<int> all(S.n, 1);

  S.metrics = metrics;
  S.t0 = t0;
  S.side = form == L_TRANS ? "left" : "right";
  // the caller's initial amplitudes and final-amplitude buffer belong to the
  // right-hand solve
  const bool warm = op.x0 != nullptr && form == L_PLAIN;
  void* const x_out = form == L_PLAIN ? op.x_out : nullptr;

  lrcc_status result = LRCC_OK;
  double final_rel = 0;
  if (!ir) {
    if (warm) LRCC_HIP(h, pack_to_block<double>(op.x0, LRCC_C128, S.g, S.tab, S.x, h->stream));
    S.phase = "fp64";
    result = jacobi_diis(S, S.b, S.x, LRCC_FP64, op.cmul, h->ls.p, O.tol, O.max_iter,
                         all.data(), warm);
    for (int r = 0; r < S.n; ++r) final_rel = std::max(final_rel, S.h_relres[r]);
    if (result == LRCC_ERR_NONFINITE) return fail(h, result, "non-finite residual");
    st = finish_alpha(S, S.x, alpha, h->stream);
    if (st != LRCC_OK) return st;
    if (x_out) LRCC_HIP(h, block_to_pack<double>(S.x, S.g, S.tab, x_out, LRCC_C128, h->stream));
  } else {
    // iterative refinement: x2 = 0 (or the initial amplitudes), rk = b - A x2
    if (warm) LRCC_HIP(h, pack_to_block<double>(op.x0, LRCC_C128, S.g, S.tab, S.x2, h->stream));
    else LRCC_HIP(h, fill_zero(S.x2, vb, h->stream));
    LRCC_HIP(h, hipMemcpyAsync(S.rk, S.b, vb, hipMemcpyDeviceToDevice, h->stream));
    std::vector<int> act(S.n, 1);
    std::vector<double> rel(S.n, 1.0);
    auto outer_residual = [&](const std::vector<int>& flags) -> lrcc_status {
      return refine_residual(S, flags, rel, h->stream);
    };
    // whether sx is the FP64 ladder of the whole iterate (then rel is the true
    // FP64 residual), or an estimate built from reduced-precision ladders
    bool sx_exact = false;
    result = LRCC_ERR_NOT_CONVERGED;
    int nact0 = S.n;
    if (warm) {
      // residual of the initial amplitudes, with the full-iterate ladder
      LRCC_HIP(h, hipMemcpyAsync(S.active, act.data(), S.n * sizeof(int), hipMemcpyHostToDevice,
                                 h->stream));
      st = apply_sigma(S, S.x2, anchor, op.cmul, h->ls.p);
      if (st != LRCC_OK) return st;
      LRCC_HIP(h, hipMemcpyAsync(S.sx, S.s, vb, hipMemcpyDeviceToDevice, h->stream));
      sx_exact = anchor == LRCC_FP64;
      st = outer_residual(act);
      if (st != LRCC_OK) return st;
      nact0 = 0;
      for (int r = 0; r < S.n; ++r) {
        if (rel[r] < O.tol) act[r] = 0;
        else ++nact0;
      }
      S.phase = "outer";
      S.sweep = -1;
      write_metrics(S, 0, nact0, rel.data());
      if (nact0 == 0) result = LRCC_OK;
    }
    // the precision of the full-iterate ladders: the anchor, and FP64 once a
    // check of the returned iterate has run (its staged vectors replace the
    // anchor's)
    lrcc_prec full_prec = anchor;
    bool exact_sweeps = op.resid_fp64_every != 0;
    int outer = 0;
    for (;;) {
      for (; outer < O.max_outer && nact0 > 0; ++outer) {
        S.phase = "inner";
        S.sweep = outer;
        lrcc_status is = jacobi_diis(S, S.rk, S.x, op.prec, op.cmul, h->ls2.p, O.inner_tol,
                                     O.max_iter, act.data());
        // an inner solve that stops short is refined further; any other
        // failure ends the solve
        if (is == LRCC_ERR_NONFINITE) return fail(h, is, "non-finite residual");
        if (is != LRCC_OK && is != LRCC_ERR_NOT_CONVERGED) return is;
        // x2 += d; sx = ladder(x2): the full-iterate ladder in the first sweep
        // (or every sweep), else sx += reduced-precision ladder of the
        // correction d; then rk = b - (D - w) x2 - sx
        LRCC_HIP(h, hipMemcpyAsync(S.active, act.data(), S.n * sizeof(int),
                                   hipMemcpyHostToDevice, h->stream));
        hipLaunchKernelGGL(k_add, grid_rhs(S, S.n), dim3(RB), 0, h->stream, S.d, S.active, S.x,
                           S.x2);
        LRCC_HIP(h, hipGetLastError());
        if (outer == 0 || exact_sweeps) {
          st = apply_sigma(S, S.x2, full_prec, op.cmul, h->ls.p);
          if (st != LRCC_OK) return st;
          LRCC_HIP(h, hipMemcpyAsync(S.sx, S.s, vb, hipMemcpyDeviceToDevice, h->stream));
          sx_exact = full_prec == LRCC_FP64;
        } else {
          st = apply_sigma(S, S.x, op.prec, op.cmul, h->ls2.p);
          if (st != LRCC_OK) return st;
          hipLaunchKernelGGL(k_acc, grid_rhs(S, S.n), dim3(RB), 0, h->stream, S.d, S.active,
                             S.s, S.sx);
          LRCC_HIP(h, hipGetLastError());
          sx_exact = false;
        }
        st = outer_residual(act);
        if (st != LRCC_OK) return st;
        int nact = 0;
        for (int r = 0; r < S.n; ++r) {
          if (!act[r]) continue;
          if (rel[r] < O.tol) act[r] = 0;
          else ++nact;
        }
        S.phase = "outer";
        write_metrics(S, 0, nact, rel.data());
        nact0 = nact;
      }
      if (nact0 > 0 || sx_exact) break;  // out of sweeps, or converged on the FP64 residual
      // The stopping test used an estimate of the ladder of x2 (an FP32
      // anchor, or an FP64 anchor plus reduced-precision ladders of the later
      // corrections).  The reported residual is the FP64 one of the returned
      // iterate: one FP64 ladder of every right-hand side's x2.  Where it
      // misses the tolerance the refinement goes on from that residual, with
      // an FP64 ladder of the whole iterate in every further sweep.
      if (full_prec != LRCC_FP64) {
        st = stage_for(S, L, LRCC_FP64, op.cmul, h->ls, form);
        if (st != LRCC_OK) return st;
        full_prec = LRCC_FP64;
      }
      std::vector<int> every(S.n, 1);
      LRCC_HIP(h, hipMemcpyAsync(S.active, every.data(), S.n * sizeof(int),
                                 hipMemcpyHostToDevice, h->stream));
      st = apply_sigma(S, S.x2, LRCC_FP64, op.cmul, h->ls.p);
      if (st != LRCC_OK) return st;
      LRCC_HIP(h, hipMemcpyAsync(S.sx, S.s, vb, hipMemcpyDeviceToDevice, h->stream));
      st = outer_residual(every);
      if (st != LRCC_OK) return st;
      sx_exact = true;
      exact_sweeps = true;
      nact0 = 0;
      for (int r = 0; r < S.n; ++r) {
        act[r] = !(rel[r] < O.tol);
        nact0 += act[r];
      }
      S.phase = "final";
      write_metrics(S, 0, nact0, rel.data());
      if (nact0 == 0) break;
    }
    result = nact0 == 0 ? LRCC_OK : LRCC_ERR_NOT_CONVERGED;
    for (int r = 0; r < S.n; ++r) final_rel = std::max(final_rel, rel[r]);
    st = finish_alpha(S, S.x2, alpha, h->stream);
    if (st != LRCC_OK) return st;
    if (x_out) LRCC_HIP(h, block_to_pack<double>(S.x2, S.g, S.tab, x_out, LRCC_C128, h->stream));
  }
  tally->iters_max = std::max(tally->iters_max, S.iters_max);
  tally->n_sigma_fp64 += S.n_sigma64;
  tally->n_sigma_lowp += S.n_sigma_lp;
  tally->final_relres = std::max(tally->final_relres, final_rel);
  return result;
}

}  // namespace

lrcc_status solve_impl(lrcc_handle h, int o, int v, int nchol, const double* eps, const void* L,
                       int ncomp, const void* mu, int nomega, const double* omegas,
                       const lrcc_solve_opts* opts_in, double* alpha, lrcc_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  lrcc_solve_opts op;
  Opts O;
  lrcc_status st = read_opts(h, opts_in, &op, &O);
  if (st != LRCC_OK) return st;
  if (op.response != 0 && op.response != 1) return fail(h, LRCC_ERR_ARG, "unknown response mode");
  // deterministic ladders for this solve (the handle's setting is restored after)
  struct DetGuard {
    lrcc_handle h;
    int prev;
    ~DetGuard() { h->deterministic = prev; }
  } det{h, h->deterministic};
  if (op.deterministic) h->deterministic = 1;
  // per-iteration metrics: one JSON line per iteration appended to the file
  struct MetricsFile {
    FILE* f = nullptr;
    ~MetricsFile() {
      if (f) std::fclose(f);
    }
  } mf;
  if (op.metrics_path) {
    mf.f = std::fopen(op.metrics_path, "a");
    if (!mf.f) return fail(h, LRCC_ERR_ARG, std::string("cannot open ") + op.metrics_path);
  }
  const size_t np = (size_t)nomega * ncomp * ncomp;
  {
    const Geom g = make_geom(o, v, nchol, nomega * ncomp, 1);
    if (g.M == 0 || g.npv == 0) {
      for (size_t p = 0; p < 2 * np; ++p) alpha[p] = 0;
      if (info) *info = lrcc_solve_info{0, 0, 0, 0.0, 0.0};
      return LRCC_OK;
    }
    st = ensure_tab(h, g.nbv);
    if (st != LRCC_OK) return st;
  }
  lrcc_solve_info tally{0, 0, 0, 0.0, 0.0};
  lrcc_status result;
  if (op.response == 0) {
    // right-hand amplitudes: alpha_xy = -<xi_x | X_y(w)>
    result = solve_side(h, o, v, nchol, eps, L, ncomp, mu, nomega, omegas, op, O, L_PLAIN, false,
                        alpha, &tally, mf.f, t0);
  } else {
    // full linear response function (Sec. 2.2): right-hand X(w) from
    // (A - w) X = -xi, left-hand Y(w) from Y (A + w) = -eta with eta =
    // conj(xi) and F = 0 in this model, i.e. (A^T + w) Y^T = -eta: the same
    // solver with L^T, -w and the conjugate right-hand side.  With
    // f_xy = sum Y_y xi_x + sum eta_x X_y = -(aL + aR)_xy, the response
    // function is (f_xy + conj f_yx) / 2 and alpha = -(that).
    std::vector<double> ar(2 * np), al(2 * np), wneg(nomega);
    lrcc_status rr = solve_side(h, o, v, nchol, eps, L, ncomp, mu, nomega, omegas, op, O,
                                L_PLAIN, false, ar.data(), &tally, mf.f, t0);
    if (rr != LRCC_OK && rr != LRCC_ERR_NOT_CONVERGED) return rr;
    for (int w = 0; w < nomega; ++w) wneg[w] = -omegas[w];
    lrcc_status rl = solve_side(h, o, v, nchol, eps, L, ncomp, mu, nomega, wneg.data(), op, O,
                                L_TRANS, true, al.data(), &tally, mf.f, t0);
    if (rl != LRCC_OK && rl != LRCC_ERR_NOT_CONVERGED) return rl;
    for (int w = 0; w < nomega; ++w)
      for (int x = 0; x < ncomp; ++x)
        for (int y = 0; y < ncomp; ++y) {
          const size_t pxy = 2 * (((size_t)w * ncomp + x) * ncomp + y);
          const size_t pyx = 2 * (((size_t)w * ncomp + y) * ncomp + x);
          alpha[pxy] = 0.5 * ((ar[pxy] + al[pxy]) + (ar[pyx] + al[pyx]));
          alpha[pxy + 1] = 0.5 * ((ar[pxy + 1] + al[pxy + 1]) - (ar[pyx + 1] + al[pyx + 1]));
        }
    result = rr != LRCC_OK ? rr : rl;
  }
  if (info) {
    *info = tally;
    info->seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (result == LRCC_ERR_NOT_CONVERGED) return fail(h, result, "tolerance not reached");
  return result;
}


// ---------------------------------------------------------------------------
// Batched solve: every instance keeps its own state; per iteration one
// persistent ladder launch serves all active instances from one work queue,
// and the whole iteration (queue reset, accumulator zeroing, ladder, and each
// instance's residual / DIIS / extrapolation / counter kernels) is captured
// once into a hip graph and replayed until the active set changes.

// Batched iterative refinement (reduced-precision inner solves).  Per sweep:
// the correction equation (A - w) d = r of every instance with unconverged
// right-hand sides, one instance after another with the reduced-precision
// ladder (the DIIS ring, the reduced-precision doubles and staged vectors
// shared, `ls2` restaged per instance); x2 += d; then the FP64 ladder of
// every such instance's x2 in ONE persistent launch, and each instance's
// FP64 residual r = b - (D - w) x2 - ladder(x2).  Every sweep ends on that
// FP64 residual, which is the stopping test and the reported residual.
template <class Upload>
lrcc_status batched_refine(lrcc_handle h, int ninst, const lrcc_instance* inst,
                           const lrcc_solve_opts& op, const Opts& O,
                           std::vector<std::unique_ptr<Solver>>& S, const std::vector<int>& live,
                           Upload& upload_desc, Buf& desc, size_t desc_bytes, Buf& counter, int nx,
                           Buf& ls2, hipStream_t cs, lrcc_solve_info* info,
                           std::chrono::steady_clock::time_point t0) {
  lrcc_status st;
  hipStream_t hs = h->stream;
  LRCC_HIP(h, hipStreamSynchronize(cs));  // the set-up ran on cs
  std::vector<std::vector<int>> act(ninst);
  std::vector<std::vector<double>> rel(ninst);
  for (int i : live) {
    Solver& Si = *S[i];
    act[i].assign(Si.n, 1);
    rel[i].assign(Si.n, 1.0);
    const size_t vb = (size_t)2 * Si.d.plane * 8;
    LRCC_HIP(h, fill_zero(Si.x2, vb, hs));
    LRCC_HIP(h, hipMemcpyAsync(Si.rk, Si.b, vb, hipMemcpyDeviceToDevice, hs));
  }
  int n_outer = 0;
  for (int sweep = 0; sweep < O.max_outer; ++sweep) {
    std::vector<int> now;
    for (int i : live)
      if (std::count(act[i].begin(), act[i].end(), 1) > 0) now.push_back(i);
    if (now.empty()) break;
    for (int i : now) {
      Solver& Si = *S[i];
      // the reduced-precision ladders take the handle's block-pair table
      st = ensure_tab(h, Si.g.nbv);
      if (st != LRCC_OK) return st;
      st = stage_for(Si, inst[i].L, op.prec, op.cmul, ls2, L_PLAIN);
      if (st != LRCC_OK) return st;
      Si.phase = "inner";
      Si.sweep = sweep;
      lrcc_status is = jacobi_diis(Si, Si.rk, Si.x, op.prec, op.cmul, ls2.p, O.inner_tol,
                                   O.max_iter, act[i].data());
      if (is == LRCC_ERR_NONFINITE) return fail(h, is, "non-finite residual");
      if (is != LRCC_OK && is != LRCC_ERR_NOT_CONVERGED) return is;
      LRCC_HIP(h, hipMemcpyAsync(Si.active, act[i].data(), Si.n * sizeof(int),
                                 hipMemcpyHostToDevice, hs));
      hipLaunchKernelGGL(k_add, grid_rhs(Si, Si.n), dim3(RB), 0, hs, Si.d, Si.active, Si.x, Si.x2);
      LRCC_HIP(h, hipGetLastError());
      LRCC_HIP(h, fill_zero(Si.s, (size_t)2 * Si.d.plane * 8, hs));
    }
    // the FP64 ladder of every refined iterate in one persistent launch
    st = upload_desc(now, true, hs);
    if (st != LRCC_OK) return st;
    LRCC_HIP(h, fill_zero(counter.p, 64, hs));
    LRCC_HIP(h, ppl_queue_launch(desc.as<BatchInst>(), (int)now.size(),
                                 reinterpret_cast<const long*>(desc.as<char>() + desc_bytes), nx,
                                 counter.as<unsigned>(), h->ncu, op.cmul == LRCC_CMUL_3M, hs));
    ++n_outer;
    for (int i : now) {
      Solver& Si = *S[i];
      LRCC_HIP(h, hipMemcpyAsync(Si.sx, Si.s, (size_t)2 * Si.d.plane * 8,
                                 hipMemcpyDeviceToDevice, hs));
      st = refine_residual(Si, act[i], rel[i], hs);
      if (st != LRCC_OK) return st;
      for (int r = 0; r < Si.n; ++r)
        if (act[i][r] && rel[i][r] < O.tol) act[i][r] = 0;
    }
  }
  lrcc_status result = LRCC_OK;
  double final_rel = 0;
  int iters_max = 0, n_lowp = 0;
  for (int i : live) {
    Solver& Si = *S[i];
    for (int r = 0; r < Si.n; ++r) {
      final_rel = std::max(final_rel, rel[i][r]);
      if (act[i][r]) result = LRCC_ERR_NOT_CONVERGED;
    }
    st = finish_alpha(Si, Si.x2, inst[i].alpha, hs);
    if (st != LRCC_OK) return st;
    iters_max = std::max(iters_max, Si.iters_max);
    n_lowp += Si.n_sigma_lp;
  }
  if (info) {
    info->iters_max = iters_max;
    info->n_sigma_fp64 = n_outer;
    info->n_sigma_lowp = n_lowp;
    info->final_relres = final_rel;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (result == LRCC_ERR_NOT_CONVERGED) return fail(h, result, "tolerance not reached");
  return result;
}

lrcc_status solve_batched_impl(lrcc_handle h, int ninst, const lrcc_instance* inst,
                               const lrcc_solve_opts* opts_in, lrcc_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  lrcc_solve_opts op;
  Opts O;
  lrcc_status st = read_opts(h, opts_in, &op, &O);
  if (st != LRCC_OK) return st;
  const bool ir = op.prec != LRCC_FP64;
  if (ir && op.anchor_prec != LRCC_FP64)
    return fail(h, LRCC_ERR_UNSUPPORTED,
                "the batched refinement takes its residuals from the FP64 ladder (anchor_prec)");
  if (op.x0 || op.x_out || op.metrics_path)
    return fail(h, LRCC_ERR_UNSUPPORTED,
                "the batched solve takes no initial amplitudes, amplitude output or metrics file");
  if (op.deterministic || h->deterministic)
    return fail(h, LRCC_ERR_UNSUPPORTED,
                "the batched solve's persistent ladder sums with atomics (no deterministic mode)");
  if (op.response != 0)
    return fail(h, LRCC_ERR_UNSUPPORTED, "the batched solve gives the right-hand response");
  if (op.L_oo || op.L_ov)
    return fail(h, LRCC_ERR_UNSUPPORTED, "the batched solve has no hole-hole ladder or ring term");
  constexpr int KC = 16;  // chunk of the persistent FP64 ladder
  std::vector<std::unique_ptr<Solver>> S(ninst);
  std::vector<std::unique_ptr<Buf[]>> own(ninst);
  std::vector<int> live;  // instances with work
  struct Free {
    std::vector<std::unique_ptr<Buf[]>>* o;
    ~Free() {
      for (auto& b : *o)
        if (b)
          for (int k = 0; k < NBUF; ++k) b[k].release();
    }
  } freer{&own};
  hipStream_t cs = nullptr;
  LRCC_HIP(h, hipStreamSynchronize(h->stream));
  LRCC_HIP(h, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  struct StreamFree {
    hipStream_t s;
    ~StreamFree() {
      if (s) (void)hipStreamDestroy(s);
    }
  } sfree{cs};
  const int nx = std::min(QXMAX, std::max(1, h->ncu / 32));  // XCDs
  // Refinement: the inner solves run one instance at a time, so the DIIS
  // ring, the reduced-precision copies of the doubles and the reduced-
  // precision staged vectors are one set, sized for the largest instance
  // and shared by all; each instance keeps its own iterate, residual and
  // ladder of the iterate.
  Buf shared[4];  // 0 ring X~, 1 ring e, 2 x32/s32, 3 staged reduced-precision vectors
  struct SharedFree {
    Buf* b;
    ~SharedFree() {
      for (int k = 0; k < 4; ++k) b[k].release();
    }
  } shfree{shared};
  if (ir) {
    size_t vmax = 0;
    for (int i = 0; i < ninst; ++i) {
      const Geom gi = make_geom(inst[i].o, inst[i].v, inst[i].nchol, inst[i].nomega * inst[i].ncomp, 1);
      if (gi.M == 0 || gi.npv == 0) continue;
      vmax = std::max(vmax, (size_t)2 * gi.xb_plane() * 8);
    }
    LRCC_HIP(h, shared[0].ensure(std::max<size_t>(vmax * O.mdim, 16)));
    LRCC_HIP(h, shared[1].ensure(std::max<size_t>(vmax * O.mdim, 16)));
    LRCC_HIP(h, shared[2].ensure(std::max<size_t>(vmax, 16)));
  }
  for (int i = 0; i < ninst; ++i) {
    const lrcc_instance& I = inst[i];
    S[i].reset(new Solver());
    own[i].reset(new Buf[NBUF]);
    Solver& Si = *S[i];
    for (int k = 0; k < NBUF; ++k) Si.buf[k] = &own[i][k];
    if (ir) {
      Si.buf[3] = &shared[0];
      Si.buf[4] = &shared[1];
      Si.buf[10] = &shared[2];
    }
    const Geom g0 = make_geom(I.o, I.v, I.nchol, I.nomega * I.ncomp, 1);
    if (g0.M == 0 || g0.npv == 0) {
      for (int p = 0; p < 2 * I.nomega * I.ncomp * I.ncomp; ++p) I.alpha[p] = 0;
      continue;
    }
    // block-pair table and tile order of this instance
    std::vector<int> tab, ord;
    block_pair_table(g0.nbv, &tab);
    supertile_order(g0, 0, g0.nbp, h->order_s[LRCC_FP64] > 0 ? h->order_s[LRCC_FP64] : 4, nx,
                    true, &ord);
    LRCC_HIP(h, own[i][13].ensure(tab.size() * 4));
    LRCC_HIP(h, own[i][14].ensure(ord.size() * 4));
    LRCC_HIP(h, hipMemcpyAsync(own[i][13].p, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, cs));
    LRCC_HIP(h, hipMemcpyAsync(own[i][14].p, ord.data(), ord.size() * 4, hipMemcpyHostToDevice, cs));
    LRCC_HIP(h, hipStreamSynchronize(cs));
    st = setup(Si, h, I.o, I.v, I.nchol, I.eps, I.ncomp, I.mu, I.nomega, I.omegas, O.mdim, ir,
               own[i][13].as<int>(), false, cs);
    if (st != LRCC_OK) return st;
    Geom gs = Si.g;
    gs.ncp = (int)roundup(gs.nchol, KC);
    LRCC_HIP(h, own[i][12].ensure(ppl_ls_bytes(LRCC_FP64, LRCC_CMUL_4M, gs)));
    LRCC_HIP(h, herm_check(I.L, LRCC_C128, I.v, I.nchol, Si.nonherm, cs));
    if (gs.nchol > 0)
      LRCC_HIP(h, stage_L<double>(I.L, LRCC_C128, gs, L_PLAIN, own[i][12].as<double>(), cs));
    std::vector<int> one(Si.n, 1);
    if (!ir) {
      st = start_iteration(Si, Si.b, Si.x, one.data(), cs);
      if (st != LRCC_OK) return st;
    }
    LRCC_HIP(h, hipStreamSynchronize(cs));  // `one` goes out of scope
    live.push_back(i);
  }
  // queue descriptors, longest tile first (tile cost ~ 2 ncp + Mp), then
  // the per-XCD item totals
  Buf desc, counter;
  struct DescFree {
    Buf* a;
    Buf* b;
    ~DescFree() {
      a->release();
      b->release();
    }
  } dfree{&desc, &counter};
  const size_t desc_bytes = roundup((long)sizeof(BatchInst) * std::max(1, ninst), 256);
  LRCC_HIP(h, desc.ensure(desc_bytes + sizeof(long) * QXMAX));
  LRCC_HIP(h, counter.ensure(64));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct GraphFree {
    hipGraph_t* g;
    hipGraphExec_t* e;
    ~GraphFree() {
      if (*e) (void)hipGraphExecDestroy(*e);
      if (*g) (void)hipGraphDestroy(*g);
    }
  } gfree{&graph, &exec};
  // queue descriptors of the instances `now` (longest tile first: tile cost
  // ~ 2 ncp + Mp), the ladder reading x (or x2, the refined iterate) and
  // writing s, then the per-XCD item totals; synchronises `q`
  auto by_cost = [&](std::vector<int>& now) {
    std::stable_sort(now.begin(), now.end(), [&](int a, int b) {
      const Solver &A = *S[a], &B = *S[b];
      return 2 * roundup(A.g.nchol, KC) + A.g.Mp > 2 * roundup(B.g.nchol, KC) + B.g.Mp;
    });
  };
  auto upload_desc = [&](std::vector<int>& now, bool use_x2, hipStream_t q) -> lrcc_status {
    by_cost(now);
    std::vector<BatchInst> d(now.size());
    long total = 0;
    std::vector<long> xtotal(QXMAX, 0);
    for (size_t k = 0; k < now.size(); ++k) {
      const Solver& Si = *S[now[k]];
      d[k] = BatchInst{own[now[k]][12].as<double>(), use_x2 ? Si.x2 : Si.x, Si.s, Si.tab,
                       own[now[k]][14].as<int>(), Si.nonherm, Si.g.nbv, Si.g.nbp,
                       (int)roundup(Si.g.nchol, KC), (int)Si.g.Mp, Si.g.v, total, {}};
      const long items = Si.g.nchol > 0 ? 2 * ppl_ntile(Si.g) : 0;  // tiles, then mirrors
      for (int x = 0; x < nx; ++x) {
        d[k].xstart[x] = xtotal[x];
        xtotal[x] += items > x ? (items - x + nx - 1) / nx : 0;  // items l = x mod nx
      }
      total += items;
    }
    LRCC_HIP(h, hipMemcpyAsync(desc.p, d.data(), d.size() * sizeof(BatchInst),
                               hipMemcpyHostToDevice, q));
    LRCC_HIP(h, hipMemcpyAsync(desc.as<char>() + desc_bytes, xtotal.data(), sizeof(long) * QXMAX,
                               hipMemcpyHostToDevice, q));
    LRCC_HIP(h, hipStreamSynchronize(q));
    return LRCC_OK;
  };
  if (ir) return batched_refine(h, ninst, inst, op, O, S, live, upload_desc, desc, desc_bytes,
                                counter, nx, shared[3], cs, info, t0);
  std::vector<int> active_set;  // instances in the captured graph
  lrcc_status result = LRCC_OK;
  int n_launch = 0;
  for (int it = 0;; ++it) {
    std::vector<int> now;
    for (int i : live) {
      bool any = false;
      for (int a : S[i]->act) any = any || a;
      if (any) now.push_back(i);
    }
    if (now.empty()) break;
    by_cost(now);  // the order of the captured set, so an unchanged set is not captured again
    if (now != active_set) {
      // (re)build the queue descriptors and capture one iteration
      st = upload_desc(now, false, cs);
      if (st != LRCC_OK) return st;
      if (exec) {
        LRCC_HIP(h, hipGraphExecDestroy(exec));
        exec = nullptr;
      }
      if (graph) {
        LRCC_HIP(h, hipGraphDestroy(graph));
        graph = nullptr;
      }
      LRCC_HIP(h, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      lrcc_status cst = LRCC_OK;
      hipError_t ce = fill_zero(counter.p, 64, cs);
      for (int i : now)
        if (ce == hipSuccess) ce = fill_zero(S[i]->s, (size_t)2 * S[i]->d.plane * 8, cs);
      if (ce == hipSuccess)
        ce = ppl_queue_launch(desc.as<BatchInst>(), (int)now.size(),
                              reinterpret_cast<const long*>(desc.as<char>() + desc_bytes), nx,
                              counter.as<unsigned>(), h->ncu, op.cmul == LRCC_CMUL_3M, cs);
      for (int i : now)
        if (ce == hipSuccess && cst == LRCC_OK)
          cst = iterate_vectors(*S[i], S[i]->b, S[i]->x, O.tol, O.max_iter, cs);
      hipError_t ee = hipStreamEndCapture(cs, &graph);
      if (ce != hipSuccess) return hip_fail(h, ce, "batched iteration capture");
      if (cst != LRCC_OK) return cst;
      LRCC_HIP(h, ee);
      LRCC_HIP(h, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      active_set = now;
    }
    LRCC_HIP(h, hipGraphLaunch(exec, cs));
    ++n_launch;
    for (int i : now) {
      st = fetch_flags(*S[i], cs);
      if (st != LRCC_OK) return st;
    }
    LRCC_HIP(h, hipStreamSynchronize(cs));
    for (int i : now) {
      S[i]->n_sigma64 += 1;
      absorb_flags(*S[i], it, O.tol, &result);
    }
    if (result == LRCC_ERR_NONFINITE) return fail(h, result, "non-finite residual");
  }
  double final_rel = 0;
  int iters_max = 0, nsig = 0;
  for (int i : live) {
    st = finish_alpha(*S[i], S[i]->x, inst[i].alpha, cs);
    if (st != LRCC_OK) return st;
    for (int r = 0; r < S[i]->n; ++r) final_rel = std::max(final_rel, S[i]->h_relres[r]);
    iters_max = std::max(iters_max, S[i]->iters_max);
    nsig = std::max(nsig, S[i]->n_sigma64);
  }
  if (info) {
    info->iters_max = iters_max;
    info->n_sigma_fp64 = n_launch;
    info->n_sigma_lowp = 0;
    info->final_relres = final_rel;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  (void)nsig;
  if (result == LRCC_ERR_NOT_CONVERGED) return fail(h, result, "tolerance not reached");
  return result;
}

}  // namespace lrcc
