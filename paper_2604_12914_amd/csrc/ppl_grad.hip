// Gradient of sigma = PPL(L, X) with respect to the Cholesky vectors.
//
// For a real loss with upstream gradient G (PyTorch's complex convention),
//   Lbar^P = 2 sum_m G_m conj(L^P) X_m^H,
// with G_m, X_m the full antisymmetric v x v matrices of row m = (r, ij).
// Taking the complex conjugate, Lbar = 2 conj(Z) with
//   Z^P_ac = sum_{b,d} R[(a,b),(c,d)] L^P_bd,   R[(a,b),(c,d)] = sum_m conj(G_m^ab) X_m^cd.
// R is antisymmetric in (a, b) and in (c, d), so it is formed only on packed
// pairs a < b, c < d, block pair by block pair:
//   R'(AB, CD)[(a b), (c d)] = sum_m conj(G[m, AB]) X[m, CD]   (k_grad_r)
// -- a quarter of the full v^2 x v^2 product over the rows m -- for a panel
// of consecutive rows AB at a time.  Each R' element then serves four
// entries of R: (a b, c d), (b a, c d) with a minus sign, and so on, so that
// for an output block (X, Y) of Z and a contracted block pair (B, D)
//   R~[(x y), (b d)] = s(x, b) s(y, d) R'[(min max of x, b), (min max of y, d)]
// (s = +1 for x < b, -1 for x > b, 0 for x = b).  k_grad_z is an atomic-free
// GEMM in which each workgroup owns a tile of Z (128 Cholesky indices P x the
// 64 slots (x, y) of one block pair of virtual blocks (X, Y)) for a whole
// panel and runs over every (B, D) whose R' tile lies in the panel: R~ is
// gathered from the panel into LDS with its signs, the Cholesky vectors of
// block (B, D) are read straight from the staged layout, and the products
// use the 3M complex form (three real matrix-core products per complex one).
// Z lives in the staged layout of L and is finally conjugated, doubled and
// unpacked into dL (k_grad_out).
//
// Work: R' costs v^4 M / 4 complex products (M = rows), the Z products
// v^4 Nchol; the full-R route of two plain GEMMs costs v^4 (M + Nchol).
#include <algorithm>

#include "internal.hpp"
#include "panels.hpp"

namespace lrcc {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4 t; };
template <> struct Acc<float> { typedef f4 t; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Output row of accumulator item r in lane group lk (column = lane % 16):
// rows lk + 4 r for the f64 16x16x4 MFMA, 4 lk + r for the f32 one; inputs
// A[i][k], B[k][j] from lane i + 16 k, j + 16 k for both.
template <typename T> __device__ __forceinline__ int out_row(int lk, int r);
template <> __device__ __forceinline__ int out_row<double>(int lk, int r) { return lk + 4 * r; }
template <> __device__ __forceinline__ int out_row<float>(int lk, int r) { return 4 * lk + r; }

constexpr int PT = 128;  // Cholesky indices per Z tile (4 waves x 32)
constexpr int RS = NS + 1;  // padded row of the R~ tile in LDS

// ---------------------------------------------------------------------------
// R'(AB, CD) for the panel rows AB = ab0 + t / nbp, CD = t % nbp: one
// workgroup per tile, wave w the rows (a b) 16 w .. 16 w + 15, all 64 columns
// (c d); operands straight from the block layout (G and X planar,
// [plane][bp][m][64]), K = the Mp rows m in steps of 4.  Written as
// Rp[t][plane][64 (a b)][64 (c d)].
template <typename T>
__global__ __launch_bounds__(WG, 1) void k_grad_r(const T* __restrict__ Gb,
                                                  const T* __restrict__ Xb, int nbp, int Mp,
                                                  int ab0, T* __restrict__ Rp) {
  typedef typename Acc<T>::t acc_t;
  const long t = blockIdx.x;
  const int ab = ab0 + (int)(t / nbp), cd = (int)(t % nbp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const size_t plane = (size_t)nbp * Mp * NS;
  const T* gr = Gb + (size_t)ab * Mp * NS + 16 * wave + li;  // column (a b) of this lane
  const T* gi = gr + plane;
  const T* xr = Xb + (size_t)cd * Mp * NS + li;
  const T* xi = xr + plane;
  acc_t sr[4], si[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    sr[j] = acc_t{0, 0, 0, 0};
    si[j] = sr[j];
  }
  // conj(g) x = (gr xr + gi xi) + i (gr xi - gi xr)
  for (int m0 = 0; m0 < Mp; m0 += 4) {
    const size_t row = (size_t)(m0 + lk) * NS;
    const T ar = gr[row], ai = gi[row], nai = -ai;
    T br[4], bi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      br[j] = xr[row + 16 * j];
      bi[j] = xi[row + 16 * j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sr[j] = mfma(ar, br[j], sr[j]);
      si[j] = mfma(ar, bi[j], si[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sr[j] = mfma(ai, bi[j], sr[j]);
      si[j] = mfma(nai, br[j], si[j]);
    }
  }
  T* out = Rp + (size_t)t * 2 * NS * NS;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * wave + out_row<T>(lk, r), col = 16 * j + li;
      out[row * NS + col] = sr[j][r];
      out[NS * NS + row * NS + col] = si[j][r];
    }
}

// Block-pair index of blocks (p, q), p <= q.
__host__ __device__ __forceinline__ int bpair(int p, int q, int nbv) {
  return p * nbv - p * (p - 1) / 2 + (q - p);
}

// Packed slot and sign of the virtual pair (x, b) inside the block pair of
// blocks (X, B): the R' slot (min, max) and s(x, b).
__device__ __forceinline__ void slot_sign(int X, int B, int xl, int bl, int* slot, int* sign) {
  const int x = X * TB + xl, b = B * TB + bl;
  *sign = x < b ? 1 : (x > b ? -1 : 0);
  *slot = X < B || (X == B && xl < bl) ? xl * TB + bl : bl * TB + xl;
}

// Z tile (X, Y, P range pr) += sum over (B, D), {X, B} in the panel rows
// [A0, A1) x all, of L[P, (B, D)] R~((X,Y), (B,D))^T, in the 3M form.
// Workgroup: wave w the P rows 32 w .. 32 w + 31 (two 16-row blocks), all 64
// output slots (x y); K = the 64 slots (b d) of block (B, D) in steps of 4.
// Blocks of X with no contribution in this panel (X < A0) are not launched.
template <typename T>
__global__ __launch_bounds__(WG, 1) void k_grad_z(const T* __restrict__ Ls,
                                                  const T* __restrict__ Rp, int nbv, int nbp,
                                                  int ncp, int v, int A0, int A1, int ab0,
                                                  T* __restrict__ Z) {
  typedef typename Acc<T>::t acc_t;
  __shared__ T rt[2 * NS * RS];  // R~ [plane][n = (x y)][k = (b d)], rows padded
  const int npr = ncp / PT;
  const int pr = blockIdx.x % npr;
  const int XY = blockIdx.x / npr;
  const int X = A0 + XY / nbv, Y = XY % nbv;
  const int P0 = pr * PT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  acc_t t1[2][4], t2[2][4], t3[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      t1[i][j] = acc_t{0, 0, 0, 0};
      t2[i][j] = t1[i][j];
      t3[i][j] = t1[i][j];
    }
  // B with {X, B} in the panel: B >= A0 when X < A1 (then min(X, B) is in
  // [A0, A1) or is X itself), else B in [A0, A1)
  const int Bend = X < A1 ? nbv : A1;
  for (int B = A0; B < Bend; ++B) {
    const int pXB = X <= B ? bpair(X, B, nbv) : bpair(B, X, nbv);
    for (int D = 0; D < nbv; ++D) {
      const int pYD = Y <= D ? bpair(Y, D, nbv) : bpair(D, Y, nbv);
      const T* src = Rp + ((size_t)(pXB - ab0) * nbp + pYD) * 2 * NS * NS;
      __syncthreads();  // every wave is done with the previous R~
      for (int e = threadIdx.x; e < NS * NS; e += WG) {
        const int n = e >> 6, k = e & 63;
        int s1, g1, s2, g2;
        slot_sign(X, B, n >> 3, k >> 3, &s1, &g1);
        slot_sign(Y, D, n & 7, k & 7, &s2, &g2);
        const T sg = (T)(g1 * g2);
        rt[n * RS + k] = sg * src[s1 * NS + s2];
        rt[NS * RS + n * RS + k] = sg * src[NS * NS + s1 * NS + s2];
      }
      __syncthreads();
      const T* lr = Ls + ((size_t)(B * nbv + D) * ncp + P0 + 32 * wave + li) * 2 * NS;
#pragma unroll 4
      for (int k0 = 0; k0 < NS; k0 += 4) {
        const int k = k0 + lk;
        T ar[2], ai[2], as[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          ar[i] = lr[(size_t)16 * i * 2 * NS + k];
          ai[i] = lr[(size_t)16 * i * 2 * NS + NS + k];
          as[i] = ar[i] + ai[i];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = 16 * j + li;
          const T br = rt[n * RS + k], bi = rt[NS * RS + n * RS + k], bs = br + bi;
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            t1[i][j] = mfma(ar[i], br, t1[i][j]);
            t2[i][j] = mfma(ai[i], bi, t2[i][j]);
            t3[i][j] = mfma(as[i], bs, t3[i][j]);
          }
        }
      }
    }
  }
  // Z[(X, Y)][P][plane][(x y)] += (t1 - t2) + i (t3 - t1 - t2); this
  // workgroup is the only writer of its tile in this launch
  T* zr = Z + ((size_t)(X * nbv + Y) * ncp + P0 + 32 * wave) * 2 * NS;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t o = (size_t)(16 * i + out_row<T>(lk, r)) * 2 * NS + 16 * j + li;
        zr[o] += t1[i][j][r] - t2[i][j][r];
        zr[o + NS] += t3[i][j][r] - t1[i][j][r] - t2[i][j][r];
      }
}

// dL[P][a][c] = 2 conj(Z[(A, C)][P][(a c)]) in the caller's dtype.
template <typename T>
__global__ void k_grad_out(const T* __restrict__ Z, int v, int nchol, int nbv, int ncp,
                           lrcc_dtype dt, void* __restrict__ dL) {
  const long total = (long)nchol * v * v;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % v), a = (int)((e / v) % v);
    const long P = e / ((long)v * v);
    const size_t src = ((size_t)((a / TB) * nbv + c / TB) * ncp + P) * 2 * NS + (a % TB) * TB + c % TB;
    const double re = 2.0 * (double)Z[src], im = -2.0 * (double)Z[src + NS];
    if (dt == LRCC_C128) static_cast<double2*>(dL)[e] = make_double2(re, im);
    else static_cast<float2*>(dL)[e] = make_float2((float)re, (float)im);
  }
}

inline int grid_for(long n) {
  long g = (n + 255) / 256;
  return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

template <typename T>
lrcc_status grad_run(lrcc_handle h, const Geom& g0, const void* L, const void* X, const void* G,
                     void* dL, lrcc_dtype dt) {
  hipStream_t st = h->stream;
  Geom g = g0;
  g.ncp = (int)roundup(g.nchol, PT);  // staged L padded to whole P tiles
  const int nbv = g.nbv, nbp = g.nbp;
  lrcc_status s = ensure_tab(h, nbv);
  if (s != LRCC_OK) return s;
  const int* tab = h->tab.as<int>();
  const size_t es = sizeof(T);
  const size_t lsz = (size_t)nbv * nbv * g.ncp * 2 * NS * es;  // staged L, and Z
  const size_t xsz = (size_t)2 * g.xb_plane() * es;            // block-layout G or X
  LRCC_HIP(h, h->ls.ensure(lsz));
  LRCC_HIP(h, h->ls2.ensure(lsz));
  LRCC_HIP(h, h->xb.ensure(xsz));
  LRCC_HIP(h, h->gb.ensure(xsz));
  T* Ls = h->ls.as<T>();
  T* Z = h->ls2.as<T>();
  LRCC_HIP(h, stage_L<T>(L, dt, g, L_PLAIN, Ls, st));
  LRCC_HIP(h, pack_to_block<T>(X, dt, g, tab, h->xb.as<T>(), st));
  LRCC_HIP(h, pack_to_block<T>(G, dt, g, tab, h->gb.as<T>(), st));
  LRCC_HIP(h, fill_zero(Z, lsz, st));
  // panels of whole block rows A (all pairs (A, B), B >= A) within the
  // workspace limit of the bf16x3 ladder (min(16 GiB, half the free memory)
  // unless set), at least one row
  if (h->panel_cap == 0) {
    size_t freeb = 0, totalb = 0;
    LRCC_HIP(h, hipMemGetInfo(&freeb, &totalb));
    h->panel_cap = std::max<size_t>(std::min((size_t)16 << 30, freeb / 2), (size_t)64 << 20);
  }
  const size_t tile = (size_t)2 * NS * NS * es;
  // the workspace holds the first (largest) panel and no later panel is
  // larger than it
  const PanelPlan plan = plan_row_panels(nbv, (size_t)nbp * tile, h->panel_cap);
  LRCC_HIP(h, h->vws.ensure(plan.bytes));
  T* Rp = h->vws.as<T>();
  for (const auto& pr : plan.rows) {
    const int A0 = pr.first, A1 = pr.second;
    const int ab0 = bpair(A0, A0, nbv);
    const long ntile = panel_pairs(nbv, A0, A1) * nbp;
    if ((size_t)ntile * tile > h->vws.n)  // (the plan guarantees it; checked before any launch)
      return fail(h, LRCC_ERR_NOMEM, "gradient panel exceeds its workspace");
    if (ntile > 0x7fffffffL) return fail(h, LRCC_ERR_SHAPE, "gradient panel too large");
    hipLaunchKernelGGL((k_grad_r<T>), dim3((unsigned)ntile), dim3(WG), 0, st, h->gb.as<T>(),
                       h->xb.as<T>(), nbp, (int)g.Mp, ab0, Rp);
    LRCC_HIP(h, hipGetLastError());
    const long nz = (long)(nbv - A0) * nbv * (g.ncp / PT);
    if (nz > 0x7fffffffL) return fail(h, LRCC_ERR_SHAPE, "gradient grid too large");
    hipLaunchKernelGGL((k_grad_z<T>), dim3((unsigned)nz), dim3(WG), 0, st, Ls, Rp, nbv, nbp,
                       g.ncp, g.v, A0, A1, ab0, Z);
    LRCC_HIP(h, hipGetLastError());
  }
  hipLaunchKernelGGL((k_grad_out<T>), dim3(grid_for((long)g.nchol * g.v * g.v)), dim3(256), 0, st,
                     Z, g.v, g.nchol, nbv, g.ncp, dt, dL);
  LRCC_HIP(h, hipGetLastError());
  return LRCC_OK;
}

}  // namespace

lrcc_status grad_L(lrcc_handle h, const Geom& g, const void* L, const void* X, const void* G,
                   void* dL, lrcc_dtype dt) {
  const size_t es = dt == LRCC_C128 ? 16 : 8;
  const size_t nl = (size_t)g.nchol * g.v * g.v;
  if (nl == 0) return LRCC_OK;
  if (g.M == 0 || g.npv == 0) {  // sigma does not depend on L: zero gradient
    LRCC_HIP(h, fill_zero(dL, nl * es, h->stream));
    return LRCC_OK;
  }
  // complex128: FP64 arithmetic; complex64: FP32
  return dt == LRCC_C128 ? grad_run<double>(h, g, L, X, G, dL, dt)
                         : grad_run<float>(h, g, L, X, G, dL, dt);
}

}  // namespace lrcc
