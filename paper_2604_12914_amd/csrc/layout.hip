// Staging and layout kernels: packed <-> block-pair layout, Cholesky
// vectors -> planar 8x8 blocks.  All are HBM-bound streaming kernels with one
// thread per output element of the block layout.
#include <algorithm>

#include "internal.hpp"

namespace lrcc {

namespace {

template <typename T> struct Cx;
template <> struct Cx<double> { typedef double2 t; };
template <> struct Cx<float> { typedef float2 t; };

__device__ inline double2 load_c(const void* p, lrcc_dtype dt, size_t i) {
  if (dt == LRCC_C128) return static_cast<const double2*>(p)[i];
  float2 f = static_cast<const float2*>(p)[i];
  return make_double2(f.x, f.y);
}

__device__ inline void store_c(void* p, lrcc_dtype dt, size_t i, double re, double im) {
  if (dt == LRCC_C128) static_cast<double2*>(p)[i] = make_double2(re, im);
  else static_cast<float2*>(p)[i] = make_float2((float)re, (float)im);
}

// Packed index of the pair p<q among n indices (row-major upper triangle).
__device__ inline long pidx(long p, long q, long n) { return p * (2 * n - p - 1) / 2 + (q - p - 1); }

template <typename T>
__global__ void k_stage_L(const void* __restrict__ L, lrcc_dtype dt, int v, int nchol,
                          int nbv, int ncp, int form, T* __restrict__ Ls) {
  // one thread per (block A, block C, P, slot)
  const long total = (long)nbv * nbv * ncp * NS;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int s = e % NS;
    const long r = e / NS;
    const int P = r % ncp;
    const long blk = r / ncp;
    const int C = blk % nbv, A = blk / nbv;
    const int a = A * TB + s / TB, c = C * TB + s % TB;
    double re = 0.0, im = 0.0;
    if (a < v && c < v && P < nchol) {
      // (L^H)^P_ac = conj(L^P_ca)
      const size_t src = form != L_PLAIN ? ((size_t)P * v + c) * v + a : ((size_t)P * v + a) * v + c;
      double2 z = load_c(L, dt, src);
      re = z.x;
      im = form == L_ADJ ? -z.y : z.y;
    }
    T* dst = Ls + (r * 2) * NS + s;
    dst[0] = (T)re;
    dst[NS] = (T)im;
  }
}

template <typename T>
__global__ void k_pack_to_block(const void* __restrict__ X, lrcc_dtype dt, int v, long npv,
                                long M, long Mp, int nbp, const int* __restrict__ tab,
                                T* __restrict__ Xb) {
  const long plane = (long)nbp * Mp * NS;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < plane;
       e += (long)gridDim.x * blockDim.x) {
    const int s = e % NS;
    const long m = (e / NS) % Mp;
    const int bp = e / (NS * Mp);
    const int AB = tab[bp];
    const int a = (AB >> 16) * TB + s / TB, b = (AB & 0xffff) * TB + s % TB;
    double re = 0.0, im = 0.0;
    if (a < b && b < v && m < M) {
      double2 z = load_c(X, dt, (size_t)m * npv + pidx(a, b, v));
      re = z.x;
      im = z.y;
    }
    Xb[e] = (T)re;
    Xb[e + plane] = (T)im;
  }
}

template <typename T>
__global__ void k_block_to_pack(const T* __restrict__ Sb, int v, long npv, long M, long Mp,
                                int nbp, const int* __restrict__ tab, void* __restrict__ S,
                                lrcc_dtype dt) {
  const long plane = (long)nbp * Mp * NS;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < plane;
       e += (long)gridDim.x * blockDim.x) {
    const int s = e % NS;
    const long m = (e / NS) % Mp;
    const int bp = e / (NS * Mp);
    const int AB = tab[bp];
    const int a = (AB >> 16) * TB + s / TB, b = (AB & 0xffff) * TB + s % TB;
    if (a < b && b < v && m < M)
      store_c(S, dt, (size_t)m * npv + pidx(a, b, v), (double)Sb[e], (double)Sb[e + plane]);
  }
}

// One pass over L comparing L^P_ac with conj L^P_ca for a <= c; a wave that
// finds a mismatch stores 1 (a plain store: every writer writes the same).
__global__ void k_herm_check(const void* __restrict__ L, lrcc_dtype dt, int v, long n,
                             int* __restrict__ nonherm) {
  bool bad = false;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    const int c = e % v, a = (e / v) % v;
    if (a > c) continue;
    const double2 z = load_c(L, dt, e);
    const double2 w = load_c(L, dt, e + (long)(c - a) * (v - 1));  // element (c, a)
    bad = bad || !(z.x == w.x && z.y == -w.y);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) *nonherm = 1;
}

__global__ void k_zero(uint4* p, size_t n16) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_zero8(uint2* p, size_t n8) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n8;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint2(0, 0);
}

inline int grid_for(long n) {
  long g = (n + 255) / 256;
  return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

}  // namespace

template <typename T>
hipError_t stage_L(const void* L, lrcc_dtype dt, const Geom& g, LForm form,
                   T* Ls, hipStream_t st) {
  const long total = (long)g.nbv * g.nbv * g.ncp * NS;
  hipLaunchKernelGGL(k_stage_L<T>, dim3(grid_for(total)), dim3(256), 0, st, L, dt, g.v,
                     g.nchol, g.nbv, g.ncp, (int)form, Ls);
  return hipGetLastError();
}

template <typename T>
hipError_t pack_to_block(const void* X, lrcc_dtype dt, const Geom& g, const int* tab, T* Xb,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_pack_to_block<T>, dim3(grid_for(g.xb_plane())), dim3(256), 0, st, X,
                     dt, g.v, g.npv, g.M, g.Mp, g.nbp, tab, Xb);
  return hipGetLastError();
}

template <typename T>
hipError_t block_to_pack(const T* Sb, const Geom& g, const int* tab, void* S, lrcc_dtype dt,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_block_to_pack<T>, dim3(grid_for(g.xb_plane())), dim3(256), 0, st, Sb,
                     g.v, g.npv, g.M, g.Mp, g.nbp, tab, S, dt);
  return hipGetLastError();
}

// Zero a device buffer with a fill kernel (a plain kernel node stays valid
// under graph capture, unlike a memset node).
// Zeroes with a kernel (no memset node, so a caller may capture it): 16-byte
// stores where p and bytes allow, else 8-byte ones; hipErrorInvalidValue for
// other sizes or alignments.
hipError_t fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  if (bytes % 16 == 0 && a % 16 == 0)
    hipLaunchKernelGGL(k_zero, dim3(grid_for((long)(bytes / 16))), dim3(256), 0, st,
                       static_cast<uint4*>(p), bytes / 16);
  else if (bytes % 8 == 0 && a % 8 == 0)
    hipLaunchKernelGGL(k_zero8, dim3(grid_for((long)(bytes / 8))), dim3(256), 0, st,
                       static_cast<uint2*>(p), bytes / 8);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t herm_check(const void* L, lrcc_dtype dt, int v, int nchol, int* nonherm,
                      hipStream_t st) {
  hipError_t e = fill_zero(nonherm, 16, st);
  if (e != hipSuccess) return e;
  const long n = (long)nchol * v * v;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_herm_check, dim3(std::min(grid_for(n), 4096)), dim3(256), 0, st, L, dt,
                     v, n, nonherm);
  return hipGetLastError();
}

template hipError_t stage_L<double>(const void*, lrcc_dtype, const Geom&, LForm, double*,
                                    hipStream_t);
template hipError_t stage_L<float>(const void*, lrcc_dtype, const Geom&, LForm, float*,
                                   hipStream_t);
template hipError_t pack_to_block<double>(const void*, lrcc_dtype, const Geom&, const int*,
                                          double*, hipStream_t);
template hipError_t pack_to_block<float>(const void*, lrcc_dtype, const Geom&, const int*,
                                         float*, hipStream_t);
template hipError_t block_to_pack<double>(const double*, const Geom&, const int*, void*,
                                          lrcc_dtype, hipStream_t);
template hipError_t block_to_pack<float>(const float*, const Geom&, const int*, void*,
                                         lrcc_dtype, hipStream_t);

}  // namespace lrcc
