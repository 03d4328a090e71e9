// Fused particle-particle-ladder kernel for gfx950 (FP64 and FP32 MFMA).
//
// One workgroup (4 waves) owns one tile pair (AB, CD) of virtual block pairs
// with bp(AB) <= bp(CD) and does, without leaving the CU:
//   1. build   W1[(a,c),(b,d)] = sum_P L^P_ac L^P_bd   (a in A, c in C, b in B, d in D)
//              W2[(a,d),(b,c)] = sum_P L^P_ad L^P_bc
//      as two 64 x 64 complex GEMMs over the Cholesky index on the matrix
//      cores (16x16x4 MFMA, complex product in 4M form), operands streamed
//      through LDS in chunks of KC vectors;
//   2. antisymmetrise in LDS: V[(ab),(cd)] = 2 (W1 - W2) = 2 <ab||cd>, dead
//      slots zeroed (the 2 turns the unrestricted c,d sum into the packed
//      c<d sum);
//   3. contract   sigma[m, ab] += sum_cd X[m, cd] V[ab, cd] for every row m,
//      on the matrix cores, and add the 64-slot partial sums to the block-
//      layout accumulator with device-scope atomics;
//   4. for AB != CD, the mirror tile (CD, AB): when every L^P is Hermitian
//      (L^P_ca = conj L^P_ac) the ladder operator is Hermitian,
//      V[cd, ab] = conj V[ab, cd], and the same LDS tile is contracted a
//      second time, transposed and conjugated, into sigma[:, CD] (half the
//      integral builds); otherwise the mirror tile is built and contracted
//      like the first.  A flag written by the staging pass on the device
//      selects the branch, so the launch needs no host round trip.
// The integral tile never reaches HBM.
#include <cstdlib>

#include "internal.hpp"

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

// Output row of accumulator item r in lane group lk (column = lane % 16).
// The f64 16x16x4 MFMA interleaves rows across lane groups (row lk + 4r);
// the f32 one keeps them together (row 4 lk + r).  Inputs: A[i][k] and
// B[k][j] come from lane i + 16 k and j + 16 k for both.
template <typename T> __device__ __forceinline__ int out_row(int lk, int r);
template <> __device__ __forceinline__ int out_row<double>(int lk, int r) { return lk + 4 * r; }
template <> __device__ __forceinline__ int out_row<float>(int lk, int r) { return 4 * lk + r; }

template <typename T> struct Vec16;
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));
template <> struct Vec16<double> { typedef dv2 t; static constexpr int n = 2; };
template <> struct Vec16<float> { typedef fv4 t; static constexpr int n = 4; };

__device__ __forceinline__ void atomic_add(double* p, double x) { unsafeAtomicAdd(p, x); }
__device__ __forceinline__ void atomic_add(float* p, float x) { unsafeAtomicAdd(p, x); }

// Row stride of the V tile in LDS: one element of padding makes both the
// row-wise reads of the first contraction and the column-wise reads of the
// mirror contraction (and the antisymmetrisation stores) conflict-free.
constexpr int VS = NS + 1;

// LDS bytes: 4 blocks x KC vectors x 2 planes x 64 of T; the 64 x 64 complex
// V tile (2 planes x 64 x VS of T) reuses the same space after the build.
template <typename T, int KC>
struct Smem {
  static constexpr int chunk = 2 * NS * KC;        // elements of one block's chunk
  static constexpr int build = 4 * chunk;
  static constexpr int vtile = 2 * NS * VS;
  static constexpr int elems = build > vtile ? build : vtile;
};

// Integral tile of block pairs (ab, cd): V[(ab),(cd)] = 2 <ab||cd>, built on
// the matrix cores (4M form) and left in LDS as V[cd slot * VS + ab slot]
// (planes re, im).  Ends with a barrier: every wave may read V.  NW waves:
// wave w builds rows 16 (w mod 4) .. + 15 of W1 and W2 and, with 8 waves,
// half of the 64 columns (two waves per SIMD, half the accumulators each).
template <typename T, int KC, int OCC, bool DL, int NW>
__device__ __forceinline__ void build_v_4m(const T* __restrict__ Ls, const int* __restrict__ tab,
                                           int nbv, int ncp, int v, int ab, int cd, T* lds) {
  typedef typename Acc<T>::t acc_t;
  typedef typename Vec16<T>::t vec_t;
  constexpr int VN = Vec16<T>::n;
  constexpr int CH = Smem<T, KC>::chunk;
  const int pAB = tab[ab], pCD = tab[cd];
  const int A = pAB >> 16, B = pAB & 0xffff, C = pCD >> 16, D = pCD & 0xffff;

  static_assert(NW == 4 || (NW == 8 && DL), "eight waves load chunks straight into LDS");
  constexpr int NJ = 16 / NW;  // 16-column blocks per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rw = wave & 3, j0 = (wave >> 2) * NJ;

  // ---- 1. build W1 (rows (a,c) of this wave, its columns (b,d)) and W2 ----
  const size_t bstride = (size_t)ncp * 2 * NS;
  const T* const gblk[4] = {Ls + (size_t)(A * nbv + C) * bstride,
                            Ls + (size_t)(B * nbv + D) * bstride,
                            Ls + (size_t)(A * nbv + D) * bstride,
                            Ls + (size_t)(B * nbv + C) * bstride};

  acc_t w1r[NJ], w1i[NJ], w2r[NJ], w2i[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    w1r[j] = acc_t{0, 0, 0, 0};
    w1i[j] = w1r[j];
    w2r[j] = w1r[j];
    w2i[j] = w1r[j];
  }

  // chunk of KC vectors of the four blocks: contiguous runs of CH elements.
  // DL = false: prefetched into registers one chunk ahead of the MFMA work,
  // then stored to LDS.  DL = true: loaded straight into LDS (1 KB per wave
  // instruction, lane i's 16 bytes at offset 16 i); with one workgroup per
  // CU a two-chunk ring overlaps the next chunk's load with this chunk's
  // MFMAs, with two workgroups per CU the other workgroup covers the wait.
  constexpr int nvec = 4 * CH / VN;
  constexpr int NPF = DL ? 1 : nvec / WG;  // vectors per thread per chunk
  constexpr int KPB = CH / VN / WG;        // of which per block
  static_assert(DL || NPF == 4 * KPB, "chunk must split evenly over the workgroup");
  constexpr int PPB = CH * (int)sizeof(T) / 1024;  // 1 KB pieces per block chunk
  static_assert(!DL || (PPB % NW == 0), "direct loads need whole pieces per wave");
  vec_t pf[NPF];
  auto fetch = [&](int p0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const vec_t* src = reinterpret_cast<const vec_t*>(gblk[q] + (size_t)p0 * 2 * NS);
#pragma unroll
      for (int k = 0; k < KPB; ++k) pf[q * KPB + k] = src[k * WG + threadIdx.x];
    }
  };
  auto issue = [&](int p0, T* buf) {
#pragma unroll
    for (int k = 0; k < 4 * PPB / NW; ++k) {  // block q, piece wave + NW m
      const int q = k / (PPB / NW), pb = wave + NW * (k % (PPB / NW));
      const char* src = reinterpret_cast<const char*>(gblk[q] + (size_t)p0 * 2 * NS) +
                        pb * 1024 + lane * 16;
      __builtin_amdgcn_global_load_lds(
          src, (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(buf + q * CH) +
                                                         pb * 1024),
          16, 0, 0);
    }
  };
  T* const ring0 = lds;
  T* const ring1 = lds + (DL && OCC == 1 ? 4 * CH : 0);
  __syncthreads();  // LDS may still hold the V tile of a previous contraction
  if (DL && OCC == 1) issue(0, ring0);
  if (!DL) fetch(0);
  for (int p0 = 0, c = 0; p0 < ncp; p0 += KC, ++c) {
    T* cur = lds;
    if (DL && OCC == 1) {
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this chunk has landed
      __syncthreads();                     // every wave: loads landed, previous chunk done
      cur = (c & 1) ? ring1 : ring0;
      // the next chunk (the last one again on the last pass: a branch-free
      // loop body keeps the accumulators in place across iterations)
      issue(min(p0 + KC, ncp - KC), (c & 1) ? ring0 : ring1);
    } else if (DL) {
      __syncthreads();
      issue(p0, lds);
      __builtin_amdgcn_s_waitcnt(0x0F70);
      __syncthreads();
    } else {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int k = 0; k < KPB; ++k)
          reinterpret_cast<vec_t*>(lds + q * CH)[k * WG + threadIdx.x] = pf[q * KPB + k];
      }
      __syncthreads();
      fetch(min(p0 + KC, ncp - KC));  // branch-free, as above
    }
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int p = 4 * ks + lk;  // vector within the chunk used by this lane
      const T* lac = cur + 0 * CH + p * 2 * NS;
      const T* lbd = cur + 1 * CH + p * 2 * NS;
      const T* lad = cur + 2 * CH + p * 2 * NS;
      const T* lbc = cur + 3 * CH + p * 2 * NS;
      const T acr = lac[16 * rw + li], aci = lac[NS + 16 * rw + li];
      const T adr = lad[16 * rw + li], adi = lad[NS + 16 * rw + li];
      T bdr[NJ], bdi[NJ], bcr[NJ], bci[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        bdr[j] = lbd[16 * (j0 + j) + li];
        bdi[j] = lbd[NS + 16 * (j0 + j) + li];
        bcr[j] = lbc[16 * (j0 + j) + li];
        bci[j] = lbc[NS + 16 * (j0 + j) + li];
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        w1r[j] = mfma(acr, bdr[j], w1r[j]);
        w1i[j] = mfma(acr, bdi[j], w1i[j]);
        w2r[j] = mfma(adr, bcr[j], w2r[j]);
        w2i[j] = mfma(adr, bci[j], w2i[j]);
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        w1r[j] = mfma(-aci, bdi[j], w1r[j]);
        w1i[j] = mfma(aci, bdr[j], w1i[j]);
        w2r[j] = mfma(-adi, bci[j], w2r[j]);
        w2i[j] = mfma(adi, bcr[j], w2i[j]);
      }
    }
  }
  if (DL && OCC == 1) __builtin_amdgcn_s_waitcnt(0x0F70);  // the spare load has landed
  __syncthreads();  // every wave is done with the chunk buffers

  // ---- 2. antisymmetrise into V[cd][ab] (planar) in LDS --------------------
  T* Vr = lds;
  T* Vi = lds + NS * VS;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rw + out_row<T>(lk, r), jj = 16 * (j0 + j) + li;
      // W1 element: i = (a_l, c_l), jj = (b_l, d_l)
      const int idx = ((i & 7) * TB + (jj & 7)) * VS + (i >> 3) * TB + (jj >> 3);
      Vr[idx] = (T)2 * w1r[j][r];
      Vi[idx] = (T)2 * w1i[j][r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rw + out_row<T>(lk, r), jj = 16 * (j0 + j) + li;
      // W2 element: i = (a_l, d_l), jj = (b_l, c_l)
      const int al = i >> 3, dl = i & 7, bl = jj >> 3, cl = jj & 7;
      const int idx = (cl * TB + dl) * VS + al * TB + bl;
      const bool live = (A < B || al < bl) && (B * TB + bl < v) && (C < D || cl < dl) &&
                        (D * TB + dl < v);
      Vr[idx] = live ? Vr[idx] - (T)2 * w2r[j][r] : (T)0;
      Vi[idx] = live ? Vi[idx] - (T)2 * w2i[j][r] : (T)0;
    }
  }
  __syncthreads();
}

// Contraction of 16 rows m0 .. m0 + 15 (this lane holds X[m0 + li][16 lk + s]
// in xr[s], xi[s]) with NN column blocks n0 .. n0 + NN - 1 of the LDS tile V
// into the accumulators sr, si (see contract_v for TR).  CM3: the 3M form,
// three real products per complex product (t1 = xr vr, t2 = xi vi,
// t3 = (xr + xi)(vr +- vi), the sums formed in registers), combined into
// sr, si at the end.
template <typename T, bool TR, int NN, bool CM3>
__device__ __forceinline__ void contract_rows(const T* Vr, const T* Vi, const T (&xr)[16],
                                              const T (&xi)[16], int n0,
                                              typename Acc<T>::t (&sr)[NN],
                                              typename Acc<T>::t (&si)[NN]) {
  typedef typename Acc<T>::t acc_t;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  if constexpr (CM3) {
    acc_t t1[NN], t2[NN], t3[NN];
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      t1[n] = acc_t{0, 0, 0, 0};
      t2[n] = t1[n];
      t3[n] = t1[n];
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k = 16 * lk + s;  // contracted slot fed by this lane at step s
      T vr[NN], vi[NN];
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        const int c = 16 * (n0 + n) + li;
        const int a = TR ? c * VS + k : k * VS + c;
        vr[n] = Vr[a];
        vi[n] = Vi[a];
      }
      const T xrs = xr[s], xis = xi[s], xs = xrs + xis;
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        t1[n] = mfma(xrs, vr[n], t1[n]);
        t2[n] = mfma(xis, vi[n], t2[n]);
        t3[n] = mfma(xs, TR ? vr[n] - vi[n] : vr[n] + vi[n], t3[n]);
      }
      // (three accumulator sets: a shorter look-ahead than in the 4M form)
      if (s & 1) __builtin_amdgcn_sched_barrier(0);
    }
    // (xr + i xi)(vr + i vi) = (t1 - t2) + i (t3 - t1 - t2); for the mirror
    // (xr + i xi)(vr - i vi) = (t1 + t2) + i (t3 - t1 + t2)
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      sr[n] = TR ? t1[n] + t2[n] : t1[n] - t2[n];
      si[n] = TR ? t3[n] - t1[n] + t2[n] : t3[n] - t1[n] - t2[n];
    }
  } else {
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      sr[n] = acc_t{0, 0, 0, 0};
      si[n] = sr[n];
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k = 16 * lk + s;  // contracted slot fed by this lane at step s
      T vr[NN], vi[NN];
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        const int c = 16 * (n0 + n) + li;
        const int a = TR ? c * VS + k : k * VS + c;
        vr[n] = Vr[a];
        vi[n] = Vi[a];
      }
      // (xr + i xi)(vr + i vi), or (xr + i xi)(vr - i vi) for the mirror
      const T xrs = xr[s], xis = xi[s];
      const T s_r = TR ? xis : -xis, s_i = TR ? -xrs : xrs;
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        sr[n] = mfma(xrs, vr[n], sr[n]);
        si[n] = mfma(s_i, vi[n], si[n]);
      }
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        sr[n] = mfma(s_r, vi[n], sr[n]);
        si[n] = mfma(xis, vr[n], si[n]);
      }
      // keep the scheduler from hoisting every step's LDS reads to the top
      // (that would hold 16 steps of V operands in registers at once)
      if ((s & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Add the accumulators of rows m0 .. m0 + 15, column blocks n0 .. n0 + NN - 1
// to sigma with device-scope atomics.
template <typename T, typename TA, int NN>
__device__ __forceinline__ void store_rows(const typename Acc<T>::t (&sr)[NN],
                                           const typename Acc<T>::t (&si)[NN], int n0, int m0,
                                           TA* sr_g, TA* si_g) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int n = 0; n < NN; ++n) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const size_t o = (size_t)(m0 + out_row<T>(lk, r)) * NS + 16 * (n0 + n) + li;
      atomic_add(sr_g + o, (TA)sr[n][r]);
      atomic_add(si_g + o, (TA)si[n][r]);
    }
  }
}

// Contraction of the LDS tile V of block pairs (x, y) with the rows of X:
//   TR = false:  sigma[m, x slots] += sum_k X[m, y slot k] V[x, k]
//   TR = true:   sigma[m, y slots] += sum_k X[m, x slot k] conj V[k, y]
// (the second is the mirror tile (y, x) of a Hermitian operator).  src / dst
// are the block pairs whose X rows are read and whose sigma rows receive the
// 64-slot partial sums (device-scope atomics).  V is only read.  Chunks of 16
// rows go to the NW waves in turn; the last Mp/16 mod NW chunks are split into
// (chunk, 16-column block) items dealt out to all waves, so no wave does an
// extra whole chunk.
template <typename T, typename TA, int OCC, bool TR, int NW, bool CM3>
__device__ __forceinline__ void contract_v(const T* lds, const T* __restrict__ Xb,
                                           TA* __restrict__ Sb, int nbp, int Mp, int src,
                                           int dst) {
  typedef typename Vec16<T>::t vec_t;
  constexpr int VN = Vec16<T>::n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const T* Vr = lds;
  const T* Vi = lds + NS * VS;
  const size_t plane = (size_t)nbp * Mp * NS;
  const T* xr_g = Xb + (size_t)src * Mp * NS;
  const T* xi_g = xr_g + plane;
  TA* sr_g = Sb + (size_t)dst * Mp * NS;
  TA* si_g = sr_g + plane;
  const int nch = Mp / 16, nfull = nch - nch % NW;
  // lane (row li, group lk) holds X[m0+li][16 lk .. 16 lk + 15]; the rows of
  // the next m-chunk are fetched while this one is contracted
  constexpr int NX = 16 / VN;
  vec_t xpr[NX], xpi[NX];
  auto fetch_x = [&](int m0) {
    const vec_t* pr = reinterpret_cast<const vec_t*>(xr_g + (size_t)(m0 + li) * NS + 16 * lk);
    const vec_t* pi = reinterpret_cast<const vec_t*>(xi_g + (size_t)(m0 + li) * NS + 16 * lk);
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      xpr[k] = pr[k];
      xpi[k] = pi[k];
    }
  };
  auto unpack = [&](T (&xr)[16], T (&xi)[16]) {
#pragma unroll
    for (int k = 0; k < NX; ++k) {
#pragma unroll
      for (int t = 0; t < VN; ++t) {
        xr[k * VN + t] = xpr[k][t];
        xi[k * VN + t] = xpi[k][t];
      }
    }
  };
  // With one wave per SIMD the next rows are requested before the matrix
  // work (prefetch).  With two (two workgroups per CU, or eight waves) the
  // other wave covers the load latency and registers are scarce, so they are
  // requested after it, but still before this chunk's atomics: the vector-
  // memory counter retires in order, and a load issued after the atomics
  // would wait for their round trip too.
  constexpr bool PF = OCC == 1 && NW == 4;
  typedef typename Acc<T>::t acc_t;
  const int ntail = (nch - nfull) * 4;  // (chunk, column block) items of the tail
  auto tail_m0 = [&](int it) { return (nfull + it / 4) * 16; };
  // rows of this wave's next item after main chunk mc (-1: none)
  auto next_main = [&](int mc) {
    return mc + NW < nfull ? (mc + NW) * 16 : (wave < ntail ? tail_m0(wave) : -1);
  };
  if (wave < nfull) fetch_x(wave * 16);
  else if (wave < ntail) fetch_x(tail_m0(wave));
  for (int mc = wave; mc < nfull; mc += NW) {
    const int m0 = mc * 16;
    T xr[16], xi[16];
    unpack(xr, xi);
    const int nm = next_main(mc);
    if (PF && nm >= 0) fetch_x(nm);
    if constexpr (CM3) {
      // two passes of two column blocks (three accumulator sets each), both
      // before the next rows are requested, so those rows and this chunk's
      // X operands are never live together
      acc_t sr0[2], si0[2], sr1[2], si1[2];
      contract_rows<T, TR, 2, true>(Vr, Vi, xr, xi, 0, sr0, si0);
      contract_rows<T, TR, 2, true>(Vr, Vi, xr, xi, 2, sr1, si1);
      if (!PF && nm >= 0) fetch_x(nm);
      store_rows<T, TA, 2>(sr0, si0, 0, m0, sr_g, si_g);
      store_rows<T, TA, 2>(sr1, si1, 2, m0, sr_g, si_g);
    } else {
      acc_t sr[4], si[4];
      contract_rows<T, TR, 4, false>(Vr, Vi, xr, xi, 0, sr, si);
      if (!PF && nm >= 0) fetch_x(nm);
      store_rows<T, TA, 4>(sr, si, 0, m0, sr_g, si_g);
    }
  }
  for (int it = wave; it < ntail; it += NW) {
    const int m0 = tail_m0(it);
    T xr[16], xi[16];
    unpack(xr, xi);
    acc_t sr[1], si[1];
    contract_rows<T, TR, 1, CM3>(Vr, Vi, xr, xi, it % 4, sr, si);
    if (it + NW < ntail) fetch_x(tail_m0(it + NW));
    store_rows<T, TA, 1>(sr, si, it % 4, m0, sr_g, si_g);
  }
}

// Work item w of a ladder launch over the ntile tile pairs (ab, cd), ab <= cd,
// listed by `order`: items [0, ntile) build tile (ab, cd), contract it into
// sigma[:, AB] and, for a Hermitian operator, its conjugate transpose into
// sigma[:, CD]; items [ntile, 2 ntile) build the mirror tiles (cd, ab) of a
// non-Hermitian operator (nothing to do for a Hermitian one or ab = cd).
// Returns false for an empty item (uniform over the workgroup).
__device__ __forceinline__ bool decode_item(const int* __restrict__ order, long ntile, int nbp,
                                            long w, bool nonherm, int* x, int* y,
                                            bool* mirror) {
  const bool second = w >= ntile;
  if (second && !nonherm) return false;
  const int tile = order[second ? w - ntile : w];
  const int ab = tile / nbp, cd = tile - ab * nbp;
  if (second && ab == cd) return false;
  *x = second ? cd : ab;
  *y = second ? ab : cd;
  *mirror = !nonherm && ab != cd;
  return true;
}

template <typename T, typename TA, int OCC, int NW, bool CM3, typename Build>
__device__ __forceinline__ void tile_item(Build build, const T* __restrict__ Xb,
                                          TA* __restrict__ Sb, int nbp, int Mp, int x, int y,
                                          bool mirror, T* lds) {
  build(x, y);
  contract_v<T, TA, OCC, false, NW, CM3>(lds, Xb, Sb, nbp, Mp, y, x);
  if (mirror) contract_v<T, TA, OCC, true, NW, CM3>(lds, Xb, Sb, nbp, Mp, x, y);
}

template <typename T, typename TA, int KC, int OCC, bool DL, int NW>
__global__ __launch_bounds__(64 * NW, OCC) void k_ppl_4m(const T* __restrict__ Ls,
                                                    const T* __restrict__ Xb,
                                                    TA* __restrict__ Sb,
                                                    const int* __restrict__ tab,
                                                    const int* __restrict__ order,
                                                    const int* __restrict__ nonherm, int nbv,
                                                    int nbp, int ncp, int Mp, int v) {
  constexpr int NE = (DL && OCC == 1) ? 2 * Smem<T, KC>::build : Smem<T, KC>::elems;
  __shared__ __attribute__((aligned(16))) T lds[NE > Smem<T, KC>::elems ? NE : Smem<T, KC>::elems];
  int x, y;
  bool mirror;
  if (!decode_item(order, (long)nbp * (nbp + 1) / 2, nbp, blockIdx.x, *nonherm != 0, &x, &y,
                   &mirror))
    return;
  tile_item<T, TA, OCC, NW, false>(
      [&](int p, int q) { build_v_4m<T, KC, OCC, DL, NW>(Ls, tab, nbv, ncp, v, p, q, lds); },
      Xb, Sb, nbp, Mp, x, y, mirror, lds);
}

// 3M form of the integral build: from the staged planes (re, im) of the
// Cholesky blocks, T1 = sum ar br, T2 = sum ai bi, T3 = sum (ar+ai)(br+bi)
// (the sums formed in registers) give re = T1 - T2 and im = T3 - T1 - T2:
// three real MFMA products per complex product instead of four.  The
// contraction that follows it uses the 3M form as well (contract_rows).
template <typename T, int KC, bool DL, int NW>
__device__ __forceinline__ void build_v_3m(const T* __restrict__ Ls, const int* __restrict__ tab,
                                           int nbv, int ncp, int v, int ab, int cd, T* lds) {
  typedef typename Acc<T>::t acc_t;
  typedef typename Vec16<T>::t vec_t;
  constexpr int VN = Vec16<T>::n;
  constexpr int CH = Smem<T, KC>::chunk;
  static_assert(NW == 4 || (NW == 8 && DL), "eight waves load chunks straight into LDS");
  constexpr int NJ = 16 / NW;  // 16-column blocks per wave
  const int pAB = tab[ab], pCD = tab[cd];
  const int A = pAB >> 16, B = pAB & 0xffff, C = pCD >> 16, D = pCD & 0xffff;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rw = wave & 3, j0 = (wave >> 2) * NJ;

  const size_t bstride = (size_t)ncp * 2 * NS;
  const T* const g0 = Ls + (size_t)(A * nbv + C) * bstride;
  const T* const g1 = Ls + (size_t)(B * nbv + D) * bstride;
  const T* const g2 = Ls + (size_t)(A * nbv + D) * bstride;
  const T* const g3 = Ls + (size_t)(B * nbv + C) * bstride;
  acc_t t1[2][NJ], t2[2][NJ], t3[2][NJ];  // [W1 / W2][column block]
#pragma unroll
  for (int w = 0; w < 2; ++w)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      t1[w][j] = acc_t{0, 0, 0, 0};
      t2[w][j] = t1[w][j];
      t3[w][j] = t1[w][j];
    }
  // DL = false: chunks prefetched through registers one ahead; DL = true:
  // loaded straight into a two-chunk LDS ring (1 KB per wave instruction)
  constexpr int KPB = DL ? 1 : CH / VN / WG;
  static_assert(DL || KPB * VN * WG == CH, "chunk must split evenly over the workgroup");
  constexpr int PPB = CH * (int)sizeof(T) / 1024;  // 1 KB pieces per block chunk
  static_assert(!DL || (CH * (int)sizeof(T)) % 1024 == 0, "whole pieces per block");
  static_assert(!DL || (4 * PPB) % NW == 0, "whole pieces per wave");
  vec_t pf[4 * KPB];
  auto fetch = [&](int p0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T* gq = q == 0 ? g0 : q == 1 ? g1 : q == 2 ? g2 : g3;
      const vec_t* src = reinterpret_cast<const vec_t*>(gq + (size_t)p0 * 2 * NS);
#pragma unroll
      for (int k = 0; k < KPB; ++k) pf[q * KPB + k] = src[k * WG + threadIdx.x];
    }
  };
  auto issue = [&](int p0, T* buf) {
#pragma unroll
    for (int k = 0; k < 4 * PPB / NW; ++k) {
      const int gp = k * NW + wave, q = gp / PPB, pb = gp - q * PPB;
      const T* gq = q == 0 ? g0 : q == 1 ? g1 : q == 2 ? g2 : g3;
      __builtin_amdgcn_global_load_lds(
          reinterpret_cast<const char*>(gq + (size_t)p0 * 2 * NS) + pb * 1024 + lane * 16,
          (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(buf + q * CH) +
                                                    pb * 1024),
          16, 0, 0);
    }
  };
  T* const ring0 = lds;
  T* const ring1 = lds + (DL ? 4 * CH : 0);
  __syncthreads();  // LDS may still hold the V tile of a previous contraction
  if (DL) issue(0, ring0);
  else fetch(0);
  for (int p0 = 0, c = 0; p0 < ncp; p0 += KC, ++c) {
    T* cur = lds;
    if (DL) {
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this chunk has landed
      __syncthreads();                     // every wave: loads landed, previous chunk done
      cur = (c & 1) ? ring1 : ring0;
      issue(min(p0 + KC, ncp - KC), (c & 1) ? ring0 : ring1);  // branch-free: last again
    } else {
      __syncthreads();  // previous chunk no longer read
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < KPB; ++k)
          reinterpret_cast<vec_t*>(lds + q * CH)[k * WG + threadIdx.x] = pf[q * KPB + k];
      __syncthreads();
      fetch(min(p0 + KC, ncp - KC));
    }
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int p = 4 * ks + lk;
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        // W1: rows from L_AC (block 0), columns from L_BD (block 1);
        // W2: rows from L_AD (block 2), columns from L_BC (block 3)
        const T* la = cur + (2 * w) * CH + p * 2 * NS + 16 * rw + li;
        const T* lb = cur + (2 * w + 1) * CH + p * 2 * NS + 16 * j0 + li;
        // the third operand of each side, re + im, formed in registers
        const T a0 = la[0], a1 = la[NS], a2 = a0 + a1;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const T b0 = lb[16 * j], b1 = lb[NS + 16 * j];
          t1[w][j] = mfma(a0, b0, t1[w][j]);
          t2[w][j] = mfma(a1, b1, t2[w][j]);
          t3[w][j] = mfma(a2, b0 + b1, t3[w][j]);
        }
      }
    }
  }
  if (DL) __builtin_amdgcn_s_waitcnt(0x0F70);  // the spare load has landed
  __syncthreads();

  // antisymmetrise into V[cd][ab] (planar re, im) in LDS
  T* Vr = lds;
  T* Vi = lds + NS * VS;
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rw + out_row<T>(lk, r), jj = 16 * (j0 + j) + li;  // (a,c), (b,d)
      const int idx = ((i & 7) * TB + (jj & 7)) * VS + (i >> 3) * TB + (jj >> 3);
      Vr[idx] = (T)2 * (t1[0][j][r] - t2[0][j][r]);
      Vi[idx] = (T)2 * (t3[0][j][r] - t1[0][j][r] - t2[0][j][r]);
    }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * rw + out_row<T>(lk, r), jj = 16 * (j0 + j) + li;  // (a,d), (b,c)
      const int al = i >> 3, dl = i & 7, bl = jj >> 3, cl = jj & 7;
      const int idx = (cl * TB + dl) * VS + al * TB + bl;
      const bool live = (A < B || al < bl) && (B * TB + bl < v) && (C < D || cl < dl) &&
                        (D * TB + dl < v);
      const T re = t1[1][j][r] - t2[1][j][r], im = t3[1][j][r] - t1[1][j][r] - t2[1][j][r];
      Vr[idx] = live ? Vr[idx] - (T)2 * re : (T)0;
      Vi[idx] = live ? Vi[idx] - (T)2 * im : (T)0;
    }
  __syncthreads();
}

// Persistent ladder over several instances (eight waves, chunks loaded
// straight into a two-chunk LDS ring: the fastest FP64 launch variant).  A
// workgroup on XCD x takes the next item of x's queue (the instances' items
// l = x mod nx, instances ordered longest tile first): with each instance's
// tile order split into per-XCD super-tile shares, the workgroups of one XCD
// work on tiles that share Cholesky blocks in its L2.  When x's queue is
// empty the workgroup takes items from the next XCDs' queues, so uneven
// instances share one launch without a tail.  Every workgroup leaves once it
// has found all nx queues empty.
// CM3: the 3M form (three real products per complex product) in the build
// and the contraction; otherwise 4M.
constexpr int QNW = 8;
template <bool CM3>
__global__ __launch_bounds__(64 * QNW, 1) void k_ppl_queue(const BatchInst* __restrict__ inst,
                                                          int ninst,
                                                          const long* __restrict__ xtotal,
                                                          int nx,
                                                          unsigned* __restrict__ counter) {
  __shared__ __attribute__((aligned(16))) double lds[2 * Smem<double, 16>::build];
  __shared__ unsigned item;
  const int x0 = blockIdx.x % nx;
  for (int xi = 0; xi < nx;) {
    const int x = (x0 + xi) % nx;
    __syncthreads();  // every wave is done with the previous item and its LDS
    if (threadIdx.x == 0) item = atomicAdd(counter + x, 1u);
    __syncthreads();
    // the item is the same for every lane: keep it (and what is derived from
    // it) in scalar registers
    const long c = (unsigned)__builtin_amdgcn_readfirstlane((int)item);
    if (c >= xtotal[x]) {  // this XCD's queue is empty: move on to the next
      ++xi;
      continue;
    }
    int i = 0;
    while (i + 1 < ninst && c >= inst[i + 1].xstart[x]) ++i;
    const BatchInst& I = inst[i];
    const long l = (c - I.xstart[x]) * nx + x;
    int p, q;
    bool mirror;
    if (!decode_item(I.order, (long)I.nbp * (I.nbp + 1) / 2, I.nbp, l, *I.nonherm != 0, &p, &q,
                     &mirror))
      continue;
    tile_item<double, double, 1, QNW, CM3>(
        [&](int a, int b) {
          if constexpr (CM3)
            build_v_3m<double, 16, true, QNW>(I.Ls, I.tab, I.nbv, I.ncp, I.v, a, b, lds);
          else
            build_v_4m<double, 16, 1, true, QNW>(I.Ls, I.tab, I.nbv, I.ncp, I.v, a, b, lds);
        },
        I.Xb, I.Sb, I.nbp, I.Mp, p, q, mirror, lds);
  }
}


template <typename T, typename TA, int KC, bool DL, int NW>
__global__ __launch_bounds__(64 * NW, 1) void k_ppl_3m(const T* __restrict__ Ls,
                                                       const T* __restrict__ Xb,
                                                       TA* __restrict__ Sb,
                                                       const int* __restrict__ tab,
                                                       const int* __restrict__ order,
                                                       const int* __restrict__ nonherm, int nbv,
                                                       int nbp, int ncp, int Mp, int v) {
  constexpr int NE = DL ? 8 * Smem<T, KC>::chunk : Smem<T, KC>::elems;
  __shared__ __attribute__((aligned(16))) T lds[NE > Smem<T, KC>::elems ? NE : Smem<T, KC>::elems];
  int x, y;
  bool mirror;
  if (!decode_item(order, (long)nbp * (nbp + 1) / 2, nbp, blockIdx.x, *nonherm != 0, &x, &y,
                   &mirror))
    return;
  tile_item<T, TA, 1, NW, true>(
      [&](int p, int q) { build_v_3m<T, KC, DL, NW>(Ls, tab, nbv, ncp, v, p, q, lds); }, Xb,
      Sb, nbp, Mp, x, y, mirror, lds);
}


// Deterministic ladder (a debugging mode): one workgroup per block pair AB
// owns sigma[:, AB].  It builds every tile V(AB, CD), CD = 0 .. nbp - 1 in
// ascending order (no Hermitian halving: each tile is built by the
// workgroup of its row block pair), and adds X[:, CD] V(AB, CD)^T to its
// rows with plain read-modify-writes; each wave owns whole 16-row chunks.
// Every run performs the same additions in the same order, so sigma is
// reproducible bit for bit, at the cost of twice the builds and nbp
// workgroups only.
template <typename T, typename TA, int KC>
__global__ __launch_bounds__(WG, 1) void k_ppl_det(const T* __restrict__ Ls,
                                                   const T* __restrict__ Xb,
                                                   TA* __restrict__ Sb,
                                                   const int* __restrict__ tab, int nbv, int nbp,
                                                   int ncp, int Mp, int v) {
  typedef typename Acc<T>::t acc_t;
  typedef typename Vec16<T>::t vec_t;
  constexpr int VN = Vec16<T>::n;
  constexpr int NX = 16 / VN;
  __shared__ __attribute__((aligned(16))) T lds[Smem<T, KC>::elems];
  const int ab = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const size_t plane = (size_t)nbp * Mp * NS;
  TA* const sr_g = Sb + (size_t)ab * Mp * NS;
  TA* const si_g = sr_g + plane;
  const T* const Vr = lds;
  const T* const Vi = lds + NS * VS;
  for (int cd = 0; cd < nbp; ++cd) {
    build_v_4m<T, KC, 1, false, 4>(Ls, tab, nbv, ncp, v, ab, cd, lds);
    const T* xr_g = Xb + (size_t)cd * Mp * NS;
    const T* xi_g = xr_g + plane;
    for (int mc = wave; mc < Mp / 16; mc += 4) {
      const int m0 = mc * 16;
      T xr[16], xi[16];
      const vec_t* pr = reinterpret_cast<const vec_t*>(xr_g + (size_t)(m0 + li) * NS + 16 * lk);
      const vec_t* pi = reinterpret_cast<const vec_t*>(xi_g + (size_t)(m0 + li) * NS + 16 * lk);
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        const vec_t a = pr[k], b = pi[k];
#pragma unroll
        for (int t = 0; t < VN; ++t) {
          xr[k * VN + t] = a[t];
          xi[k * VN + t] = b[t];
        }
      }
      acc_t sr[4], si[4];
      contract_rows<T, false, 4, false>(Vr, Vi, xr, xi, 0, sr, si);
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const size_t o = (size_t)(m0 + out_row<T>(lk, r)) * NS + 16 * n + li;
          sr_g[o] += (TA)sr[n][r];
          si_g[o] += (TA)si[n][r];
        }
    }
    // (build_v_4m starts with a barrier: the next tile waits for every wave
    // to finish reading this one)
  }
}

constexpr int KC64 = 16;
constexpr int KC32 = 32;

}  // namespace

hipError_t ppl_det_launch(lrcc_prec prec, bool acc64, const Geom& g, const void* Ls,
                          const void* Xb, void* Sb, const int* tab, hipStream_t st) {
  if (g.nbp == 0 || g.Mp == 0) return hipSuccess;
#define LRCC_LD(T, TA, KC)                                                                      \
  hipLaunchKernelGGL((k_ppl_det<T, TA, KC>), dim3(g.nbp), dim3(WG), 0, st,                     \
                     static_cast<const T*>(Ls), static_cast<const T*>(Xb), static_cast<TA*>(Sb), \
                     tab, g.nbv, g.nbp, g.ncp, (int)g.Mp, g.v)
  if (prec == LRCC_FP64) LRCC_LD(double, double, KC64);
  else if (prec == LRCC_FP32 && acc64) LRCC_LD(float, double, KC32);
  else if (prec == LRCC_FP32) LRCC_LD(float, float, KC32);
  else return hipErrorNotSupported;
#undef LRCC_LD
  return hipGetLastError();
}

// Launch variants of the 4M kernel (chosen by the tuner; the environment
// variable LRCC_VARIANT sets the default): 1 = one workgroup per CU, chunks
// of 16 / 32 vectors prefetched through registers; 2 = two workgroups per CU
// through registers (FP32 only: the FP64 accumulators need the full register
// file); 3 = one workgroup per CU, chunks loaded straight into a two-chunk
// LDS ring; 4 = two workgroups per CU, direct loads into one LDS chunk;
// 5 = as 3 with eight waves (two per SIMD, each holding half the tile's
// accumulators).
bool ppl_has_variant(lrcc_prec prec, lrcc_cmul cmul, int variant) {
  if (cmul == LRCC_CMUL_3M)  // 3M: register prefetch, or eight waves with the ring
    return (prec == LRCC_FP64 || prec == LRCC_FP32) && (variant == 1 || variant == 5);
  if (prec == LRCC_FP64) return variant == 1 || variant == 3 || variant == 5;  // 4 would spill
  if (prec == LRCC_FP32) return variant >= 1 && variant <= 5;
  return variant == 1;
}

// Both complex forms read the same staged planes (re, im) in the same chunks;
// the chunk of the occupancy-2 variant divides that of occupancy 1, so one
// staged layout (padded to the larger chunk) serves every launch variant.
int ppl_chunk(lrcc_prec prec, lrcc_cmul) { return prec == LRCC_FP64 ? KC64 : KC32; }

size_t ppl_ls_bytes(lrcc_prec prec, lrcc_cmul, const Geom& g) {
  const size_t es = prec == LRCC_FP64 ? 8 : 4;
  return (size_t)g.nbv * g.nbv * g.ncp * 2 * NS * es;  // planes re, im
}
size_t ppl_xb_bytes(lrcc_prec prec, const Geom& g) {
  return (size_t)2 * g.xb_plane() * (prec == LRCC_FP64 ? 8 : 4);
}

long ppl_ntile(const Geom& g) { return (long)g.nbp * (g.nbp + 1) / 2; }

hipError_t ppl_launch(lrcc_prec prec, lrcc_cmul cmul, bool acc64, const Geom& g,
                      const void* Ls, const void* Xb, void* Sb, const int* tab,
                      const int* order, const int* nonherm, int occ, hipStream_t st) {
  const long ntile = ppl_ntile(g);
  if (ntile == 0 || g.Mp == 0) return hipSuccess;
  if (2 * ntile > 0x7fffffffL) return hipErrorInvalidValue;
  if (prec != LRCC_FP64 && prec != LRCC_FP32) return hipErrorNotSupported;
  const dim3 grid((unsigned)(2 * ntile));  // tiles, then their mirrors
  if (occ == 0) {
    // untuned default (the fastest measured at the baseline and precision
    // workloads): FP64 and 3M eight waves with the direct-to-LDS chunk ring;
    // FP32 4M two workgroups per CU, with direct loads when the sums are FP32
    const char* e = getenv("LRCC_VARIANT");
    occ = e ? atoi(e) : cmul != LRCC_CMUL_4M || prec == LRCC_FP64 ? 5 : acc64 ? 2 : 4;
  }
  if (!ppl_has_variant(prec, cmul, occ)) occ = 1;
  if (cmul == LRCC_CMUL_3M) {
#define LRCC_L3(T, TA, KC, DL, NW)                                                              \
  hipLaunchKernelGGL((k_ppl_3m<T, TA, KC, DL, NW>), grid, dim3(64 * NW), 0, st,                 \
                     static_cast<const T*>(Ls), static_cast<const T*>(Xb), static_cast<TA*>(Sb), \
                     tab, order, nonherm, g.nbv, g.nbp, g.ncp, (int)g.Mp, g.v)
    const bool w8 = occ == 5;
    if (prec == LRCC_FP64) {
      if (w8) LRCC_L3(double, double, KC64, true, 8);
      else LRCC_L3(double, double, KC64, false, 4);
    } else if (acc64) {
      if (w8) LRCC_L3(float, double, KC32, true, 8);
      else LRCC_L3(float, double, KC32, false, 4);
    } else {
      if (w8) LRCC_L3(float, float, KC32, true, 8);
      else LRCC_L3(float, float, KC32, false, 4);
    }
#undef LRCC_L3
    return hipGetLastError();
  }
#define LRCC_L4(T, TA, KC, OCC, DL, NW)                                                     \
  hipLaunchKernelGGL((k_ppl_4m<T, TA, KC, OCC, DL, NW>), grid, dim3(64 * NW), 0, st,         \
                     static_cast<const T*>(Ls), static_cast<const T*>(Xb), static_cast<TA*>(Sb), \
                     tab, order, nonherm, g.nbv, g.nbp, g.ncp, (int)g.Mp, g.v)
  if (prec == LRCC_FP64) {
    if (occ == 3) LRCC_L4(double, double, KC64, 1, true, 4);
    else if (occ == 5) LRCC_L4(double, double, KC64, 1, true, 8);
    else LRCC_L4(double, double, KC64, 1, false, 4);
  } else if (acc64) {
    if (occ == 2) LRCC_L4(float, double, 16, 2, false, 4);
    else if (occ == 3) LRCC_L4(float, double, KC32, 1, true, 4);
    else if (occ == 4) LRCC_L4(float, double, 16, 2, true, 4);
    else if (occ == 5) LRCC_L4(float, double, KC32, 1, true, 8);
    else LRCC_L4(float, double, KC32, 1, false, 4);
  } else {
    if (occ == 2) LRCC_L4(float, float, 16, 2, false, 4);
    else if (occ == 3) LRCC_L4(float, float, KC32, 1, true, 4);
    else if (occ == 4) LRCC_L4(float, float, 16, 2, true, 4);
    else if (occ == 5) LRCC_L4(float, float, KC32, 1, true, 8);
    else LRCC_L4(float, float, KC32, 1, false, 4);
  }
#undef LRCC_L4
  return hipGetLastError();
}

hipError_t ppl_queue_launch(const BatchInst* inst, int ninst, const long* xtotal, int nx,
                            unsigned* counter, int nwg, bool cm3, hipStream_t st) {
  if (ninst == 0 || nx < 1 || nx > QXMAX) return nx < 1 || nx > QXMAX ? hipErrorInvalidValue
                                                                       : hipSuccess;
  if (cm3)
    hipLaunchKernelGGL(k_ppl_queue<true>, dim3(nwg), dim3(64 * QNW), 0, st, inst, ninst, xtotal,
                       nx, counter);
  else
    hipLaunchKernelGGL(k_ppl_queue<false>, dim3(nwg), dim3(64 * QNW), 0, st, inst, ninst,
                       xtotal, nx, counter);
  return hipGetLastError();
}

}  // namespace lrcc
