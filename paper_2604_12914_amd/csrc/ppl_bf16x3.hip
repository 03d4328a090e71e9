// Split-BF16 (bf16x3) ladder for gfx950.
//
// Every real operand x is split as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even), and a real product is taken as
// hi*hi + hi*lo + lo*hi (the lo*lo term is dropped), all on the bf16 matrix
// cores with FP32 accumulation.  Complex products use the 4M form, so one
// complex multiply-accumulate costs 12 bf16 MFMA products.
//
// The ladder is evaluated in panels of consecutive block pairs AB, each
// holding the tiles (AB, CD) with CD >= AB (the upper triangle of the block-
// pair matrix) in both orientations:
//   k_vbuild   one workgroup per (AB, CG, DG), CG <= DG two groups of two
//              virtual blocks: W1 = sum_P L_(A,CG) (x) L_(B,DG) and
//              W2 = sum_P L_(A,DG) (x) L_(B,CG), two 128 x 128 complex
//              products on the 32x32x16 bf16 matrix cores, give the four
//              tiles V(AB, CD) = 2 <ab||cd>, C in CG, D in DG (each output
//              element of W1 and W2 is an integral one of the tiles needs, so
//              each Cholesky byte feeds twice the matrix work of a single
//              64 x 64 tile pair); antisymmetrised in LDS, split to hi/lo and
//              written to the panel (32 KB per tile).  The mirror tile
//              V(CD, AB) goes beside it: for Hermitian L^P it is the conjugate
//              transpose of the tile just built (one build per pair), otherwise
//              the same workgroup builds it from the transposed block roles (a
//              flag set on the device by the staging pass decides, so no host
//              round trip);
//   k_contract sigma[m, Q] += sum_{CD >= Q} X[m, CD] V(Q, CD)^T
//                           + sum_{AB < Q, AB in panel} X[m, AB] V(Q, AB)^T,
//              a bf16x3 GEMM in which each workgroup owns its output tile
//              (an m-block of rows x 64 slots of block pair Q) for the whole
//              panel: no atomics.  With one panel every workgroup runs over
//              nbp tiles.
// The integral panel is transient: at most one panel exists.
// The reason for the split: the fused kernel's atomic accumulation of sigma
// across CD tiles runs at the device's atomic throughput, which caps the fast
// bf16 arithmetic; a panel costs one extra write and read of V per apply.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "internal.hpp"

namespace lrcc {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

constexpr int KB = 16;                 // Cholesky vectors per chunk (MFMA k of the build)
constexpr int NPL = 4;                 // planes: re_hi, re_lo, im_hi, im_lo
constexpr int CHUNK = NPL * NS * KB;   // bf16 per block per chunk (8 KB): [plane][64][16]
constexpr int VT = NPL * NS * NS;      // bf16 per V tile (32 KB)
// LDS rows of the contraction's V tiles are padded so that the 8 lanes of
// one 16-byte LDS read phase hit distinct banks: rows of 64 bf16 (128 B)
// get a stride of 72 (144 B).
constexpr int NSP = NS + 8;
constexpr int VTP = NPL * NS * NSP;     // padded V tile in LDS

__device__ __forceinline__ f4 mfma(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Output row of accumulator item r in lane group lk (column = lane % 16).
__device__ __forceinline__ int out_row(int lk, int r) { return 4 * lk + r; }

__device__ __forceinline__ bf8 neg(bf8 x) {
  u4 u = __builtin_bit_cast(u4, x);
  u ^= (u4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(bf8, u);
}

__device__ __forceinline__ void split(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// acc += x * y for real operands given as (hi, lo): hi*hi + hi*lo + lo*hi
__device__ __forceinline__ f4 mac3(bf8 xh, bf8 xl, bf8 yh, bf8 yl, f4 acc) {
  acc = mfma(xh, yh, acc);
  acc = mfma(xh, yl, acc);
  acc = mfma(xl, yh, acc);
  return acc;
}

__device__ inline double2 load_c(const void* p, lrcc_dtype dt, size_t i) {
  if (dt == LRCC_C128) return static_cast<const double2*>(p)[i];
  float2 f = static_cast<const float2*>(p)[i];
  return make_double2(f.x, f.y);
}

__device__ inline long pidx(long p, long q, long n) { return p * (2 * n - p - 1) / 2 + (q - p - 1); }

// L -> Ls16[A][C][chunk][plane][64 (a,c)][16 P]
__global__ void k_stage_L16(const void* __restrict__ L, lrcc_dtype dt, int v, int nchol, int nbv,
                            int ncp, int form, __bf16* __restrict__ Ls) {
  const long total = (long)nbv * nbv * ncp * NS;  // (block, P, slot)
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int p = e % KB;
    const int s = (e / KB) % NS;
    const long rest = e / (KB * NS);  // (block, chunk)
    const int pc = rest % (ncp / KB);
    const long blk = rest / (ncp / KB);
    const int C = blk % nbv, A = blk / nbv;
    const int a = A * TB + s / TB, c = C * TB + s % TB, P = pc * KB + p;
    float re = 0.f, im = 0.f;
    if (a < v && c < v && P < nchol) {
      const size_t src = form != L_PLAIN ? ((size_t)P * v + c) * v + a : ((size_t)P * v + a) * v + c;
      double2 z = load_c(L, dt, src);
      re = (float)z.x;
      im = (float)(form == L_ADJ ? -z.y : z.y);
    }
    __bf16* dst = Ls + (size_t)rest * CHUNK + s * KB + p;
    split(re, dst[0], dst[NS * KB]);
    split(im, dst[2 * NS * KB], dst[3 * NS * KB]);
  }
}

// The bf16 X planes hold each block pair's 64 slots as two halves of 32
// (the two k-steps of the contraction), row after row within a half:
// Xb16[plane][bp][half][m][32].  One contraction load of 16 rows x 32 slots
// is then 1 KB of whole cache lines.
__device__ __forceinline__ long x16_index(long bp, long m, int s, long Mp) {
  return ((bp * 2 + (s >> 5)) * Mp + m) * 32 + (s & 31);
}

// Packed doubles -> Xb16 (hi/lo split, zeros in dead slots)
__global__ void k_pack_x16(const void* __restrict__ X, lrcc_dtype dt, int v, long npv, long M,
                           long Mp, int nbp, const int* __restrict__ tab, __bf16* __restrict__ Xb) {
  const long plane = (long)nbp * Mp * NS;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < plane;
       e += (long)gridDim.x * blockDim.x) {
    const int s = e % NS;
    const long m = (e / NS) % Mp;
    const int bp = e / (NS * Mp);
    const int AB = tab[bp];
    const int a = (AB >> 16) * TB + s / TB, b = (AB & 0xffff) * TB + s % TB;
    float re = 0.f, im = 0.f;
    if (a < b && b < v && m < M) {
      double2 z = load_c(X, dt, (size_t)m * npv + pidx(a, b, v));
      re = (float)z.x;
      im = (float)z.y;
    }
    const long d = x16_index(bp, m, s, Mp);
    split(re, Xb[d], Xb[d + plane]);
    split(im, Xb[d + 2 * plane], Xb[d + 3 * plane]);
  }
}

// FP64 block planes [plane][bp][m][64] -> Xb16 hi/lo planes
__global__ void k_split_x16(long plane, long Mp, const double* __restrict__ x,
                            __bf16* __restrict__ Xb) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < plane;
       e += (long)gridDim.x * blockDim.x) {
    const long d = x16_index(e / (NS * Mp), (e / NS) % Mp, (int)(e % NS), Mp);
    split((float)x[e], Xb[d], Xb[d + plane]);
    split((float)x[e + plane], Xb[d + 2 * plane], Xb[d + 3 * plane]);
  }
}

// ---------------------------------------------------------------------------
// Integral build.  Tile index, within the panel that starts at block pair
// ab0, of the upper tile (ab0 + abl, cd), cd >= ab0 + abl: rows of the
// triangle one after another.
__device__ __forceinline__ long panel_tile(int nbp, int ab0, int abl, int cd) {
  return (long)abl * nbp - (long)abl * ab0 - (long)abl * (abl - 1) / 2 + (cd - ab0 - abl);
}

typedef float f16v __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f16v mfma32(bf8 a, bf8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// acc += x * y for real operands given as (hi, lo): hi*hi + hi*lo + lo*hi
__device__ __forceinline__ f16v mac3_32(bf8 xh, bf8 xl, bf8 yh, bf8 yl, f16v acc) {
  acc = mfma32(xh, yh, acc);
  acc = mfma32(xh, yl, acc);
  acc = mfma32(xl, yh, acc);
  return acc;
}

// Block-pair index of the virtual blocks (C, D), C <= D.
__device__ __forceinline__ int bp_index(int C, int D, int nbv) {
  return C * nbv - C * (C - 1) / 2 + (D - C);
}

// Byte offset, inside one [64 rows][16 P] plane (2 KB) of a staged block
// chunk held in LDS, of the 16-byte half h (P 8h .. 8h + 7) of row r.  The
// halves are swapped where bits 2 and 3 of the row differ, so that the 16
// consecutive rows one 16-byte LDS read covers per cycle (64 banks of 4
// bytes) fall on 16 distinct 16-byte bank groups, and any 8 aligned ones on
// 8 distinct groups of 128 bytes.
__device__ __forceinline__ int lds_swz(int r) { return ((r >> 2) ^ (r >> 3)) & 1; }
__device__ __forceinline__ int lds_half(int r, int h) { return r * 32 + ((h ^ lds_swz(r)) << 4); }

// Output row / column of element r of a 32x32 MFMA accumulator in lane l
// (32x32x16: rows in four groups of eight, lanes 32..63 holding rows 4..7 of
// each group).
__device__ __forceinline__ int out_row32(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }

constexpr int BW = 8;                    // waves of a build workgroup (two per SIMD)
constexpr int BWG = 64 * BW;
constexpr int CHB = CHUNK * 2;           // bytes per staged block chunk (8 KB)
constexpr int VR = NS + 1;               // padded row of the W staging areas (floats)
constexpr int AREA = 2 * NS * VR;        // floats per W staging area (re, im planes)
constexpr int BLDS = (2 * 8 * CHB > 4 * AREA * 4) ? 2 * 8 * CHB : 4 * AREA * 4;

// One workgroup per item (AB, CG, DG): the panel row ab = ab0 + abl with
// blocks (A, B), the block groups CG = {2 cg, 2 cg + 1} and DG = {2 dg,
// 2 dg + 1}, cg <= dg.  Its tiles are (AB, C D) for C in CG, D in DG with
// C <= D < nbv and cd = bp(C, D) >= ab.
//
// Roles.  A tile V(XY, ZW)[(x y), (z w)] = 2 (W1[(x z), (y w)] - W2[(x w),
// (y z)]) with W1 = sum_P L_XZ (x) L_YW and W2 = sum_P L_XW (x) L_YZ.  In the
// upper pass X = A, Y = B, Z = C_r, W = D_j: W1 is the 128 x 128 product of
// the blocks (A, C_0..1) with (B, D_0..1), W2 that of (A, D_0..1) with
// (B, C_0..1).  In the mirror pass (non-Hermitian L only) X = C_r, Y = D_j,
// Z = A, W = B, which gives V(CD, AB) itself: W1 from (C_0..1, A) x
// (D_0..1, B), W2 from (C_0..1, B) x (D_0..1, A).
//
// The eight operand blocks of a chunk of 16 Cholesky vectors go straight
// from global memory into a two-chunk LDS ring (8 KB each, slot s loaded by
// wave s); wave w < 4 computes the 64 x 64 quadrant (w >> 1, w & 1) of W1
// from slots (w >> 1) and 2 + (w & 1), wave 4 + q the quadrant (q >> 1, q & 1)
// of W2 from slots 4 + (q >> 1) and 6 + (q & 1): 2 x 2 MFMAs of 32 x 32 per
// plane product, 48 per chunk.  Then, two tiles at a time, the quadrants go to
// LDS at their V positions and every thread forms, splits and stores V.
__global__ __launch_bounds__(BWG, 1) void k_vbuild(const __bf16* __restrict__ Ls,
                                                   const int* __restrict__ tab,
                                                   const int2* __restrict__ items,
                                                   const int* __restrict__ nonherm, int nbv,
                                                   int nbp, int nch, int v, int ab0,
                                                   __bf16* __restrict__ Vdir,
                                                   __bf16* __restrict__ Vmir) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[BLDS];
  const bool nh = *nonherm != 0;
  const int2 item = items[blockIdx.x];
  const int abl = item.x, cg = item.y >> 16, dg = item.y & 0xffff;
  const int ab = ab0 + abl;
  const int A = tab[ab] >> 16, B = tab[ab] & 0xffff;
  const int Cb[2] = {2 * cg, 2 * cg + 1}, Db[2] = {2 * dg, 2 * dg + 1};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // operand slots read by this wave, and whether it computes W1 or W2
  const bool w1 = wave < 4;
  const int q = w1 ? wave : wave - 4;
  const int aslot = (w1 ? 0 : 4) + (q >> 1), bslot = (w1 ? 2 : 6) + (q & 1);

  for (int mode = 0; mode < (nh ? 2 : 1); ++mode) {
    // staged block loaded by this wave into ring slot `wave` (blocks past the
    // last virtual block, in a last group of one, are replaced by that last
    // block: in bounds, and their tiles are never stored)
    int blk;
    {
      const int t = wave & 1;
      const int Ct = min(Cb[t], nbv - 1), Dt = min(Db[t], nbv - 1);
      if (mode == 0) {
        const int rowb[4] = {A * nbv + Ct, B * nbv + Dt, A * nbv + Dt, B * nbv + Ct};
        blk = rowb[wave >> 1];
      } else {
        const int rowb[4] = {Ct * nbv + A, Dt * nbv + B, Ct * nbv + B, Dt * nbv + A};
        blk = rowb[wave >> 1];
      }
    }
    const char* const gsrc = reinterpret_cast<const char*>(Ls + (size_t)blk * nch * CHUNK);
    // piece k (1 KB) of this wave's slot: plane k >> 1, rows 32 (k & 1) ..
    // + 31; lane l writes LDS bytes 16 l of the piece, which hold row
    // 32 (k & 1) + l / 2, half (l & 1) as placed by lds_half, so it reads
    // the global half (l & 1) ^ lds_swz(row) (the same for both row halves
    // of a plane: 32 is a multiple of 16)
    const int goff = (lane >> 1) * 32 + (((lane & 1) ^ lds_swz(lane >> 1)) << 4);
    auto issue = [&](int c, unsigned char* buf) {
      const char* src = gsrc + (size_t)c * CHB + goff;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        __builtin_amdgcn_global_load_lds(
            src + k * 1024,
            (__attribute__((address_space(3))) void*)(buf + wave * CHB + k * 1024), 16, 0, 0);
    };
    f16v wr[2][2], wi[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int e = 0; e < 16; ++e) wr[i][j][e] = 0.f;
        wi[i][j] = wr[i][j];
      }
    // W += A B over one chunk: re += Ar Br - Ai Bi, im += Ar Bi + Ai Br (the
    // minus sign on the Bi operand)
    // this lane's operand bytes in a plane: row (lane & 31) (+ 32 for the
    // second MFMA block, which leaves bits 2 and 3 of the row unchanged), half lane >> 5
    const int loff = lds_half(lane & 31, lane >> 5);
    auto mma = [&](const unsigned char* buf) {
      const unsigned char* as = buf + aslot * CHB + loff;
      const unsigned char* bs = buf + bslot * CHB + loff;
      bf8 a[2][4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int p = 0; p < 4; ++p)
          a[i][p] = *reinterpret_cast<const bf8*>(as + p * 2048 + i * 1024);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        bf8 b[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
          b[p] = *reinterpret_cast<const bf8*>(bs + p * 2048 + j * 1024);
        const bf8 nb2 = neg(b[2]), nb3 = neg(b[3]);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          wr[i][j] = mac3_32(a[i][0], a[i][1], b[0], b[1], wr[i][j]);  // Ar Br
          wr[i][j] = mac3_32(a[i][2], a[i][3], nb2, nb3, wr[i][j]);    // -Ai Bi
          wi[i][j] = mac3_32(a[i][0], a[i][1], b[2], b[3], wi[i][j]);  // Ar Bi
          wi[i][j] = mac3_32(a[i][2], a[i][3], b[0], b[1], wi[i][j]);  // Ai Br
        }
      }
    };
    // Two-chunk ring: chunk c sits in buffer c & 1.  At the top of chunk c
    // every wave waits for its own loads of c, the barrier makes all of them
    // visible and shows that chunk c - 1 is no longer read, and chunk c + 1
    // is requested into the other buffer (the last chunk again on the last
    // pass: a branch-free loop body).
    __syncthreads();  // LDS may still hold the previous pass's W areas
    issue(0, lds);
    for (int c = 0; c < nch; ++c) {
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads of chunk c landed
      __syncthreads();
      issue(min(c + 1, nch - 1), lds + ((c + 1) & 1) * 8 * CHB);
      mma(lds + (c & 1) * 8 * CHB);
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // the spare load has landed
    __syncthreads();                     // every wave is done with the ring

    // ---- tiles, two at a time: round t holds tiles (C_0, D_t) and (C_1, D_t).
    // Tile (r, j) takes W1 quadrant (r, j) (wave 2 r + j) and W2 quadrant
    // (j, r) in the upper pass (rows X W = A D_j), (r, j) in the mirror pass
    // (rows X W = C_r B): wave 4 + 2 j + r, or 4 + 2 r + j.
    float* const area = reinterpret_cast<float*>(lds);
    for (int t = 0; t < 2; ++t) {
      int k = -1;  // area of this wave's quadrant in this round (0, 1: W1; 2, 3: W2)
      if (w1) {
        if ((q & 1) == t) k = q >> 1;
      } else if (mode == 0) {
        if ((q >> 1) == t) k = 2 + (q & 1);
      } else {
        if ((q & 1) == t) k = 2 + (q >> 1);
      }
      if (k >= 0) {
        float* const ar = area + k * AREA;
        float* const ai = ar + NS * VR;
        // (the empty asm makes the lane index opaque here, so the index
        // arithmetic below is not computed ahead of the chunk loop and kept
        // live across it)
        int ln = lane;
        asm volatile("" : "+v"(ln));
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
              const int ii = 32 * i + out_row32(ln, e), jj = 32 * j + (ln & 31);
              // W1: ii = (x, z), jj = (y, w);  W2: ii = (x, w), jj = (y, z)
              const int idx = w1 ? ((ii >> 3) * TB + (jj >> 3)) * VR + (ii & 7) * TB + (jj & 7)
                                 : ((ii >> 3) * TB + (jj >> 3)) * VR + (jj & 7) * TB + (ii & 7);
              ar[idx] = wr[i][j][e];
              ai[idx] = wi[i][j][e];
            }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int C = Cb[r], D = Db[t];
        if (C >= nbv || D >= nbv || C > D) continue;  // uniform
        const int cd = bp_index(C, D, nbv);
        if (cd < ab || (mode == 1 && cd == ab)) continue;
        const long tt = panel_tile(nbp, ab0, abl, cd);
        const int X = mode == 0 ? A : C, Y = mode == 0 ? B : D;
        const int Z = mode == 0 ? C : A, W = mode == 0 ? D : B;
        const float* const w1r = area + r * AREA;
        const float* const w1i = w1r + NS * VR;
        const float* const w2r = area + (2 + r) * AREA;
        const float* const w2i = w2r + NS * VR;
        // write [plane][row slot][column slot]; ct: the conjugate transpose
        auto store = [&](__bf16* dst, bool ct) {
          int row = threadIdx.x >> 3, qc = (threadIdx.x & 7) * 8;
          asm volatile("" : "+v"(row), "+v"(qc));  // computed here, not ahead of the loop
          bf8 rh, rl, ih, il;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            // element V[xy][zw] of the tile built here
            const int xy = ct ? qc + e : row, zw = ct ? row : qc + e;
            const int xl = xy >> 3, yl = xy & 7, zl = zw >> 3, wl = zw & 7;
            const bool live = (X < Y || xl < yl) && (Y * TB + yl < v) && (Z < W || zl < wl) &&
                              (W * TB + wl < v);
            const int idx = xy * VR + zw;
            const float vr = live ? 2.f * (w1r[idx] - w2r[idx]) : 0.f;
            const float vi = live ? 2.f * (w1i[idx] - w2i[idx]) : 0.f;
            __bf16 hi, lo;
            split(vr, hi, lo);
            rh[e] = hi;
            rl[e] = lo;
            split(ct ? -vi : vi, hi, lo);
            ih[e] = hi;
            il[e] = lo;
          }
          *reinterpret_cast<bf8*>(dst + 0 * NS * NS + row * NS + qc) = rh;
          *reinterpret_cast<bf8*>(dst + 1 * NS * NS + row * NS + qc) = rl;
          *reinterpret_cast<bf8*>(dst + 2 * NS * NS + row * NS + qc) = ih;
          *reinterpret_cast<bf8*>(dst + 3 * NS * NS + row * NS + qc) = il;
        };
        if (mode == 0) {
          store(Vdir + tt * VT, false);
          if (!nh && cd != ab) store(Vmir + tt * VT, true);
        } else {
          store(Vmir + tt * VT, false);
        }
      }
      __syncthreads();  // the areas are rewritten in the next round
    }
  }
}

// ---------------------------------------------------------------------------
// Contraction of one panel [ab0, ab1): workgroup (m-block of rb rows, block
// pair q >= ab0); wave w owns rows 32w .. 32w+31 of the block and all 64
// slots of q.  Its tiles, in ascending order of the contracted block pair b:
// the mirror tiles V(q, b) of the panel rows b < q, then the upper tiles
// V(q, b), b >= q, when q is in the panel.  With one panel every workgroup
// visits b = 0, 1, ..., nbp - 1 in the same order, so workgroups of
// different q read the same X rows at about the same time.
//
// Workgroup w runs on XCD w mod nx (round-robin dispatch).  Each XCD takes a
// contiguous share of the logical work list, which is ordered in groups of
// QG block pairs x all m-blocks: the workgroups resident on one XCD then
// share the V tiles of a few q (across m-blocks) and the X rows of a few
// m-blocks (across q) in its L2.
constexpr int QG = 8;

// The list is split into nsplit parts (outermost): part p of a workgroup's
// tiles goes to a workgroup of its own, so that short grids still fill whole
// rounds of resident workgroups; parts add their sums atomically.
// With several panels the workgroups of block pairs inside the panel run the
// whole list and the others only the panel's mirror tiles: there (grouped =
// false) the plain order, q ascending with its m-blocks and parts, dispatches
// the long workgroups first and spreads them over all XCDs.
__device__ __forceinline__ void contract_item(int w, int total, int nx, int nmb, int nq,
                                              bool grouped, int* q, int* mb, int* part) {
  if (!grouped) {
    const int ns = total / (nmb * nq), r = w % (nmb * ns);
    *q = w / (nmb * ns);
    *mb = r / ns;
    *part = r % ns;
    return;
  }
  const int x = w % nx, j = w / nx;
  const int share = total / nx, rem = total % nx;
  int L = x * share + (x < rem ? x : rem) + j;
  *part = L / (nmb * nq);
  L -= *part * nmb * nq;
  const int group = L / (QG * nmb), r = L - group * QG * nmb;
  const int gq = min(QG, nq - group * QG);
  *mb = r / gq;
  *q = group * QG + r % gq;
}
// NWV waves per workgroup, each owning 32 rows of the m-block (rb rows, a
// multiple of 16 up to 32 NWV; the host balances rb over the m-blocks).
// Four waves: two workgroups per CU, so that while one waits for its X rows
// (loaded straight into registers, half a tile ahead) the other keeps the
// matrix cores busy.  Eight waves: one workgroup per CU over twice the rows,
// so every V tile is read from memory half as often.
template <typename TA, int NWV>
__global__ __launch_bounds__(64 * NWV, NWV == 4 ? 2 : 1) void k_contract(
    const __bf16* __restrict__ Xb, const __bf16* __restrict__ Vdir,
    const __bf16* __restrict__ Vmir, int nbp, int Mp, int nmb, int rb, int ab0, int ab1, int nx,
    int grouped, TA* __restrict__ Sb) {
  constexpr int CWG = 64 * NWV;
  __shared__ __attribute__((aligned(16))) __bf16 vt[2 * VTP];  // two V tiles, 72 KB
  int mb, ql, part;
  contract_item(blockIdx.x, (int)gridDim.x, nx, nmb, nbp - ab0, grouped != 0, &ql, &mb, &part);
  const int nsplit = (int)gridDim.x / (nmb * (nbp - ab0));
  const int q = ab0 + ql;
  const int ndir = q < ab1 ? nbp - q : 0;
  const int nmir = (q < ab1 ? q : ab1) - ab0;
  const int it0 = (int)((long)(ndir + nmir) * part / nsplit);
  const int ntl = (int)((long)(ndir + nmir) * (part + 1) / nsplit);
  // tile it of this workgroup and the block pair whose X rows it contracts
  // (selects, no branches: the loads that use them stay where they are put)
  auto tile_of = [&](int it, int* xblk) -> const __bf16* {
    const bool mir = it < nmir;
    const int d = it - nmir;
    *xblk = mir ? ab0 + it : q + d;
    const long t = mir ? panel_tile(nbp, ab0, it, q) : panel_tile(nbp, ab0, q - ab0, q + d);
    return (mir ? Vmir : Vdir) + t * VT;
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const size_t plane = (size_t)nbp * Mp * NS;
  // rows of this wave; 16-row blocks past the m-block's rb rows or past Mp
  // load row block 0 instead, so every load is unconditional and in bounds,
  // and their sums are never stored
  int mrow[2], mld[2];
  bool mok[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    mrow[i] = mb * rb + 32 * wave + 16 * i;
    mok[i] = 32 * wave + 16 * i < rb && mrow[i] < Mp;
    mld[i] = mok[i] ? mrow[i] : 0;
  }
  // a wave whose rows all lie past the m-block still loads and stores its
  // share of every V tile but skips the matrix work (its second row block
  // lies past the first)
  const bool busy = mok[0];
  f4 sr[2][4], si[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sr[i][j] = (f4){0, 0, 0, 0};
      si[i][j] = sr[i][j];
    }
  // X operands of one CD: [mblk][k-step][plane], 8 consecutive cd per lane.
  // The two k-steps rotate through the loads: k-step 1 of this tile is
  // requested while k-step 0 is contracted, k-step 0 of the next tile while
  // k-step 1 is; the vector-memory counter retires in order, so each wait
  // covers exactly the loads issued before the ones still in flight.
  bf8 xa[2][2][4];
  auto fetch_x = [&](int cd, int ks) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        xa[i][ks][p] = *reinterpret_cast<const bf8*>(
            Xb + p * plane + (((size_t)cd * 2 + ks) * Mp + mld[i] + li) * 32 + 8 * lk);
  };
  // V tiles: a two-tile LDS ring, filled through registers in two halves.
  // The first half of the next tile is requested at the start of a tile and
  // stored to the free buffer after k-step 0, the second half requested then
  // and stored at the end: one barrier per tile, each load has a k-step of
  // matrix work to land, and only half a tile is held in registers.
  constexpr int VH = VT / 8 / CWG / 2;  // 16-byte vectors per thread per half tile (4 or 2)
  static_assert(VH * 8 * CWG * 2 == VT, "half tiles split evenly over the threads");
  u4 vp[VH];
  int xnext = 0;
  const __bf16* vsrc = Vdir;
  auto fetch_v = [&](int h) {
#pragma unroll
    for (int k = 0; k < VH; ++k)
      vp[k] = reinterpret_cast<const u4*>(vsrc)[(h * VH + k) * CWG + threadIdx.x];
  };
  auto store_v = [&](__bf16* buf, int h) {
#pragma unroll
    for (int k = 0; k < VH; ++k) {
      // vector e of the tile: plane-row (e / 8), 8-bf16 part (e % 8)
      const int e = (h * VH + k) * CWG + threadIdx.x;
      *reinterpret_cast<u4*>(buf + (e >> 3) * NSP + (e & 7) * 8) = vp[k];
    }
  };
  // sigma_r += Xr Vr^T - Xi Vi^T, sigma_i += Xr Vi^T + Xi Vr^T (the minus
  // sign goes on the Vi operand: sign flips of its bf16 halves)
  auto contract_ks = [&](const __bf16* vb, int ks) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf8 b[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        b[p] = *reinterpret_cast<const bf8*>(vb + (p * NS + 16 * j + li) * NSP + 32 * ks +
                                             8 * lk);
      const bf8 nb2 = neg(b[2]), nb3 = neg(b[3]);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        sr[i][j] = mac3(xa[i][ks][0], xa[i][ks][1], b[0], b[1], sr[i][j]);
        sr[i][j] = mac3(xa[i][ks][2], xa[i][ks][3], nb2, nb3, sr[i][j]);
        si[i][j] = mac3(xa[i][ks][0], xa[i][ks][1], b[2], b[3], si[i][j]);
        si[i][j] = mac3(xa[i][ks][2], xa[i][ks][3], b[0], b[1], si[i][j]);
      }
    }
  };
  if (ntl > it0) {
    vsrc = tile_of(it0, &xnext);
    fetch_v(0);
    __builtin_amdgcn_sched_barrier(0);  // same load order as in the loop
    fetch_x(xnext, 0);
    store_v(vt, 0);
    fetch_v(1);
    store_v(vt, 1);
  }
  for (int it = it0; it < ntl; ++it) {
    const int xcur = xnext;
    const int par = (it - it0) & 1;
    const __bf16* const cur = vt + par * VTP;
    __bf16* const nxt = vt + (par ^ 1) * VTP;
    // this tile's V is visible to every wave, and every wave is done with
    // the other buffer
    __syncthreads();
    fetch_x(xcur, 1);
    // the next tile (this one again on the last pass: branch-free loads)
    vsrc = tile_of(min(it + 1, ntl - 1), &xnext);
    fetch_v(0);
    // scheduling barriers keep each load group between the two k-steps
    // instead of letting the scheduler sink it to the next barrier
    __builtin_amdgcn_sched_barrier(0);
    if (busy) contract_ks(cur, 0);
    __builtin_amdgcn_sched_barrier(0);
    store_v(nxt, 0);
    fetch_v(1);
    fetch_x(xnext, 0);
    __builtin_amdgcn_sched_barrier(0);
    if (busy) contract_ks(cur, 1);
    __builtin_amdgcn_sched_barrier(0);
    store_v(nxt, 1);
  }
  // add this part's share of sigma[rows, q]: a plain update when the
  // workgroup is the only writer in this launch, atomic across parts
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (!mok[i]) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t o = ((size_t)q * Mp + mrow[i] + out_row(lk, r)) * NS + 16 * j + li;
        if (nsplit == 1) {
          Sb[o] += (TA)sr[i][j][r];
          Sb[o + plane] += (TA)si[i][j][r];
        } else {
          unsafeAtomicAdd(Sb + o, (TA)sr[i][j][r]);
          unsafeAtomicAdd(Sb + o + plane, (TA)si[i][j][r]);
        }
      }
  }
}

inline int grid_for(long n) {
  long g = (n + 255) / 256;
  return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

}  // namespace

int bf16x3_chunk() { return KB; }
size_t bf16x3_ls_bytes(const Geom& g) { return (size_t)g.nbv * g.nbv * g.ncp * NS * NPL * 2; }
size_t bf16x3_xb_bytes(const Geom& g) { return (size_t)NPL * g.xb_plane() * 2; }

hipError_t bf16x3_stage_L(const void* L, lrcc_dtype dt, const Geom& g, LForm form, void* Ls,
                          hipStream_t st) {
  const long total = (long)g.nbv * g.nbv * g.ncp * NS;
  hipLaunchKernelGGL(k_stage_L16, dim3(grid_for(total)), dim3(256), 0, st, L, dt, g.v, g.nchol,
                     g.nbv, g.ncp, (int)form, static_cast<__bf16*>(Ls));
  return hipGetLastError();
}

hipError_t bf16x3_pack_x(const void* X, lrcc_dtype dt, const Geom& g, const int* tab, void* Xb,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_pack_x16, dim3(grid_for(g.xb_plane())), dim3(256), 0, st, X, dt, g.v,
                     g.npv, g.M, g.Mp, g.nbp, tab, static_cast<__bf16*>(Xb));
  return hipGetLastError();
}

hipError_t bf16x3_split_x(const double* x, const Geom& g, void* Xb, hipStream_t st) {
  hipLaunchKernelGGL(k_split_x16, dim3(grid_for(g.xb_plane())), dim3(256), 0, st, g.xb_plane(),
                     g.Mp, x, static_cast<__bf16*>(Xb));
  return hipGetLastError();
}

// Upper tiles of the panel rows [ab0, ab0 + n).
long bf16x3_panel_tiles(const Geom& g, int ab0, int n) {
  return (long)n * g.nbp - (long)n * ab0 - (long)n * (n - 1) / 2;
}

size_t bf16x3_panel_bytes(const Geom& g, int ab0, int n) {
  return (size_t)bf16x3_panel_tiles(g, ab0, n) * 2 * VT * sizeof(__bf16);  // tile + mirror
}

// Build items of the panels starting at starts[k] (rows [starts[k],
// starts[k + 1])), concatenated panel after panel (off[k] = first item of
// panel k).  An item (abl, cg << 16 | dg) exists when at least one of its
// tiles lies in the upper triangle: its last tile (min(C_max, D_max), D_max)
// has cd >= ab.  Within a panel the items are sorted by super-tile (sw-wide
// ranges of A and B, sw/2-wide ranges of the block groups), and each XCD
// receives a contiguous share (workgroup w runs on XCD w mod nx, as the
// (w / nx)-th of that XCD's workgroups), so the workgroups one XCD runs at a
// time share Cholesky blocks in its L2.
void build_items(const Geom& g, const std::vector<int>& starts, int sw, int nx,
                 std::vector<int2>* items, std::vector<long>* off) {
  const int nbv = g.nbv, ng = (nbv + 1) / 2, sg = std::max(1, sw / 2);
  std::vector<int> A(g.nbp), B(g.nbp);
  for (int a = 0, k = 0; a < nbv; ++a)
    for (int b = a; b < nbv; ++b, ++k) {
      A[k] = a;
      B[k] = b;
    }
  auto bp = [&](int C, int D) { return C * nbv - C * (C - 1) / 2 + (D - C); };
  items->clear();
  off->assign(1, 0);
  for (size_t k = 0; k + 1 < starts.size(); ++k) {
    const int ab0 = starts[k], ab1 = starts[k + 1];
    struct It {
      long key;
      int abl, cgdg;
    };
    std::vector<It> all;
    for (int ab = ab0; ab < ab1; ++ab)
      for (int cg = 0; cg < ng; ++cg)
        for (int dg = cg; dg < ng; ++dg) {
          const int Cmax = std::min(2 * cg + 1, nbv - 1), Dmax = std::min(2 * dg + 1, nbv - 1);
          if (bp(std::min(Cmax, Dmax), Dmax) < ab) continue;
          const long key = (((long)(A[ab] / sw) * 4096 + B[ab] / sw) * 4096 + cg / sg) * 4096 +
                           dg / sg;
          all.push_back({key, ab - ab0, (cg << 16) | dg});
        }
    std::stable_sort(all.begin(), all.end(), [](const It& x, const It& y) { return x.key < y.key; });
    const long total = (long)all.size(), q = total / nx, r = total % nx;
    for (long w = 0; w < total; ++w) {
      const long x = w % nx, j = w / nx;
      const It& e = all[x * q + std::min<long>(x, r) + j];
      items->push_back(make_int2(e.abl, e.cgdg));
    }
    off->push_back((long)items->size());
  }
}

// Panels of consecutive block pairs, each as many rows as fit in `cap` bytes
// (at least one): build, then contract.  Sb (zeroed by the caller, FP64 or
// FP32 planes) receives the panels' shares.  *nonherm (device) selects the
// mirror tiles' source.
hipError_t bf16x3_run(lrcc_handle h, const Geom& g, const void* Ls, const void* Xb, void* Sb,
                      bool acc64, void* Vws, size_t cap, const int* tab, const int* nonherm,
                      hipStream_t st) {
  if (g.nbp == 0 || g.Mp == 0) return hipSuccess;
  // contraction shape: waves per workgroup, m-blocks and their balanced
  // row count (a multiple of 16)
  int cw = 8;
  if (const char* e = getenv("LRCC_CONTRACT_WAVES")) cw = atoi(e) == 4 ? 4 : 8;
  const int nmb = (int)((g.Mp + 32 * cw - 1) / (32 * cw));
  const int rb = (int)roundup((g.Mp + nmb - 1) / nmb, 16);
  std::vector<int> starts;
  for (int ab0 = 0, n = 1; ab0 < g.nbp; ab0 += n) {
    n = 1;
    while (ab0 + n < g.nbp && bf16x3_panel_bytes(g, ab0, n + 1) <= cap) ++n;
    starts.push_back(ab0);
  }
  starts.push_back(g.nbp);
  // build items of every panel: computed and uploaded once per geometry
  const int nx = std::max(1, h->ncu / 32);  // XCDs
  const int sw = h->order_s[LRCC_BF16X3] > 0 ? h->order_s[LRCC_BF16X3] : 4;
  std::vector<long> key = {g.nbv, nx, sw};
  key.insert(key.end(), starts.begin(), starts.end());
  if (key != h->bitems_key) {
    std::vector<int2> items;
    build_items(g, starts, sw, nx, &items, &h->bitems_off);
    h->bitems_key.clear();
    hipError_t e = h->bitems.ensure(items.size() * sizeof(int2));
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->bitems.p, items.data(), items.size() * sizeof(int2),
                         hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // `items` goes out of scope
    if (e != hipSuccess) return e;
    h->bitems_key = key;
  }
  for (size_t k = 0; k + 1 < starts.size(); ++k) {
    const int ab0 = starts[k], n = starts[k + 1] - starts[k];
    const long pt = bf16x3_panel_tiles(g, ab0, n);
    const long nit = h->bitems_off[k + 1] - h->bitems_off[k];
    if (2 * pt > 0x7fffffffL || nit > 0x7fffffffL || (long)nmb * (g.nbp - ab0) > 0x7fffffffL)
      return hipErrorInvalidValue;
    __bf16* Vdir = static_cast<__bf16*>(Vws);
    __bf16* Vmir = Vdir + (size_t)pt * VT;
    if (nit > 0)
      hipLaunchKernelGGL(k_vbuild, dim3((unsigned)nit), dim3(BWG), 0, st,
                         static_cast<const __bf16*>(Ls), tab,
                         h->bitems.as<int2>() + h->bitems_off[k], nonherm, g.nbv, g.nbp,
                         g.ncp / KB, g.v, ab0, Vdir, Vmir);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // parts per contraction list: the fewest that fill whole rounds of the
    // resident workgroups (two per CU) to within 5 %, at most 8
    const long items = (long)nmb * (g.nbp - ab0),
               slots = (cw == 4 ? 2L : 1L) * std::max(1, h->ncu);
    int nsplit = 1;
    double best = 0;
    // (deterministic mode: one part, no atomic additions)
    for (int sp = 1; sp <= (h->deterministic ? 1 : 8) && (long)sp * 4 <= g.nbp; ++sp) {
      const long tot = sp * items, rounds = (tot + slots - 1) / slots;
      const double eff = (double)tot / (double)(rounds * slots);
      if (eff > best + 1e-9) {
        best = eff;
        nsplit = sp;
      }
      if (eff >= 0.95) break;
    }
    if ((long)nsplit * items > 0x7fffffffL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(nsplit * items));
#define LRCC_KC(TA, NWV)                                                                       \
  hipLaunchKernelGGL((k_contract<TA, NWV>), grid, dim3(64 * NWV), 0, st,                        \
                     static_cast<const __bf16*>(Xb), Vdir, Vmir, g.nbp, (int)g.Mp, nmb, rb, ab0, \
                     ab0 + n, nx, (int)(n == g.nbp), static_cast<TA*>(Sb))
    if (acc64) {
      if (cw == 8) LRCC_KC(double, 8);
      else LRCC_KC(double, 4);
    } else {
      if (cw == 8) LRCC_KC(float, 8);
      else LRCC_KC(float, 4);
    }
#undef LRCC_KC
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lrcc
