// Split-BF16 (bf16x3) ladder for gfx950.
//
// Every real operand x is split as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even), and a real product is taken as
// hi*hi + hi*lo + lo*hi (the lo*lo term is dropped), all on the bf16 matrix
// cores (16x16x32 MFMA) with FP32 accumulation.  Complex products use the
// 4M form, so one complex multiply-accumulate costs 12 bf16 MFMA products.
//
// The ladder is evaluated in panels of consecutive block pairs AB, each
// holding the tiles (AB, CD) with CD >= AB (the upper triangle of the block-
// pair matrix) in both orientations:
//   k_vbuild   one workgroup per upper tile (AB, CD): W1 = sum_P L_AC (x) L_BD
//              and W2 = sum_P L_AD (x) L_BC on the matrix cores,
//              antisymmetrised in LDS to V = 2 <ab||cd>, split to hi/lo and
//              written to the panel (32 KB per tile).  The mirror tile
//              V(CD, AB) goes beside it: for Hermitian L^P it is the conjugate
//              transpose of the tile just built (one build per pair), otherwise
//              a second wave of workgroups builds it (a flag set on the device
//              by the staging pass decides, so no host round trip);
//   k_contract sigma[m, Q] += sum_{CD >= Q} X[m, CD] V(Q, CD)^T
//                           + sum_{AB < Q, AB in panel} X[m, AB] V(Q, AB)^T,
//              a bf16x3 GEMM in which each workgroup owns its output tile
//              (128 rows x 64 slots of block pair Q) for the whole panel: no
//              atomics.  With one panel every workgroup runs over nbp tiles.
// The integral panel is transient: at most one panel exists.
// The reason for the split: the fused kernel's atomic accumulation of sigma
// across CD tiles runs at the device's atomic throughput, which caps the fast
// bf16 arithmetic; a panel costs one extra write and read of V per apply.
#include <hip/hip_bf16.h>

#include "internal.hpp"

namespace lrcc {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

constexpr int KB = 32;                 // Cholesky vectors per chunk (MFMA k)
constexpr int NPL = 4;                 // planes: re_hi, re_lo, im_hi, im_lo
constexpr int CHUNK = NPL * NS * KB;   // bf16 per block per chunk (16 KB)
constexpr int VT = NPL * NS * NS;      // bf16 per V tile (32 KB)
// LDS rows are padded so that the 8 lanes of one 16-byte LDS read phase hit
// distinct banks: operand rows of 32 bf16 (64 B) get a stride of 40 (80 B),
// V rows of 64 bf16 (128 B) a stride of 72 (144 B).
constexpr int KBP = KB + 8;
constexpr int CHUNKP = NPL * NS * KBP;  // padded chunk in LDS
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

// L -> Ls16[A][C][chunk][plane][64 (a,c)][32 P]
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
// V panel build.  Waves 0,1 build W1 rows (a,c) 0-31 / 32-63 x all (b,d);
// waves 2,3 build W2 rows (a,d) likewise x all (b,c).
// Tile index, within the panel that starts at block pair ab0, of the upper
// tile (ab0 + abl, cd), cd >= ab0 + abl: rows of the triangle one after another.
__device__ __forceinline__ long panel_tile(int nbp, int ab0, int abl, int cd) {
  return (long)abl * nbp - (long)abl * ab0 - (long)abl * (abl - 1) / 2 + (cd - ab0 - abl);
}

// Workgroup w < ptiles: upper tile order[w]; w >= ptiles: its mirror when L
// is not Hermitian (otherwise, or on the diagonal, nothing to do).
__global__ __launch_bounds__(WG, 2) void k_vbuild(const __bf16* __restrict__ Ls,
                                                  const int* __restrict__ tab,
                                                  const int* __restrict__ order,
                                                  const int* __restrict__ nonherm, int nbv,
                                                  int nbp, int ncp, int v, int ab0, long ptiles,
                                                  __bf16* __restrict__ Vdir,
                                                  __bf16* __restrict__ Vmir) {
  // two-chunk ring of column-side buffers during the build, then W1 and W2
  // (f32, rows padded to VR)
  constexpr int VR = NS + 1;
  constexpr int LDSB = 4 * CHUNKP > 2 * 4 * NS * VR ? 4 * CHUNKP : 2 * 4 * NS * VR;
  __shared__ __attribute__((aligned(16))) __bf16 lds[LDSB];  // 80 KB
  const bool nh = *nonherm != 0;
  const bool second = blockIdx.x >= ptiles;
  if (second && !nh) return;
  const int tile = order[second ? blockIdx.x - ptiles : blockIdx.x];
  const int abl = tile / nbp, cdu = tile - abl * nbp, abu = ab0 + abl;
  if (second && abu == cdu) return;
  const long t = panel_tile(nbp, ab0, abl, cdu);
  // built pair (ab, cd): the upper tile, or its mirror (cdu, abu)
  const int ab = second ? cdu : abu, cd = second ? abu : cdu;
  const int pAB = tab[ab], pCD = tab[cd];
  const int A = pAB >> 16, B = pAB & 0xffff, C = pCD >> 16, D = pCD & 0xffff;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wsel = wave >> 1, rb0 = (wave & 1) * 2;
  const int nch = ncp / KB;
  // row side (per wave, straight from global memory into registers) and
  // column side (shared by the two waves of one product, staged in LDS):
  // W1 = L_AC (x) L_BD for waves 0, 1; W2 = L_AD (x) L_BC for waves 2, 3
  const __bf16* const grow = Ls + (size_t)(wsel ? A * nbv + D : A * nbv + C) * nch * CHUNK;
  const __bf16* const gcol[2] = {Ls + (size_t)(B * nbv + D) * nch * CHUNK,
                                 Ls + (size_t)(B * nbv + C) * nch * CHUNK};

  f4 wr[2][4], wi[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      wr[i][j] = (f4){0, 0, 0, 0};
      wi[i][j] = wr[i][j];
    }

  constexpr int V16 = CHUNK / 8;        // 16-byte vectors per block chunk (1024)
  constexpr int KPB = V16 / WG;         // per thread per block (4)
  u4 pf[2 * KPB];
  // row-side fragments of even and odd chunks: [parity][MFMA block i][plane]
  bf8 ra[2][2][4];
  auto fetch_col = [&](int pc) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const u4* src = reinterpret_cast<const u4*>(gcol[q] + (size_t)pc * CHUNK);
#pragma unroll
      for (int k = 0; k < KPB; ++k) pf[q * KPB + k] = src[k * WG + threadIdx.x];
    }
  };
  // A fragment of MFMA block i, plane p: row 16 (rb0 + i) + li, P = 8 lk .. 8 lk + 7
  auto fetch_row = [&](int pc, int par) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        ra[par][i][p] = *reinterpret_cast<const bf8*>(
            grow + (size_t)pc * CHUNK + (p * NS + 16 * (rb0 + i) + li) * KB + 8 * lk);
  };
  auto store_col = [&](__bf16* buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int k = 0; k < KPB; ++k) {
        // vector e of the chunk: plane-row (e / 4), 8-bf16 part (e % 4)
        const int e = k * WG + threadIdx.x;
        *reinterpret_cast<u4*>(buf + q * CHUNKP + (e >> 2) * KBP + (e & 3) * 8) = pf[q * KPB + k];
      }
  };
  // W += A B over one chunk: re += Ar Br - Ai Bi, im += Ar Bi + Ai Br (the
  // minus sign on the Bi operand)
  auto mma = [&](const __bf16* buf, int par) {
    // column operands: [plane][row][32 P], lane reads 8 consecutive P at 8*lk
    const __bf16* lb = buf + wsel * CHUNKP + 8 * lk;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf8 b[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        b[p] = *reinterpret_cast<const bf8*>(lb + (p * NS + 16 * j + li) * KBP);
      const bf8 nb2 = neg(b[2]), nb3 = neg(b[3]);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const bf8 (&a)[4] = ra[par][i];
        wr[i][j] = mac3(a[0], a[1], b[0], b[1], wr[i][j]);  // Ar Br
        wr[i][j] = mac3(a[2], a[3], nb2, nb3, wr[i][j]);    // -Ai Bi
        wi[i][j] = mac3(a[0], a[1], b[2], b[3], wi[i][j]);  // Ar Bi
        wi[i][j] = mac3(a[2], a[3], b[0], b[1], wi[i][j]);  // Ai Br
      }
    }
  };
  // Two-chunk ring: chunk pc sits in buffer pc & 1 (row side in registers
  // ra[pc & 1]).  The next chunk is requested at the start of a chunk and
  // its column side stored to the free buffer at the end, so one barrier per
  // chunk suffices.  The loads of the last chunk repeat it (branch-free).
  // (Scheduling barriers keep each load group where it is issued and the
  // column loads ahead of the row loads, so that storing the column side
  // waits for those alone.)
  __bf16* const ring[2] = {lds, lds + 2 * CHUNKP};
  fetch_col(0);
  __builtin_amdgcn_sched_barrier(0);
  fetch_row(0, 0);
  store_col(ring[0]);
  for (int pc = 0; pc + 1 < nch; pc += 2) {
    __syncthreads();
    fetch_col(pc + 1);
    __builtin_amdgcn_sched_barrier(0);
    fetch_row(pc + 1, 1);
    __builtin_amdgcn_sched_barrier(0);
    mma(ring[0], 0);
    __builtin_amdgcn_sched_barrier(0);
    store_col(ring[1]);
    __syncthreads();
    fetch_col(min(pc + 2, nch - 1));
    __builtin_amdgcn_sched_barrier(0);
    fetch_row(min(pc + 2, nch - 1), 0);
    __builtin_amdgcn_sched_barrier(0);
    mma(ring[1], 1);
    __builtin_amdgcn_sched_barrier(0);
    store_col(ring[0]);
  }
  if (nch & 1) {  // the last chunk of an odd count
    __syncthreads();
    mma(ring[0], 0);
  }
  __syncthreads();

  // W1 and W2 to LDS, each already at its V position [ab slot][cd slot]
  // (plain stores by the two wave pairs at once), then the store loop forms
  // V = 2 (W1 - W2) on the live slots (a < b, c < d, inside v) on the fly
  float* const W1r = reinterpret_cast<float*>(lds);
  float* const W1i = W1r + NS * VR;
  float* const W2r = W1i + NS * VR;
  float* const W2i = W2r + NS * VR;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = 16 * (rb0 + i) + out_row(lk, r), jj = 16 * j + li;
        // W1: ii = (a,c), jj = (b,d);  W2: ii = (a,d), jj = (b,c)
        const int idx = wsel == 0
                            ? ((ii >> 3) * TB + (jj >> 3)) * VR + (ii & 7) * TB + (jj & 7)
                            : ((ii >> 3) * TB + (jj >> 3)) * VR + (jj & 7) * TB + (ii & 7);
        float* const wr_ = wsel == 0 ? W1r : W2r;
        float* const wi_ = wsel == 0 ? W1i : W2i;
        wr_[idx] = wr[i][j][r];
        wi_[idx] = wi[i][j][r];
      }
  __syncthreads();
  // split and write the tile as [plane][row slot][column slot]: the built
  // pair's V (rows ab) to the upper slot t, or, for a mirror workgroup, to
  // the mirror slot; for Hermitian L the conjugate transpose goes to the
  // mirror slot as well (V(cd, ab) = V(ab, cd)^H)
  auto store = [&](__bf16* dst, bool ct) {
    for (int w = threadIdx.x; w < NS * (NS / 8); w += WG) {
      const int row = w >> 3, q = (w & 7) * 8;
      bf8 rh, rl, ih, il;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        // element V[ab][cd] of the built pair
        const int ab = ct ? q + e : row, cd = ct ? row : q + e;
        const int al = ab >> 3, bl = ab & 7, cl = cd >> 3, dl = cd & 7;
        const bool live = (A < B || al < bl) && (B * TB + bl < v) && (C < D || cl < dl) &&
                          (D * TB + dl < v);
        const int idx = ab * VR + cd;
        const float vr = live ? 2.f * (W1r[idx] - W2r[idx]) : 0.f;
        const float vi = live ? 2.f * (W1i[idx] - W2i[idx]) : 0.f;
        __bf16 h, l;
        split(vr, h, l);
        rh[e] = h;
        rl[e] = l;
        split(ct ? -vi : vi, h, l);
        ih[e] = h;
        il[e] = l;
      }
      *reinterpret_cast<bf8*>(dst + 0 * NS * NS + row * NS + q) = rh;
      *reinterpret_cast<bf8*>(dst + 1 * NS * NS + row * NS + q) = rl;
      *reinterpret_cast<bf8*>(dst + 2 * NS * NS + row * NS + q) = ih;
      *reinterpret_cast<bf8*>(dst + 3 * NS * NS + row * NS + q) = il;
    }
  };
  store((second ? Vmir : Vdir) + t * VT, false);
  if (!second && !nh && abu != cdu) store(Vmir + t * VT, true);
}

// ---------------------------------------------------------------------------
// Contraction of one panel [ab0, ab1): workgroup (m-block of 128 rows, block
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
// Two workgroups per CU: while one waits for its X rows (loaded straight into
// registers, half a tile ahead) the other keeps the matrix cores busy.
template <typename TA>
__global__ __launch_bounds__(WG, 2) void k_contract(const __bf16* __restrict__ Xb,
                                                    const __bf16* __restrict__ Vdir,
                                                    const __bf16* __restrict__ Vmir, int nbp,
                                                    int Mp, int nmb, int ab0, int ab1, int nx,
                                                    int grouped, TA* __restrict__ Sb) {
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
  // rows of this wave; blocks past Mp (the last m-block of a short Mp) load
  // row block 0 instead, so every load is unconditional and in bounds, and
  // their sums are never stored
  int mrow[2], mld[2];
  bool mok[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    mrow[i] = mb * 128 + 32 * wave + 16 * i;
    mok[i] = mrow[i] < Mp;
    mld[i] = mok[i] ? mrow[i] : 0;
  }
  // a wave whose rows all lie past Mp (in the last m-block) still loads and
  // stores its share of every V tile but skips the matrix work
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
  constexpr int VH = VT / 8 / WG / 2;  // 16-byte vectors per thread per half tile (4)
  u4 vp[VH];
  int xnext = 0;
  const __bf16* vsrc = Vdir;
  auto fetch_v = [&](int h) {
#pragma unroll
    for (int k = 0; k < VH; ++k)
      vp[k] = reinterpret_cast<const u4*>(vsrc)[(h * VH + k) * WG + threadIdx.x];
  };
  auto store_v = [&](__bf16* buf, int h) {
#pragma unroll
    for (int k = 0; k < VH; ++k) {
      // vector e of the tile: plane-row (e / 8), 8-bf16 part (e % 8)
      const int e = (h * VH + k) * WG + threadIdx.x;
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

// Panels of consecutive block pairs, each as many rows as fit in `cap` bytes
// (at least one): build, then contract.  Sb (zeroed by the caller, FP64 or
// FP32 planes) receives the panels' shares.  *nonherm (device) selects the
// mirror tiles' source.
hipError_t bf16x3_run(lrcc_handle h, const Geom& g, const void* Ls, const void* Xb, void* Sb,
                      bool acc64, void* Vws, size_t cap, const int* tab, const int* nonherm,
                      hipStream_t st) {
  if (g.nbp == 0 || g.Mp == 0) return hipSuccess;
  const int nmb = (int)((g.Mp + 127) / 128);
  for (int ab0 = 0, n = 1; ab0 < g.nbp; ab0 += n) {
    n = 1;
    while (ab0 + n < g.nbp && bf16x3_panel_bytes(g, ab0, n + 1) <= cap) ++n;
    const long pt = bf16x3_panel_tiles(g, ab0, n);
    if (2 * pt > 0x7fffffffL || (long)nmb * (g.nbp - ab0) > 0x7fffffffL)
      return hipErrorInvalidValue;
    lrcc_status ost;
    const int* ord = tile_order(h, g, ab0, ab0 + n, true, LRCC_BF16X3, &ost);
    if (ost != LRCC_OK) return hipErrorUnknown;
    __bf16* Vdir = static_cast<__bf16*>(Vws);
    __bf16* Vmir = Vdir + (size_t)pt * VT;
    hipLaunchKernelGGL(k_vbuild, dim3((unsigned)(2 * pt)), dim3(WG), 0, st,
                       static_cast<const __bf16*>(Ls), tab, ord, nonherm, g.nbv, g.nbp, g.ncp,
                       g.v, ab0, pt, Vdir, Vmir);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // parts per contraction list: the fewest that fill whole rounds of the
    // resident workgroups (two per CU) to within 5 %, at most 8
    const long items = (long)nmb * (g.nbp - ab0), slots = 2L * std::max(1, h->ncu);
    int nsplit = 1;
    double best = 0;
    for (int sp = 1; sp <= 8 && (long)sp * 4 <= g.nbp; ++sp) {
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
    const int nx = std::max(1, h->ncu / 32);  // XCDs
    if (acc64)
      hipLaunchKernelGGL(k_contract<double>, grid, dim3(WG), 0, st,
                         static_cast<const __bf16*>(Xb), Vdir, Vmir, g.nbp, (int)g.Mp, nmb, ab0,
                         ab0 + n, nx, (int)(n == g.nbp), static_cast<double*>(Sb));
    else
      hipLaunchKernelGGL(k_contract<float>, grid, dim3(WG), 0, st,
                         static_cast<const __bf16*>(Xb), Vdir, Vmir, g.nbp, (int)g.Mp, nmb, ab0,
                         ab0 + n, nx, (int)(n == g.nbp), static_cast<float*>(Sb));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lrcc
