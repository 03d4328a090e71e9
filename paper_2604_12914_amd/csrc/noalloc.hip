// The ladder product for callers that cannot allocate device memory.
//
// lrcc_ppl_sigma_noalloc runs the same kernels as lrcc_ppl_sigma (FP64 and
// FP32 arithmetic) but keeps every intermediate -- block-pair table, tile
// order, Hermiticity flag, staged Cholesky vectors, block-layout X and the
// sigma accumulator -- in one file-scope device array of fixed size instead
// of the handle's grow-only workspace.  Its address on each device is taken
// once, when the first handle on that device is created, and only that
// address (never the array's host-side name) reaches kernels.  The tables
// are written on the device by a kernel, so a call issues kernel launches
// only: no allocation, no host-to-device copy, no memset node.
#include <mutex>

#include "internal.hpp"

namespace lrcc {

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;  // per device, held until exit
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mutex;
void* g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};
bool g_done[MAX_DEVICES] = {};

// Block-pair table tab[bp] = (A << 16) | B (A <= B, row-major upper
// triangle of the virtual blocks) and the plain tile order: the tiles
// (ab, cd), cd >= ab, row after row, entry ab * nbp + cd.  One thread per
// block pair ab writes its table entry and its row of the order.
__global__ void k_plain_tables(int nbv, int nbp, int* __restrict__ tab, int* __restrict__ order) {
  for (int ab = blockIdx.x * blockDim.x + threadIdx.x; ab < nbp; ab += gridDim.x * blockDim.x) {
    int A = 0, start = 0;
    while (start + (nbv - A) <= ab) {
      start += nbv - A;
      ++A;
    }
    tab[ab] = (A << 16) | (A + ab - start);
    const long off = (long)ab * nbp - (long)ab * (ab - 1) / 2;
    for (int cd = ab; cd < nbp; ++cd) order[off + cd - ab] = ab * nbp + cd;
  }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

size_t noalloc_scratch_bytes() { return SCRATCH_BYTES; }

// Called by lrcc_create with `device` current: the device address of this
// device's copy of the scratch array, looked up once per device.
void noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_mutex);
  if (g_done[device]) return;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  g_ptr[device] = p;
  g_err[device] = e;
  g_done[device] = true;
}

// Scratch bytes a call needs (0 when nothing is to be done).
size_t noalloc_need(const Geom& g, lrcc_prec prec) {
  const long ntile = ppl_ntile(g);
  return align256((size_t)g.nbp * 4) + align256((size_t)ntile * 4) + 256 +
         align256(ppl_ls_bytes(prec, LRCC_CMUL_4M, g)) + align256(ppl_xb_bytes(prec, g)) +
         align256((size_t)2 * g.xb_plane() * 8);
}

lrcc_status sigma_noalloc(lrcc_handle h, const Geom& g, const void* L, const void* X, void* S,
                          lrcc_dtype dt, lrcc_prec prec, lrcc_cmul cmul) {
  const size_t es = dt == LRCC_C128 ? 16 : 8;
  if ((size_t)g.M * g.npv * es == 0) return LRCC_OK;
  if (prec == LRCC_BF16X3)
    return fail(h, LRCC_ERR_UNSUPPORTED,
                "the allocation-free ladder offers FP64 and FP32 arithmetic only");
  const size_t need = noalloc_need(g, prec);
  if (need > SCRATCH_BYTES)
    return fail(h, LRCC_ERR_SHAPE,
                "problem needs " + std::to_string(need) + " bytes of scratch; the allocation-"
                "free ladder holds at most " + std::to_string(SCRATCH_BYTES));
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mutex);
    if (h->device < 0 || h->device >= MAX_DEVICES || !g_done[h->device])
      return fail(h, LRCC_ERR_DEVICE, "scratch address of this device was not looked up");
    if (!g_ptr[h->device])
      return hip_fail(h, g_err[h->device], "hipGetSymbolAddress(scratch)");
    base = g_ptr[h->device];
  }
  char* p = static_cast<char*>(base);
  int* tab = reinterpret_cast<int*>(p);
  p += align256((size_t)g.nbp * 4);
  int* order = reinterpret_cast<int*>(p);
  p += align256((size_t)ppl_ntile(g) * 4);
  int* nonherm = reinterpret_cast<int*>(p);
  p += 256;
  void* Ls = p;
  p += align256(ppl_ls_bytes(prec, LRCC_CMUL_4M, g));
  void* Xb = p;
  p += align256(ppl_xb_bytes(prec, g));
  void* Sb = p;
  const bool acc64 = dt == LRCC_C128 || prec == LRCC_FP64;
  const size_t sbytes = (size_t)2 * g.xb_plane() * (acc64 ? 8 : 4);
  hipStream_t st = h->stream;
  hipLaunchKernelGGL(k_plain_tables, dim3((g.nbp + 63) / 64), dim3(64), 0, st, g.nbv, g.nbp, tab,
                     order);
  LRCC_HIP(h, hipGetLastError());
  LRCC_HIP(h, fill_zero(Sb, sbytes, st));
  if (g.nchol > 0) {
    LRCC_HIP(h, herm_check(L, dt, g.v, g.nchol, nonherm, st));
    if (prec == LRCC_FP64) {
      LRCC_HIP(h, stage_L<double>(L, dt, g, L_PLAIN, static_cast<double*>(Ls), st));
      LRCC_HIP(h, pack_to_block<double>(X, dt, g, tab, static_cast<double*>(Xb), st));
    } else {
      LRCC_HIP(h, stage_L<float>(L, dt, g, L_PLAIN, static_cast<float*>(Ls), st));
      LRCC_HIP(h, pack_to_block<float>(X, dt, g, tab, static_cast<float*>(Xb), st));
    }
    LRCC_HIP(h, ppl_launch(prec, cmul, acc64, g, Ls, Xb, Sb, tab, order, nonherm,
                           h->occ[prec][cmul], st));
  }
  if (acc64)
    LRCC_HIP(h, block_to_pack<double>(static_cast<double*>(Sb), g, tab, S, dt, st));
  else
    LRCC_HIP(h, block_to_pack<float>(static_cast<float*>(Sb), g, tab, S, dt, st));
  return LRCC_OK;
}

}  // namespace lrcc
