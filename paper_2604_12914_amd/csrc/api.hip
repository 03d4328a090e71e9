// C ABI entry points of the ladder library: handles, validation, sigma.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>

#include "internal.hpp"

namespace lrcc {

namespace {
thread_local std::string g_last_error;

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};
}  // namespace

lrcc_status fail(lrcc_handle h, lrcc_status s, const std::string& msg) {
  if (h) h->err = msg;
  g_last_error = msg;
  return s;
}

lrcc_status hip_fail(lrcc_handle h, hipError_t e, const char* what) {
  std::string m = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
  return fail(h, e == hipErrorOutOfMemory ? LRCC_ERR_NOMEM : LRCC_ERR_DEVICE, m);
}

Geom make_geom(int o, int v, int nchol, int nrhs, int kc) {
  Geom g;
  g.o = o;
  g.v = v;
  g.nchol = nchol;
  g.nrhs = nrhs;
  g.npo = npair(o);
  g.npv = npair(v);
  g.M = (long)nrhs * g.npo;
  g.Mp = roundup(g.M, 16);
  g.nbv = (v + TB - 1) / TB;
  g.nbp = g.nbv * (g.nbv + 1) / 2;
  g.ncp = (int)roundup(nchol, kc);
  return g;
}

hipError_t Buf::ensure(size_t bytes) {
  bytes = (size_t)roundup((long)(bytes ? bytes : 16), 256);
  if (bytes <= n) return hipSuccess;
  release();
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    p = nullptr;
    n = 0;
    (void)hipGetLastError();
    return e;
  }
  n = bytes;
  return hipSuccess;
}

void Buf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  n = 0;
}

lrcc_status ensure_tab(lrcc_handle h, int nbv) {
  if (h->tab_nbv == nbv) return LRCC_OK;
  std::vector<int> t;
  block_pair_table(nbv, &t);
  LRCC_HIP(h, h->tab.ensure(t.size() * sizeof(int)));
  LRCC_HIP(h, hipMemcpyAsync(h->tab.p, t.data(), t.size() * sizeof(int), hipMemcpyHostToDevice,
                             h->stream));
  LRCC_HIP(h, hipStreamSynchronize(h->stream));
  h->tab_nbv = nbv;
  return LRCC_OK;
}

void block_pair_table(int nbv, std::vector<int>* tab) {
  tab->clear();
  for (int A = 0; A < nbv; ++A)
    for (int B = A; B < nbv; ++B) tab->push_back((A << 16) | B);
  if (tab->empty()) tab->push_back(0);
}

void supertile_order(const Geom& g, int ab0, int ab1, int sw, int nx, bool upper,
                     std::vector<int>* ord) {
  const int nbv = g.nbv, nbp = g.nbp;
  std::vector<int> A(nbp), B(nbp);
  for (int a = 0, k = 0; a < nbv; ++a)
    for (int b = a; b < nbv; ++b, ++k) {
      A[k] = a;
      B[k] = b;
    }
  const int ng = (nbv + sw - 1) / sw;
  // groups of block pairs by (A / sw, B / sw)
  std::vector<std::vector<int>> gab((size_t)ng * ng), gcd((size_t)ng * ng);
  for (int bp = 0; bp < nbp; ++bp) {
    const size_t gk = (size_t)(A[bp] / sw) * ng + B[bp] / sw;
    gcd[gk].push_back(bp);
    if (bp >= ab0 && bp < ab1) gab[gk].push_back(bp);
  }
  std::vector<int> all;
  for (const auto& ga : gab) {
    if (ga.empty()) continue;
    for (const auto& gc : gcd) {
      if (gc.empty()) continue;
      for (int ab : ga)
        for (int cd : gc)
          if (!upper || cd >= ab) all.push_back((ab - ab0) * nbp + cd);
    }
  }
  const long total = (long)all.size();
  // contiguous share per XCD; workgroup w runs on XCD w % nx, as the j-th
  // (j = w / nx) of that XCD's workgroups
  const long q = total / nx, r = total % nx;
  ord->assign(total, 0);
  for (long w = 0; w < total; ++w) {
    const long x = w % nx, j = w / nx;
    (*ord)[w] = all[x * q + std::min<long>(x, r) + j];
  }
}

const int* tile_order(lrcc_handle h, const Geom& g, int ab0, int ab1, bool upper,
                      lrcc_prec prec, lrcc_status* st) {
  const int sw = h->order_s[prec] > 0 ? h->order_s[prec] : 4;
  const long key[6] = {g.nbv, ab0, ab1, sw, h->ncu, upper};
  long* okey = h->order_key[prec];
  Buf& obuf = h->order[prec];
  bool same = true;
  for (int k = 0; k < 6; ++k) same = same && key[k] == okey[k];
  if (same) {
    *st = LRCC_OK;
    return obuf.as<int>();
  }
  std::vector<int> ord;
  supertile_order(g, ab0, ab1, sw, std::max(1, h->ncu / 32), upper, &ord);
  hipError_t e = obuf.ensure(ord.size() * sizeof(int));
  if (e == hipSuccess)
    e = hipMemcpyAsync(obuf.p, ord.data(), ord.size() * sizeof(int), hipMemcpyHostToDevice,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    *st = hip_fail(h, e, "tile order upload");
    return nullptr;
  }
  for (int k = 0; k < 6; ++k) okey[k] = key[k];
  *st = LRCC_OK;
  return obuf.as<int>();
}

lrcc_status ppl_run(lrcc_handle h, lrcc_prec prec, lrcc_cmul cmul, bool acc64, const Geom& g,
                    const void* Ls, const void* Xb, void* Sb, const int* nonherm) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->timing) {
    if (h->tev.size() < 2 * (h->tev_used + 1)) {
      for (int k = 0; k < 2; ++k) {
        hipEvent_t e;
        LRCC_HIP(h, hipEventCreate(&e));
        h->tev.push_back(e);
      }
    }
    e0 = h->tev[2 * h->tev_used];
    e1 = h->tev[2 * h->tev_used + 1];
    LRCC_HIP(h, hipEventRecord(e0, h->stream));
  }
  if (h->deterministic) {
    LRCC_HIP(h, ppl_det_launch(prec, acc64, g, Ls, Xb, Sb, h->tab.as<int>(), h->stream));
  } else {
    lrcc_status ost;
    const int* ord = tile_order(h, g, 0, g.nbp, true, prec, &ost);
    if (ost != LRCC_OK) return ost;
    LRCC_HIP(h, ppl_launch(prec, cmul, acc64, g, Ls, Xb, Sb, h->tab.as<int>(), ord, nonherm,
                           h->occ[prec][cmul], h->stream));
  }
  if (h->timing) {
    LRCC_HIP(h, hipEventRecord(e1, h->stream));
    ++h->tev_used;
  }
  return LRCC_OK;
}

lrcc_status bf16x3_apply(lrcc_handle h, const Geom& g, const void* Ls, const void* Xb, void* Sb,
                         bool acc64, const int* nonherm) {
  if (h->panel_cap == 0) {
    size_t freeb = 0, totalb = 0;
    LRCC_HIP(h, hipMemGetInfo(&freeb, &totalb));
    size_t cap = (size_t)16 << 30;
    if (const char* e = getenv("LRCC_PANEL_MB")) cap = (size_t)atol(e) << 20;
    h->panel_cap = std::max<size_t>(std::min(cap, freeb / 2), (size_t)64 << 20);
  }
  // the workspace holds the largest panel: the whole triangle if it fits,
  // else as many rows as the limit allows (at least the first, longest row)
  const size_t need = std::min(bf16x3_panel_bytes(g, 0, g.nbp),
                               std::max(h->panel_cap, bf16x3_panel_bytes(g, 0, 1)));
  LRCC_HIP(h, h->vws.ensure(need));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->timing) {
    while (h->tev.size() < 2 * (h->tev_used + 1)) {
      hipEvent_t e;
      LRCC_HIP(h, hipEventCreate(&e));
      h->tev.push_back(e);
    }
    e0 = h->tev[2 * h->tev_used];
    e1 = h->tev[2 * h->tev_used + 1];
    LRCC_HIP(h, hipEventRecord(e0, h->stream));
  }
  LRCC_HIP(h, bf16x3_run(h, g, Ls, Xb, Sb, acc64, h->vws.p, need, h->tab.as<int>(), nonherm,
                         h->stream));
  if (h->timing) {
    LRCC_HIP(h, hipEventRecord(e1, h->stream));
    ++h->tev_used;
  }
  return LRCC_OK;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

static lrcc_status check_sigma(lrcc_handle h, int o, int v, int nchol, int nrhs, const void* L,
                               const void* X, const void* S, lrcc_dtype dt, lrcc_prec prec,
                               lrcc_cmul cmul, const char* sname, bool out_optional = false) {
  if (o < 0 || v < 0 || nchol < 0 || nrhs < 0)
    return fail(h, LRCC_ERR_ARG, "o, v, nchol and nrhs must be non-negative");
  if (dt != LRCC_C128 && dt != LRCC_C64) return fail(h, LRCC_ERR_ARG, "unknown dtype");
  if (prec != LRCC_FP64 && prec != LRCC_FP32 && prec != LRCC_BF16X3)
    return fail(h, LRCC_ERR_ARG, "unknown precision");
  if (cmul != LRCC_CMUL_4M && cmul != LRCC_CMUL_3M)
    return fail(h, LRCC_ERR_ARG, "unknown complex-multiply form");
  if (v > 4096) return fail(h, LRCC_ERR_SHAPE, "v exceeds 4096");
  if (nchol > 65536) return fail(h, LRCC_ERR_SHAPE, "nchol exceeds 65536");
  if (o > 65535 || nrhs > (1 << 24))  // (bounds the products below)
    return fail(h, LRCC_ERR_SHAPE, "nrhs*o(o-1)/2 exceeds 2^24");
  const long M = (long)nrhs * npair(o);
  if (M > (1L << 24)) return fail(h, LRCC_ERR_SHAPE, "nrhs*o(o-1)/2 exceeds 2^24");
  const size_t es = dt == LRCC_C128 ? 16 : 8;
  const size_t nx = (size_t)M * npair(v) * es;
  const size_t nl = (size_t)nchol * v * v * es;
  if (nx > 0) {
    if (!X) return fail(h, LRCC_ERR_ARG, "X is NULL");
    if (!S && !out_optional) return fail(h, LRCC_ERR_ARG, std::string(sname) + " is NULL");
    if ((uintptr_t)X % es || (uintptr_t)S % es)
      return fail(h, LRCC_ERR_ARG, "X/sigma not aligned to the element size");
    if (S && overlaps(X, nx, S, nx)) return fail(h, LRCC_ERR_ARG, "sigma overlaps X");
    if (nl > 0) {
      if (!L) return fail(h, LRCC_ERR_ARG, "L is NULL");
      if ((uintptr_t)L % es) return fail(h, LRCC_ERR_ARG, "L not aligned to the element size");
      if (S && overlaps(L, nl, S, nx)) return fail(h, LRCC_ERR_ARG, "sigma overlaps L");
    }
  }
  return LRCC_OK;
}

lrcc_status sigma_packed(lrcc_handle h, const Geom& g, const void* L, bool conj_t,
                         const void* X, void* S, lrcc_dtype dt, lrcc_prec prec,
                         lrcc_cmul cmul) {
  const size_t es = dt == LRCC_C128 ? 16 : 8;
  const size_t nx = (size_t)g.M * g.npv * es;
  if (nx == 0) return LRCC_OK;
  if (cmul == LRCC_CMUL_3M && prec == LRCC_BF16X3)
    return fail(h, LRCC_ERR_UNSUPPORTED, "bf16x3 uses the 4M complex form only");
  lrcc_status st = ensure_tab(h, g.nbv);
  if (st != LRCC_OK) return st;
  const int* tab = h->tab.as<int>();
  const bool acc64 = dt == LRCC_C128 || prec == LRCC_FP64;
  if (prec == LRCC_BF16X3) {
    Geom gb = g;
    gb.ncp = (int)roundup(g.nchol, bf16x3_chunk());
    const size_t sbytes = (size_t)2 * g.xb_plane() * (acc64 ? 8 : 4);
    LRCC_HIP(h, h->sb.ensure(sbytes));
    LRCC_HIP(h, fill_zero(h->sb.p, sbytes, h->stream));
    if (g.nchol > 0) {
      LRCC_HIP(h, h->ls.ensure(bf16x3_ls_bytes(gb)));
      LRCC_HIP(h, h->xb.ensure(bf16x3_xb_bytes(gb)));
      LRCC_HIP(h, bf16x3_stage_L(L, dt, gb, conj_t ? L_ADJ : L_PLAIN, h->ls.p, h->stream));
      LRCC_HIP(h, bf16x3_pack_x(X, dt, gb, tab, h->xb.p, h->stream));
      LRCC_HIP(h, h->hflag.ensure(16));
      LRCC_HIP(h, herm_check(L, dt, g.v, g.nchol, h->hflag.as<int>(), h->stream));
      st = bf16x3_apply(h, gb, h->ls.p, h->xb.p, h->sb.p, acc64, h->hflag.as<int>());
      if (st != LRCC_OK) return st;
    }
    if (acc64)
      LRCC_HIP(h, block_to_pack<double>(h->sb.as<double>(), g, tab, S, dt, h->stream));
    else
      LRCC_HIP(h, block_to_pack<float>(h->sb.as<float>(), g, tab, S, dt, h->stream));
    return LRCC_OK;
  }
  LRCC_HIP(h, h->ls.ensure(ppl_ls_bytes(prec, cmul, g)));
  LRCC_HIP(h, h->xb.ensure(ppl_xb_bytes(prec, g)));
  const size_t sbytes = (size_t)2 * g.xb_plane() * (acc64 ? 8 : 4);
  LRCC_HIP(h, h->sb.ensure(sbytes));
  LRCC_HIP(h, fill_zero(h->sb.p, sbytes, h->stream));
  if (g.nchol > 0) {
    LRCC_HIP(h, h->hflag.ensure(16));
    LRCC_HIP(h, herm_check(L, dt, g.v, g.nchol, h->hflag.as<int>(), h->stream));
    if (prec == LRCC_FP64) {
      LRCC_HIP(h, stage_L<double>(L, dt, g, conj_t ? L_ADJ : L_PLAIN, h->ls.as<double>(),
                                  h->stream));
      LRCC_HIP(h, pack_to_block<double>(X, dt, g, tab, h->xb.as<double>(), h->stream));
    } else {
      LRCC_HIP(h, stage_L<float>(L, dt, g, conj_t ? L_ADJ : L_PLAIN, h->ls.as<float>(),
                                 h->stream));
      LRCC_HIP(h, pack_to_block<float>(X, dt, g, tab, h->xb.as<float>(), h->stream));
    }
    st = ppl_run(h, prec, cmul, acc64, g, h->ls.p, h->xb.p, h->sb.p, h->hflag.as<int>());
    if (st != LRCC_OK) return st;
  }
  if (acc64)
    LRCC_HIP(h, block_to_pack<double>(h->sb.as<double>(), g, tab, S, dt, h->stream));
  else
    LRCC_HIP(h, block_to_pack<float>(h->sb.as<float>(), g, tab, S, dt, h->stream));
  return LRCC_OK;
}

}  // namespace lrcc

using namespace lrcc;

extern "C" {

lrcc_status lrcc_create(lrcc_handle* out, int device, void* stream) {
  if (!out) return fail(nullptr, LRCC_ERR_ARG, "handle pointer is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(nullptr, LRCC_ERR_DEVICE, "no HIP device");
  }
  if (device < 0 || device >= ndev) return fail(nullptr, LRCC_ERR_ARG, "device out of range");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess)
    return fail(nullptr, LRCC_ERR_DEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, LRCC_ERR_DEVICE,
                std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  lrcc_handle h = new (std::nothrow) lrcc_handle_s();
  if (!h) return fail(nullptr, LRCC_ERR_NOMEM, "out of host memory");
  h->device = device;
  h->stream = static_cast<hipStream_t>(stream);
  h->ncu = prop.multiProcessorCount;
  if (const char* e = getenv("LRCC_DETERMINISTIC")) h->deterministic = atoi(e) != 0;
  {
    DeviceGuard dg(device);
    noalloc_init(device);  // scratch address of the allocation-free ladder on this device
  }
  *out = h;
  return LRCC_OK;
}

lrcc_status lrcc_destroy(lrcc_handle h) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  {
    DeviceGuard dg(h->device);
    (void)hipStreamSynchronize(h->stream);
    h->ls.release();
    h->ls2.release();
    h->xb.release();
    h->sb.release();
    h->gb.release();
    h->tab.release();
    h->hflag.release();
    for (auto& b : h->order) b.release();
    h->vws.release();
    h->bitems.release();
    h->hw.release();
    h->cw.release();
    h->fw.release();
    h->rw.release();
    for (auto& b : h->sv) b.release();
    for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
    if (h->rb) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(h->rb));
  }
  delete h;
  return LRCC_OK;
}

lrcc_status lrcc_set_stream(lrcc_handle h, void* stream) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  h->stream = static_cast<hipStream_t>(stream);
  return LRCC_OK;
}

lrcc_status lrcc_autotune(lrcc_handle h, int o, int v, int nchol, int nrhs, lrcc_prec prec,
                          lrcc_cmul cmul, const char* cache_path, lrcc_tune_result* out) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  lrcc_status st = check_sigma(h, o, v, nchol, nrhs, (const void*)16, (const void*)16,
                               (const void*)(1L << 40), LRCC_C128, prec, cmul, "sigma");
  if (st != LRCC_OK) return st;
  if (prec == LRCC_BF16X3 && cmul == LRCC_CMUL_3M)
    return fail(h, LRCC_ERR_UNSUPPORTED, "bf16x3 uses the 4M complex form only");
  DeviceGuard dg(h->device);
  h->err.clear();
  return autotune_impl(h, o, v, nchol, nrhs, prec, cmul, cache_path, out);
}

lrcc_status lrcc_set_timing(lrcc_handle h, int enable) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  h->timing = enable != 0;
  h->tev_used = 0;
  return LRCC_OK;
}

lrcc_status lrcc_set_deterministic(lrcc_handle h, int enable) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  h->deterministic = enable != 0;
  return LRCC_OK;
}

lrcc_status lrcc_set_workspace_limit(lrcc_handle h, size_t bytes) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  h->panel_cap = bytes;
  return LRCC_OK;
}

lrcc_status lrcc_get_timing(lrcc_handle h, double* ms, long* launches) {
  if (!h || !ms || !launches) return fail(h, LRCC_ERR_ARG, "NULL argument");
  DeviceGuard dg(h->device);
  LRCC_HIP(h, hipStreamSynchronize(h->stream));
  double total = 0;
  for (size_t k = 0; k < h->tev_used; ++k) {
    float t = 0;
    LRCC_HIP(h, hipEventElapsedTime(&t, h->tev[2 * k], h->tev[2 * k + 1]));
    total += t;
  }
  *ms = total;
  *launches = (long)h->tev_used;
  return LRCC_OK;
}

lrcc_status lrcc_check_sigma_args(int o, int v, int nchol, int nrhs, const void* L, const void* X,
                                  const void* sigma, lrcc_dtype dt, lrcc_prec prec,
                                  lrcc_cmul cmul) {
  return check_sigma(nullptr, o, v, nchol, nrhs, L, X, sigma, dt, prec, cmul, "sigma");
}

lrcc_status lrcc_ppl_sigma(lrcc_handle h, int o, int v, int nchol, int nrhs, const void* L,
                           const void* X, void* sigma, lrcc_dtype dt, lrcc_prec prec,
                           lrcc_cmul cmul) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  lrcc_status st = check_sigma(h, o, v, nchol, nrhs, L, X, sigma, dt, prec, cmul, "sigma");
  if (st != LRCC_OK) return st;
  DeviceGuard dg(h->device);
  h->err.clear();
  Geom g = make_geom(o, v, nchol, nrhs, ppl_chunk(prec, cmul));
  return sigma_packed(h, g, L, false, X, sigma, dt, prec, cmul);
}

lrcc_status lrcc_ppl_sigma_noalloc(lrcc_handle h, int o, int v, int nchol, int nrhs,
                                   const void* L, const void* X, void* sigma, lrcc_dtype dt,
                                   lrcc_prec prec, lrcc_cmul cmul) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  lrcc_status st = check_sigma(h, o, v, nchol, nrhs, L, X, sigma, dt, prec, cmul, "sigma");
  if (st != LRCC_OK) return st;
  DeviceGuard dg(h->device);
  h->err.clear();
  const Geom g = make_geom(o, v, nchol, nrhs, ppl_chunk(prec, cmul));
  return sigma_noalloc(h, g, L, X, sigma, dt, prec, cmul);
}

lrcc_status lrcc_hhl_sigma(lrcc_handle h, int o, int v, int nchol, int nrhs, const void* Loo,
                           const void* X, void* sigma, lrcc_dtype dt) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  if (o < 0 || v < 0 || nchol < 0 || nrhs < 0)
    return fail(h, LRCC_ERR_ARG, "o, v, nchol and nrhs must be non-negative");
  if (dt != LRCC_C128 && dt != LRCC_C64) return fail(h, LRCC_ERR_ARG, "unknown dtype");
  if (v > 4096) return fail(h, LRCC_ERR_SHAPE, "v exceeds 4096");
  if (o > 4096) return fail(h, LRCC_ERR_SHAPE, "o exceeds 4096");
  if (nchol > 65536) return fail(h, LRCC_ERR_SHAPE, "nchol exceeds 65536");
  const long M = (long)nrhs * npair(o);
  if (M > (1L << 24)) return fail(h, LRCC_ERR_SHAPE, "nrhs*o(o-1)/2 exceeds 2^24");
  if (nrhs > 65535) return fail(h, LRCC_ERR_SHAPE, "nrhs exceeds 65535");
  const size_t es = dt == LRCC_C128 ? 16 : 8;
  const size_t nx = (size_t)M * npair(v) * es;
  const size_t nl = (size_t)nchol * o * o * es;
  if (nx == 0) return LRCC_OK;
  if (!X || !sigma) return fail(h, LRCC_ERR_ARG, "X or sigma is NULL");
  if ((uintptr_t)X % es || (uintptr_t)sigma % es)
    return fail(h, LRCC_ERR_ARG, "X/sigma not aligned to the element size");
  if (overlaps(X, nx, sigma, nx)) return fail(h, LRCC_ERR_ARG, "sigma overlaps X");
  if (nl > 0) {
    if (!Loo) return fail(h, LRCC_ERR_ARG, "Loo is NULL");
    if ((uintptr_t)Loo % es) return fail(h, LRCC_ERR_ARG, "Loo not aligned to the element size");
    if (overlaps(Loo, nl, sigma, nx)) return fail(h, LRCC_ERR_ARG, "sigma overlaps Loo");
  }
  DeviceGuard dg(h->device);
  h->err.clear();
  const Geom g = make_geom(o, v, nchol, nrhs, 1);
  lrcc_status st = ensure_tab(h, g.nbv);
  if (st != LRCC_OK) return st;
  const int* tab = h->tab.as<int>();
  const size_t vb = (size_t)2 * g.xb_plane() * 8;
  LRCC_HIP(h, h->xb.ensure(vb));
  LRCC_HIP(h, h->sb.ensure(vb));
  const size_t wbytes = roundup((size_t)g.npo * g.npo * 16, 256);
  LRCC_HIP(h, h->hw.ensure(wbytes + (size_t)g.npo * 4));
  double2* W = h->hw.as<double2>();
  int* otab = reinterpret_cast<int*>(h->hw.as<char>() + wbytes);
  LRCC_HIP(h, pack_to_block<double>(X, dt, g, tab, h->xb.as<double>(), h->stream));
  LRCC_HIP(h, fill_zero(h->sb.p, vb, h->stream));
  LRCC_HIP(h, hh_pair_table(o, otab, h->stream));
  LRCC_HIP(h, hh_build_w(Loo, dt, o, nchol, otab, L_PLAIN, 2.0, W, h->stream));
  LRCC_HIP(h, hh_apply(W, g, h->xb.as<double>(), h->sb.as<double>(), h->stream));
  LRCC_HIP(h, block_to_pack<double>(h->sb.as<double>(), g, tab, sigma, dt, h->stream));
  return LRCC_OK;
}

lrcc_status lrcc_cholesky(lrcc_handle h, long n, const void* M, double tau, int max_vectors,
                          void* L, int* pivots, int* nvec) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  if (!nvec) return fail(h, LRCC_ERR_ARG, "nvec is NULL");
  *nvec = 0;
  if (n < 0 || max_vectors < 0) return fail(h, LRCC_ERR_ARG, "n and max_vectors must be >= 0");
  if (!(tau >= 0) || tau > 1e300) return fail(h, LRCC_ERR_ARG, "tau must be finite and >= 0");
  if (n > (1L << 20)) return fail(h, LRCC_ERR_SHAPE, "n exceeds 2^20");
  if (max_vectors > n) max_vectors = (int)n;
  if (n == 0 || max_vectors == 0) return LRCC_OK;
  if (!M || !L) return fail(h, LRCC_ERR_ARG, "M or L is NULL");
  if ((uintptr_t)M % 16 || (uintptr_t)L % 16)
    return fail(h, LRCC_ERR_ARG, "M/L not aligned to 16 bytes");
  const size_t nm = (size_t)n * n * 16, nl = (size_t)max_vectors * n * 16;
  if (overlaps(M, nm, L, nl)) return fail(h, LRCC_ERR_ARG, "L overlaps M");
  if (pivots && ((uintptr_t)pivots % 4 || overlaps(pivots, (size_t)max_vectors * 4, L, nl) ||
                 overlaps(pivots, (size_t)max_vectors * 4, M, nm)))
    return fail(h, LRCC_ERR_ARG, "pivots misaligned or overlapping M/L");
  DeviceGuard dg(h->device);
  h->err.clear();
  LRCC_HIP(h, h->cw.ensure(chol_state_bytes(n)));
  LRCC_HIP(h, chol_run(n, M, tau, max_vectors, L, pivots, h->cw.p, nvec, h->stream));
  return LRCC_OK;
}

lrcc_status lrcc_ring_sigma(lrcc_handle h, int o, int v, int nchol, int nrhs, const void* L_oo,
                            const void* L_ov, const void* L_vo, const void* L_vv, const void* X,
                            void* sigma) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  if (o < 0 || v < 0 || nchol < 0 || nrhs < 0)
    return fail(h, LRCC_ERR_ARG, "sizes must be non-negative");
  const long ov = (long)o * v;
  if (ov > 65535) return fail(h, LRCC_ERR_SHAPE, "o v exceeds 65535");
  if ((long)nrhs * ov >= (1L << 31)) return fail(h, LRCC_ERR_SHAPE, "nrhs o v reaches 2^31");
  const size_t nx = (size_t)nrhs * npair(o) * npair(v) * 16;
  if (nx == 0) return LRCC_OK;
  if (!X || !sigma) return fail(h, LRCC_ERR_ARG, "X or sigma is NULL");
  const size_t no = (size_t)nchol * o * o * 16, nov = (size_t)nchol * ov * 16,
               nv = (size_t)nchol * v * v * 16;
  if (nchol > 0 && (!L_oo || !L_ov || !L_vo || !L_vv))
    return fail(h, LRCC_ERR_ARG, "a Cholesky block is NULL");
  const void* ptrs[] = {L_oo, L_ov, L_vo, L_vv, X, sigma};
  for (const void* q : ptrs)
    if (q && (uintptr_t)q % 16) return fail(h, LRCC_ERR_ARG, "a buffer is not 16-byte aligned");
  if (overlaps(sigma, nx, X, nx) || (nchol > 0 && (overlaps(sigma, nx, L_oo, no) ||
                                                   overlaps(sigma, nx, L_ov, nov) ||
                                                   overlaps(sigma, nx, L_vo, nov) ||
                                                   overlaps(sigma, nx, L_vv, nv))))
    return fail(h, LRCC_ERR_ARG, "sigma overlaps an input");
  DeviceGuard dg(h->device);
  h->err.clear();
  LRCC_HIP(h, h->rw.ensure(ring_ws_bytes(o, v, nrhs)));
  return ring_run(h, o, v, nchol, nrhs, L_oo, L_ov, L_vo, L_vv, X, sigma, false, h->rw.p);
}

lrcc_status lrcc_fns_transform(lrcc_handle h, int v, int k, int nchol, int ncomp, int o,
                               const void* B, const void* L, const void* mu, void* Lt,
                               void* mu_t) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  if (v < 0 || k < 0 || nchol < 0 || ncomp < 0 || o < 0)
    return fail(h, LRCC_ERR_ARG, "sizes must be non-negative");
  if (k > v) return fail(h, LRCC_ERR_ARG, "k exceeds v");
  if ((L != nullptr) != (Lt != nullptr) || (mu != nullptr) != (mu_t != nullptr))
    return fail(h, LRCC_ERR_ARG, "L/Lt and mu/mu_t come in pairs");
  const size_t nb = (size_t)v * k * 16, nl = (size_t)nchol * v * v * 16,
               nlt = (size_t)nchol * k * k * 16, nm = (size_t)ncomp * o * v * 16,
               nmt = (size_t)ncomp * o * k * 16;
  const bool dol = L && nlt > 0, dom = mu && nmt > 0;
  if (!dol && !dom) return LRCC_OK;
  if (!B) return fail(h, LRCC_ERR_ARG, "B is NULL");
  const void* ps[] = {B, L, mu, Lt, mu_t};
  for (const void* q : ps)
    if (q && (uintptr_t)q % 16) return fail(h, LRCC_ERR_ARG, "a buffer is not 16-byte aligned");
  if ((dol && (overlaps(Lt, nlt, L, nl) || overlaps(Lt, nlt, B, nb) ||
               (dom && (overlaps(Lt, nlt, mu, nm) || overlaps(Lt, nlt, mu_t, nmt))))) ||
      (dom && (overlaps(mu_t, nmt, mu, nm) || overlaps(mu_t, nmt, B, nb) ||
               (dol && overlaps(mu_t, nmt, L, nl)))))
    return fail(h, LRCC_ERR_ARG, "an output overlaps an input or the other output");
  DeviceGuard dg(h->device);
  h->err.clear();
  LRCC_HIP(h, h->rw.ensure(fns_transform_ws_bytes(v, k, dol ? nchol : 0) + 256));
  return fns_transform(h, v, k, dol ? nchol : 0, dom ? ncomp * o : 0, B, L, mu, Lt, mu_t,
                       h->rw.p);
}

lrcc_status lrcc_heev(lrcc_handle h, int n, const void* A, double* w, void* V, int* sweeps) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  if (sweeps) *sweeps = 0;
  if (n < 0) return fail(h, LRCC_ERR_ARG, "n must be >= 0");
  if (n > 8192) return fail(h, LRCC_ERR_SHAPE, "n exceeds 8192");
  if (n == 0) return LRCC_OK;
  if (!A || !w) return fail(h, LRCC_ERR_ARG, "A or w is NULL");
  if ((uintptr_t)A % 16 || (uintptr_t)w % 8 || (V && (uintptr_t)V % 16))
    return fail(h, LRCC_ERR_ARG, "A/V not aligned to 16 bytes or w to 8");
  const size_t na = (size_t)n * n * 16;
  if (overlaps(w, (size_t)n * 8, A, na) || (V && (overlaps(V, na, A, na) ||
                                                  overlaps(V, na, w, (size_t)n * 8))))
    return fail(h, LRCC_ERR_ARG, "outputs overlap A or each other");
  DeviceGuard dg(h->device);
  h->err.clear();
  LRCC_HIP(h, h->fw.ensure(heev_ws_bytes(n)));
  LRCC_HIP(h, heev_run(n, A, 0, w, V, V ? n : 0, h->fw.p, nullptr, sweeps, h->stream));
  LRCC_HIP(h, hipStreamSynchronize(h->stream));
  return LRCC_OK;
}

lrcc_status lrcc_fns_plus(lrcc_handle h, int o, int v, int nchol, const double* eps,
                          const void* Lov, int ncomp, const void* A_ov, const void* A_vv,
                          const void* A_oo, double omega, double threshold, double* occ,
                          void* B, double* eps_new, int* keep, void* gamma, double* hbar,
                          lrcc_fns_info* info) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  if (!keep) return fail(h, LRCC_ERR_ARG, "keep is NULL");
  *keep = 0;
  if (info) *info = lrcc_fns_info{};
  if (o < 0 || v < 0 || nchol < 0 || ncomp < 0)
    return fail(h, LRCC_ERR_ARG, "sizes must be non-negative");
  if (!(threshold >= 0) || threshold > 1e300)
    return fail(h, LRCC_ERR_ARG, "threshold must be finite and >= 0");
  if (!(std::fabs(omega) <= 1e300)) return fail(h, LRCC_ERR_ARG, "omega must be finite");
  if (o > 255) return fail(h, LRCC_ERR_SHAPE, "o exceeds 255");
  if (v > 8192) return fail(h, LRCC_ERR_SHAPE, "v exceeds 8192");
  if ((long)o * v * v >= (1L << 31)) return fail(h, LRCC_ERR_SHAPE, "o v^2 reaches 2^31");
  if (v == 0) return LRCC_OK;
  const size_t ne = (size_t)o + v, nl = (size_t)nchol * o * v * 16;
  const size_t nov = (size_t)ncomp * o * v * 16, nvv = (size_t)ncomp * v * v * 16,
               noo = (size_t)ncomp * o * o * 16;
  if (!eps || !B || !eps_new) return fail(h, LRCC_ERR_ARG, "eps, B or eps_new is NULL");
  if (nl && o && !Lov) return fail(h, LRCC_ERR_ARG, "Lov is NULL");
  if (ncomp && (!A_vv || (o && (!A_ov || !A_oo))))
    return fail(h, LRCC_ERR_ARG, "a perturbation block is NULL");
  auto mis = [](const void* p, size_t a) { return p && (uintptr_t)p % a != 0; };
  if (mis(eps, 8) || mis(Lov, 16) || mis(A_ov, 16) || mis(A_vv, 16) || mis(A_oo, 16) ||
      mis(occ, 8) || mis(B, 16) || mis(eps_new, 8) || mis(gamma, 16) || mis(hbar, 8))
    return fail(h, LRCC_ERR_ARG, "a buffer is misaligned (complex: 16 bytes, real: 8)");
  const size_t nvv1 = (size_t)v * v * 16;
  struct Rg { const void* p; size_t n; };
  const Rg in[] = {{eps, ne * 8}, {Lov, o ? nl : 0}, {A_ov, o ? nov : 0}, {A_vv, nvv},
                   {A_oo, o ? noo : 0}};
  const Rg out[] = {{occ, (size_t)v * 8}, {B, nvv1}, {eps_new, (size_t)v * 8},
                    {gamma, nvv1}, {hbar, ne * 8}};
  for (const Rg& a : out) {
    if (!a.p) continue;
    for (const Rg& b : in)
      if (b.p && b.n && overlaps(a.p, a.n, b.p, b.n))
        return fail(h, LRCC_ERR_ARG, "an output overlaps an input");
    for (const Rg& b : out)
      if (&b != &a && b.p && overlaps(a.p, a.n, b.p, b.n))
        return fail(h, LRCC_ERR_ARG, "outputs overlap each other");
  }
  DeviceGuard dg(h->device);
  h->err.clear();
  LRCC_HIP(h, h->fw.ensure(fns_ws_bytes(o, v, ncomp)));
  return fns_run(h, o, v, nchol, eps, Lov, ncomp, A_ov, A_vv, A_oo, omega, threshold, occ, B,
                 eps_new, keep, gamma, hbar, h->fw.p, info);
}

lrcc_status lrcc_ppl_sigma_adjoint(lrcc_handle h, int o, int v, int nchol, int nrhs,
                                   const void* L, const void* X, const void* G, void* dX,
                                   void* dL, lrcc_dtype dt, lrcc_prec prec, lrcc_cmul cmul) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  lrcc_status st = check_sigma(h, o, v, nchol, nrhs, L, G, dX, dt, prec, cmul, "dX", true);
  if (st != LRCC_OK) return st;
  if (dL) {
    const size_t es = dt == LRCC_C128 ? 16 : 8;
    const size_t nl = (size_t)nchol * v * v * es;
    const size_t nx = (size_t)nrhs * npair(o) * npair(v) * es;
    if (nl > 0 && ((uintptr_t)dL % es || overlaps(dL, nl, L, nl) ||
                   (nx > 0 && (overlaps(dL, nl, X, nx) || overlaps(dL, nl, G, nx)))))
      return fail(h, LRCC_ERR_ARG, "dL misaligned or overlapping an input");
    if (nx > 0 && !X) return fail(h, LRCC_ERR_ARG, "X is NULL");
  }
  DeviceGuard dg(h->device);
  h->err.clear();
  Geom g = make_geom(o, v, nchol, nrhs, ppl_chunk(prec, cmul));
  if (dX) {
    // the adjoint ladder: sigma with (L^P)^H, applied to G
    st = sigma_packed(h, g, L, true, G, dX, dt, prec, cmul);
    if (st != LRCC_OK) return st;
  }
  if (dL) {
    st = grad_L(h, g, L, X, G, dL, dt);
    if (st != LRCC_OK) return st;
  }
  return LRCC_OK;
}

lrcc_status lrcc_solve(lrcc_handle h, int o, int v, int nchol, const double* eps, const void* L,
                       int ncomp, const void* mu, int nomega, const double* omegas,
                       const lrcc_solve_opts* opts, double* alpha, lrcc_solve_info* info) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  if (o < 0 || v < 0 || nchol < 0 || ncomp < 0 || nomega < 0)
    return fail(h, LRCC_ERR_ARG, "sizes must be non-negative");
  if (v > 4096) return fail(h, LRCC_ERR_SHAPE, "v exceeds 4096");
  if (nchol > 65536) return fail(h, LRCC_ERR_SHAPE, "nchol exceeds 65536");
  if ((long)nomega * ncomp > 4096) return fail(h, LRCC_ERR_SHAPE, "more than 4096 right-hand sides");
  if (o > 65535 || (long)nomega * ncomp * npair(o) > (1L << 24))
    return fail(h, LRCC_ERR_SHAPE, "nomega*ncomp*o(o-1)/2 exceeds 2^24");
  if (nomega * ncomp > 0) {
    if (!alpha) return fail(h, LRCC_ERR_ARG, "alpha is NULL");
    if (!omegas) return fail(h, LRCC_ERR_ARG, "omegas is NULL");
    if (o + v > 0 && !eps) return fail(h, LRCC_ERR_ARG, "eps is NULL");
    if (o > 0 && v > 0 && !mu) return fail(h, LRCC_ERR_ARG, "mu is NULL");
    if (nchol > 0 && v > 0 && !L) return fail(h, LRCC_ERR_ARG, "L is NULL");
    if ((uintptr_t)L % 16 || (uintptr_t)mu % 16 || (uintptr_t)eps % 8)
      return fail(h, LRCC_ERR_ARG, "L/mu must be 16-byte and eps 8-byte aligned");
  }
  DeviceGuard dg(h->device);
  h->err.clear();
  return solve_impl(h, o, v, nchol, eps, L, ncomp, mu, nomega, omegas, opts, alpha, info);
}

lrcc_status lrcc_solve_batched(lrcc_handle h, int ninst, const lrcc_instance* inst,
                               const lrcc_solve_opts* opts, lrcc_solve_info* info) {
  if (!h) return fail(nullptr, LRCC_ERR_ARG, "handle is NULL");
  if (ninst < 0 || (ninst > 0 && !inst)) return fail(h, LRCC_ERR_ARG, "bad instance list");
  for (int i = 0; i < ninst; ++i) {
    const lrcc_instance& I = inst[i];
    const std::string w = "instance " + std::to_string(i) + ": ";
    if (I.o < 0 || I.v < 0 || I.nchol < 0 || I.ncomp < 0 || I.nomega < 0)
      return fail(h, LRCC_ERR_ARG, w + "sizes must be non-negative");
    if (I.v > 4096 || I.nchol > 65536) return fail(h, LRCC_ERR_SHAPE, w + "v or nchol too large");
    if ((long)I.nomega * I.ncomp > 4096 || I.o > 65535 ||
        (long)I.nomega * I.ncomp * npair(I.o) > (1L << 24))
      return fail(h, LRCC_ERR_SHAPE, w + "too many right-hand sides");
    if (I.nomega * I.ncomp > 0) {
      if (!I.alpha || !I.omegas) return fail(h, LRCC_ERR_ARG, w + "alpha or omegas is NULL");
      if (I.o + I.v > 0 && !I.eps) return fail(h, LRCC_ERR_ARG, w + "eps is NULL");
      if (I.o > 0 && I.v > 0 && !I.mu) return fail(h, LRCC_ERR_ARG, w + "mu is NULL");
      if (I.nchol > 0 && I.v > 0 && !I.L) return fail(h, LRCC_ERR_ARG, w + "L is NULL");
      if ((uintptr_t)I.L % 16 || (uintptr_t)I.mu % 16 || (uintptr_t)I.eps % 8)
        return fail(h, LRCC_ERR_ARG, w + "misaligned L, mu or eps");
    }
  }
  DeviceGuard dg(h->device);
  h->err.clear();
  return solve_batched_impl(h, ninst, inst, opts, info);
}

const char* lrcc_status_str(lrcc_status s) {
  switch (s) {
    case LRCC_OK: return "ok";
    case LRCC_ERR_ARG: return "invalid argument";
    case LRCC_ERR_SHAPE: return "invalid shape";
    case LRCC_ERR_DTYPE: return "unsupported dtype";
    case LRCC_ERR_DEVICE: return "device error";
    case LRCC_ERR_NOMEM: return "out of memory";
    case LRCC_ERR_NOT_CONVERGED: return "not converged";
    case LRCC_ERR_NONFINITE: return "non-finite value";
    case LRCC_ERR_UNSUPPORTED: return "unsupported";
    default: break;
  }
  return "unknown status";
}

const char* lrcc_last_error(lrcc_handle h) {
  return h ? h->err.c_str() : g_last_error.c_str();
}

const char* lrcc_version(void) { return "lrcc 0.1 (gfx950)"; }

}  // extern "C"
