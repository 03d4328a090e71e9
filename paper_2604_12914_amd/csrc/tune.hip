// Tile-shape autotuner of the ladder launch (lrcc_autotune).
//
// Candidates: the super-tile width s of the tile order (2, 4, 8 blocks of
// virtual indices, capped by the number of blocks) and the launch variants
// of the fused 4M kernel that exist for the precision (one or two workgroups
// per CU; chunks through registers or loaded straight into LDS).  Each candidate runs the
// ladder on synthetic inputs (Hermitian L^P) of a slice of the requested shape (at most
// v = 256, nchol = 512; one warm-up, then the best of two HIP-event-timed
// launches); the fastest is kept in the handle.  The cache key keeps the
// requested shape.
// Results are cached in a plain text file, one line per key:
//   <arch> <cu> <o> <v> <nchol> <nrhs> <prec> <cmul> <s> <occ> <ms>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"

namespace lrcc {

namespace {

// Deterministic pseudo-random fill in [-1, 1) (splitmix64 of the index).
__global__ void k_fill_uniform(double* p, size_t n, unsigned long long seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

// Make every L^P Hermitian (the structure of Cholesky vectors of a Hermitian
// Coulomb metric): lower triangle = conj(upper), real diagonal.
__global__ void k_hermitize(double2* L, int v, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    const int c = e % v, a = (e / v) % v;
    if (a > c) {
      const double2 z = L[e - (long)(a - c) * (v - 1)];  // element (c, a)
      L[e] = make_double2(z.x, -z.y);
    } else if (a == c) {
      L[e].y = 0.0;
    }
  }
}

std::string tune_key(lrcc_handle h, int o, int v, int nchol, int nrhs, lrcc_prec prec,
                     lrcc_cmul cmul) {
  std::ostringstream k;
  k << "gfx950 " << h->ncu << " " << o << " " << v << " " << nchol << " " << nrhs << " "
    << (int)prec << " " << (int)cmul;
  return k.str();
}

}  // namespace

lrcc_status autotune_impl(lrcc_handle h, int o, int v, int nchol, int nrhs, lrcc_prec prec,
                          lrcc_cmul cmul, const char* cache_path, lrcc_tune_result* out) {
  if (prec == LRCC_BF16X3) {
    // the bf16x3 build has one launch form and a fixed work order (super-
    // tiles of 4 blocks): nothing to time
    h->order_s[prec] = 0;
    if (out) *out = lrcc_tune_result{4, 1, 0.0, 0};
    return LRCC_OK;
  }
  const std::string key = tune_key(h, o, v, nchol, nrhs, prec, cmul);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() ||
          line[key.size()] != ' ')
        continue;
      std::istringstream rest(line.substr(key.size()));
      int s = 0, occ = 0;
      double ms = 0;
      if (rest >> s >> occ >> ms && s > 0 && occ >= 1 && occ <= 5) {
        h->order_s[prec] = s;
        h->occ[prec][cmul] = occ;
        if (out) *out = lrcc_tune_result{s, occ, ms, 0};
        return LRCC_OK;
      }
    }
  }
  // time a reduced shape: the variants differ in per-tile efficiency, which a
  // slice of at most 32 virtual blocks and 512 Cholesky vectors ranks the
  // same way at a small fraction of the cost of the full ladder
  v = std::min(v, 256);
  nchol = std::min(nchol, 512);
  Geom g = make_geom(o, v, nchol, nrhs, 1);
  if (g.M == 0 || g.npv == 0 || nchol == 0) {
    if (out) *out = lrcc_tune_result{h->order_s[prec] > 0 ? h->order_s[prec] : 4, 1, 0.0, 0};
    return LRCC_OK;
  }
  // synthetic inputs in the packed public layout
  const size_t nl = (size_t)nchol * v * v * 2, nx = (size_t)g.M * g.npv * 2;
  Buf in;
  struct Free {
    Buf* b;
    ~Free() { b->release(); }
  } fr{&in};
  LRCC_HIP(h, in.ensure((nl + 2 * nx) * sizeof(double)));
  double* L = in.as<double>();
  double* X = L + nl;
  double* S = X + nx;
  hipLaunchKernelGGL(k_fill_uniform, dim3(1024), dim3(256), 0, h->stream, L, nl, 1ull);
  hipLaunchKernelGGL(k_fill_uniform, dim3(1024), dim3(256), 0, h->stream, X, nx, 2ull);
  hipLaunchKernelGGL(k_hermitize, dim3(1024), dim3(256), 0, h->stream,
                     reinterpret_cast<double2*>(L), v, (long)nchol * v * v);
  LRCC_HIP(h, hipGetLastError());

  std::vector<int> widths;
  for (int s : {2, 4, 8})
    if (s == 2 || s <= g.nbv) widths.push_back(s);
  std::vector<int> occs;
  for (int var = 1; var <= 5; ++var)
    if (ppl_has_variant(prec, cmul, var)) occs.push_back(var);

  const int saved_s = h->order_s[prec], saved_occ = h->occ[prec][cmul];
  const bool saved_timing = h->timing;
  int best_s = widths[0], best_occ = 1, ncand = 0;
  double best = 1e300;
  for (int s : widths) {
    for (int occ : occs) {
      h->order_s[prec] = s;
      h->occ[prec][cmul] = occ;
      double ms_best = 1e300;
      for (int rep = 0; rep < 3; ++rep) {
        h->timing = rep > 0;
        h->tev_used = 0;
        lrcc_status st = sigma_packed(h, make_geom(o, v, nchol, nrhs, ppl_chunk(prec, cmul)), L,
                                      false, X, S, LRCC_C128, prec, cmul);
        if (st != LRCC_OK) {
          h->order_s[prec] = saved_s;
          h->occ[prec][cmul] = saved_occ;
          h->timing = saved_timing;
          h->tev_used = 0;
          return st;
        }
        if (rep > 0) {
          LRCC_HIP(h, hipStreamSynchronize(h->stream));
          double ms = 0;
          for (size_t k = 0; k < h->tev_used; ++k) {
            float t = 0;
            LRCC_HIP(h, hipEventElapsedTime(&t, h->tev[2 * k], h->tev[2 * k + 1]));
            ms += t;
          }
          ms_best = std::min(ms_best, ms);
        }
      }
      ++ncand;
      if (ms_best < best) {
        best = ms_best;
        best_s = s;
        best_occ = occ;
      }
    }
  }
  h->timing = saved_timing;
  h->tev_used = 0;  // the tuner reused the timing events: totals restart
  h->order_s[prec] = best_s;
  h->occ[prec][cmul] = best_occ;
  if (out) *out = lrcc_tune_result{best_s, best_occ, best, ncand};
  if (cache_path) {
    std::ofstream app(cache_path, std::ios::app);
    if (app) app << key << " " << best_s << " " << best_occ << " " << best << "\n";
  }
  return LRCC_OK;
}

}  // namespace lrcc
