// Batched LTMP2: many independent cells (uneven sizes, uneven Laplace grids)
// evaluated together.
//
//  * Cells are grouped by FFT grid size n.  Per-cell data (orbitals, overlap
//    densities, quadrature) are prepared as for a single cell; the large
//    per-Laplace-point scratch (chi tiles, chi(r, G'), transformed-state
//    products P, transformed states w) is pooled across cells.
//  * Within a group, the outer G' loop of every cell is cut into the same
//    number of rounds.  For each Laplace point and round, every active cell
//    runs its transformed-state GEMM and synthesis, then ONE persistent fused
//    launch evaluates the Fock-like pair transforms of all cells of the group
//    (descriptor table + prefix sums over the cells' work lists).
//  * A tuner picks, per group, the slab tile of the pair transform and the
//    number of resident workgroups per CU of the persistent launch by timing
//    the candidates once; choices are cached per (grid, precision).
//  * The whole launch sequence is captured into a hipGraph after the first
//    (eager) evaluation and replayed by later calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ltmp2.h"
#include "ctx.h"
#include "dispatch.h"

using namespace ltmp2;

namespace {

// One fused pair launch: the cells of a round that share a kept-set instance.
struct Part {
  std::vector<PairCell> cells;  // host copy (for inspection)
  PairCell* d_cells = nullptr;
  long* d_prefix = nullptr;
  long total = 0;
  int ng_max = 0, kmax_max = 0, kfix = -1;
};
using Round = std::vector<Part>;

int round_kmax(const Round& r) {
  int k = 0;
  for (const Part& p : r) k = std::max(k, p.kmax_max);
  return k;
}

int sched_kmax(const std::vector<std::vector<Round>>& sched) {
  int k = 0;
  for (const auto& rounds : sched)
    for (const Round& r : rounds) k = std::max(k, round_kmax(r));
  return k;
}

struct Group {
  int n = 0;
  std::vector<int> cells;
  int rounds = 1;
  int sx = 1, wg_per_cu = 2;
  int max_ntau = 0;
  std::vector<std::vector<Round>> sched;  // [itau][round]
  double tuned_ms = 0.0;
  bool tuned = false;
};

thread_local std::string g_batch_error;

std::mutex g_tune_mu;
// (n, prec, largest kept set of the group) -> (sx, wg/CU): the slab tile that
// fits shared memory depends on the kept set, so it is part of the key
std::map<std::tuple<int, int, int>, std::pair<int, int>> g_tune_cache;

}  // namespace

struct ltmp2_batch {
  std::vector<ltmp2_ctx*> cells;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int prec = 0;
  std::string err;
  bool failed = false;
  std::vector<void*> owned;
  size_t bytes = 0;
  void *chi = nullptr, *chihat = nullptr, *P = nullptr, *wpool = nullptr;
  std::vector<Group> groups;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  long calls = 0;
  int num_cus = 256;
  // optional event timing of the fused pair launches (eager evaluation only)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> marks;
  double pair_ms = 0.0;
  long pair_n = 0;
};

namespace {

ltmp2_status bfail(ltmp2_batch* b, ltmp2_status s, const std::string& m) {
  if (b) {
    b->err = m;
    if (s == LTMP2_EDEVICE) b->failed = true;
  } else {
    g_batch_error = m;
  }
  return s;
}

ltmp2_status balloc(ltmp2_batch* b, void** p, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 1));
  if (e != hipSuccess)
    return bfail(b, e == hipErrorOutOfMemory ? LTMP2_ENOMEM : LTMP2_EDEVICE,
                 std::string("hipMalloc: ") + hipGetErrorString(e));
  b->owned.push_back(q);
  b->bytes += bytes;
  *p = q;
  return LTMP2_OK;
}

template <class T>
ltmp2_status fused_pair(ltmp2_batch* b, const Group& g, const Part& r, int sx, int wg) {
  if (r.total == 0) return LTMP2_OK;
  const GridOps<T>* ops = grid_ops<T>(g.n);
  long nblk = std::min<long>((r.total + 7) / 8 * 8, long(wg) * b->num_cus);
  nblk = std::max<long>(8, nblk / 8 * 8);
  return ops->pair_multi(r.d_cells, r.d_prefix, int(r.cells.size()), r.ng_max, r.kmax_max,
                         r.kfix, sx, int(nblk), b->stream);
}

ltmp2_status pair_launch(ltmp2_batch* b, const Group& g, const Round& rd, int sx, int wg) {
  for (const Part& r : rd) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->timing && r.total > 0 && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess)
      (void)hipEventRecord(e0, b->stream);
    const ltmp2_status s = b->prec == LTMP2_FP64 ? fused_pair<double>(b, g, r, sx, wg)
                                                 : fused_pair<float>(b, g, r, sx, wg);
    if (e1) {
      (void)hipEventRecord(e1, b->stream);
      b->marks.push_back({e0, e1});
    } else if (e0) {
      (void)hipEventDestroy(e0);
    }
    if (s) return s;
  }
  return LTMP2_OK;
}

void collect_batch_timing(ltmp2_batch* b) {
  if (b->marks.empty()) return;
  (void)hipStreamSynchronize(b->stream);
  for (auto& m : b->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.first, m.second) == hipSuccess) {
      b->pair_ms += ms;
      b->pair_n += 1;
    }
    (void)hipEventDestroy(m.first);
    (void)hipEventDestroy(m.second);
  }
  b->marks.clear();
}

// the whole evaluation of one group (enqueued on the batch stream)
ltmp2_status run_group(ltmp2_batch* b, const Group& g) {
  ltmp2_status s;
  for (int it = 0; it < g.max_ntau; ++it) {
    for (int ci : g.cells) {
      ltmp2_ctx* c = b->cells[ci];
      if (it >= c->ntau) continue;
      if ((s = run_direct(c, it, nullptr))) return bfail(b, s, "cell direct term: " + c->err);
    }
    for (int r = 0; r < g.rounds; ++r) {
      for (int ci : g.cells) {
        ltmp2_ctx* c = b->cells[ci];
        if (it >= c->ntau) continue;
        const int g0 = r * c->gblock;
        if (g0 >= c->nh) continue;
        const int gb = std::min(c->gblock, c->nh - g0);
        if ((s = exchange_block_prepare(c, it, g0, gb)))
          return bfail(b, s, "cell transformed states: " + c->err);
      }
      if ((s = pair_launch(b, g, g.sched[it][r], g.sx, g.wg_per_cu)))
        return bfail(b, s, "fused pair launch failed");
    }
    for (int ci : g.cells) {
      ltmp2_ctx* c = b->cells[ci];
      if (it >= c->ntau) continue;
      if ((s = exchange_reduce(c, it, 0, c->nh))) return bfail(b, s, "cell reduction: " + c->err);
    }
  }
  return LTMP2_OK;
}

ltmp2_status run_all(ltmp2_batch* b) {
  for (const Group& g : b->groups) {
    ltmp2_status s = run_group(b, g);
    if (s) return s;
  }
  return LTMP2_OK;
}

// Time the fused pair launch of (tau 0, round 0) for each candidate tile.
ltmp2_status tune_group(ltmp2_batch* b, Group& g) {
  const int kmax_g = sched_kmax(g.sched);
  const std::tuple<int, int, int> key{g.n, b->prec, kmax_g};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      g.sx = it->second.first;
      g.wg_per_cu = it->second.second;
      g.tuned = true;
      return LTMP2_OK;
    }
  }
  const Round& r0 = g.sched[0][0];
  ltmp2_status s;
  for (int ci : g.cells) {
    ltmp2_ctx* c = b->cells[ci];
    const int gb = std::min(c->gblock, c->nh);
    if ((s = exchange_block_prepare(c, 0, 0, gb))) return bfail(b, s, "tuning prepare: " + c->err);
  }
  // every round of the group must fit the chosen tile
  const int smax = b->prec == LTMP2_FP64 ? grid_ops<double>(g.n)->pair_sx_max(kmax_g)
                                         : grid_ops<float>(g.n)->pair_sx_max(kmax_g);
  std::vector<int> sxs{smax};
  if (smax > 1) sxs.push_back(slab_tile_at_most(g.n, smax - 1));
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) || hipEventCreate(&e1)) return bfail(b, LTMP2_EDEVICE, "event");
  double best = 1e300;
  int bsx = smax, bwg = 2;
  for (int sx : sxs)
    for (int wg : {1, 2, 3, 4}) {
      if ((s = pair_launch(b, g, r0, sx, wg))) break;  // warm-up of this variant
      (void)hipEventRecord(e0, b->stream);
      if ((s = pair_launch(b, g, r0, sx, wg))) break;
      (void)hipEventRecord(e1, b->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        bsx = sx;
        bwg = wg;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s) return bfail(b, s, "tuning launch failed");
  g.sx = bsx;
  g.wg_per_cu = bwg;
  g.tuned_ms = best;
  g.tuned = true;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = {bsx, bwg};
  return LTMP2_OK;
}

}  // namespace

extern "C" ltmp2_status ltmp2_batch_create(int n_cells, const ltmp2_params* params,
                                           const int32_t* const* miller, const double* const* eps,
                                           const double* const* coeff, const double* const* tau,
                                           const double* const* w, const char* mlp_weights,
                                           void* hip_stream, ltmp2_batch** out) {
  if (!out) return bfail(nullptr, LTMP2_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_cells < 1 || !params || !miller || !eps || !coeff)
    return bfail(nullptr, LTMP2_EINVAL, "bad batch arguments");
  const int prec = params[0].prec;
  // coefficients of each cell in real form (the caller's array when already real)
  std::vector<std::vector<double>> creal(n_cells);
  std::vector<const double*> cuse(n_cells);
  for (int k = 0; k < n_cells; ++k) {
    if (params[k].prec != prec) return bfail(nullptr, LTMP2_EINVAL, "cells differ in precision");
    if (params[k].n_extrap)
      return bfail(nullptr, LTMP2_EINVAL,
                   "cell " + std::to_string(k) +
                       ": the cutoff extrapolation runs per context (ltmp2_setup), not batched");
    ltmp2_status s = validate_inputs(&params[k], miller[k], eps[k], coeff[k],
                                     tau ? tau[k] : nullptr, w ? w[k] : nullptr, creal[k],
                                     &cuse[k]);
    if (s) return bfail(nullptr, s, "cell " + std::to_string(k) + ": " + setup_error());
  }
  ltmp2_batch* b = new ltmp2_batch();
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (!b->stream) {  // graph capture needs a stream of its own (default priority)
    if (hipStreamCreate(&b->stream) != hipSuccess) {
      delete b;
      return bfail(nullptr, LTMP2_EDEVICE, "stream creation failed");
    }
    b->own_stream = true;
  }
  b->prec = prec;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      b->num_cus = prop.multiProcessorCount;
  }
  // per-cell preparation without private scratch
  for (int k = 0; k < n_cells; ++k) {
    ltmp2_ctx* c = new ltmp2_ctx();
    c->prm = params[k];
    c->stream = b->stream;
    c->own_scratch = false;
    if (mlp_weights) c->mlp_path = mlp_weights;
    b->cells.push_back(c);
    ltmp2_status s = setup_cell(c, miller[k], eps[k], cuse[k], tau ? tau[k] : nullptr,
                                w ? w[k] : nullptr);
    std::vector<double>().swap(creal[k]);
    if (s) {
      const std::string m = "cell " + std::to_string(k) + ": " + setup_error();
      ltmp2_batch_destroy(b);
      return bfail(nullptr, s, m);
    }
  }
  // groups by grid size; rounds so one group's transformed states fit the budget
  std::map<int, std::vector<int>> byn;
  for (int k = 0; k < n_cells; ++k) byn[b->cells[k]->n].push_back(k);
  const size_t budget = size_t(16) << 30;  // transformed states of one group
  size_t es = b->cells[0]->esz, chi_b = 0, chihat_b = 0, P_b = 0, w_b = 0;
  for (auto& kv : byn) {
    Group g;
    g.n = kv.first;
    g.cells = kv.second;
    for (;;) {
      size_t need = 0;
      for (int ci : g.cells) {
        ltmp2_ctx* c = b->cells[ci];
        const int gb = (c->nh + g.rounds - 1) / g.rounds;
        need += 2 * es * size_t(gb) * c->no * c->nrp;
      }
      if (need <= budget || g.rounds >= 64) {
        w_b = std::max(w_b, need);
        break;
      }
      ++g.rounds;
    }
    for (int ci : g.cells) {
      ltmp2_ctx* c = b->cells[ci];
      c->gblock = (c->nh + g.rounds - 1) / g.rounds;
      g.max_ntau = std::max(g.max_ntau, c->ntau);
      chi_b = std::max(chi_b, es * size_t(c->nrp) * c->nrp);
      chihat_b = std::max(chihat_b, 2 * es * size_t(c->nh) * c->nrp);
      P_b = std::max(P_b, 2 * es * size_t(c->gblock) * c->no * c->npw);
    }
    b->groups.push_back(g);
  }
  ltmp2_status s;
  if ((s = balloc(b, &b->chi, chi_b)) || (s = balloc(b, &b->chihat, chihat_b)) ||
      (s = balloc(b, &b->P, P_b)) || (s = balloc(b, &b->wpool, w_b))) {
    const std::string m = b->err;
    ltmp2_batch_destroy(b);
    return bfail(nullptr, s, m);
  }
  // scratch pointers and the fused-launch schedules
  for (Group& g : b->groups) {
    size_t off = 0;
    for (int ci : g.cells) {
      ltmp2_ctx* c = b->cells[ci];
      c->d_chi = b->chi;
      c->d_chihat = b->chihat;
      c->d_P = b->P;
      c->d_w = static_cast<char*>(b->wpool) + off;
      off += 2 * es * size_t(c->gblock) * c->no * c->nrp;
    }
    g.sched.assign(g.max_ntau, std::vector<Round>(g.rounds));
    int (*kept)(int) = b->prec == LTMP2_FP64 ? grid_ops<double>(g.n)->pair_kept
                                             : grid_ops<float>(g.n)->pair_kept;
    for (int it = 0; it < g.max_ntau; ++it)
      for (int r = 0; r < g.rounds; ++r) {
        // one part per kept-set instance among the round's active cells
        std::map<int, std::vector<int>> by_kept;
        for (int ci : g.cells) {
          ltmp2_ctx* c = b->cells[ci];
          if (it >= c->ntau || r * c->gblock >= c->nh) continue;
          by_kept[kept(c->kmax_aux)].push_back(ci);
        }
        for (auto& kv : by_kept) {
          Part rd;
          rd.kfix = kv.first;
          std::vector<long> prefix{0};
          for (int ci : kv.second) {
            ltmp2_ctx* c = b->cells[ci];
            const int g0 = r * c->gblock;
            const int gb = std::min(c->gblock, c->nh - g0);
            rd.cells.push_back(PairCell{c->d_psi, c->d_w, c->d_pairs, c->d_gdesc, c->d_v,
                                        c->d_xpart + size_t(g0) * c->npairs, c->nrp, c->no,
                                        c->npairs, gb, c->ng, c->kmax_aux, c->dV * c->dV});
            prefix.push_back(prefix.back() + long(c->npairs) * gb);
            rd.ng_max = std::max(rd.ng_max, c->ng);
            rd.kmax_max = std::max(rd.kmax_max, c->kmax_aux);
          }
          rd.total = prefix.back();
          void *pc = nullptr, *pp = nullptr;
          if ((s = balloc(b, &pc, sizeof(PairCell) * rd.cells.size())) ||
              (s = balloc(b, &pp, sizeof(long) * prefix.size()))) {
            ltmp2_batch_destroy(b);
            return bfail(nullptr, s, "schedule allocation failed");
          }
          rd.d_cells = static_cast<PairCell*>(pc);
          rd.d_prefix = static_cast<long*>(pp);
          if (hipMemcpy(pc, rd.cells.data(), sizeof(PairCell) * rd.cells.size(),
                        hipMemcpyHostToDevice) ||
              hipMemcpy(pp, prefix.data(), sizeof(long) * prefix.size(), hipMemcpyHostToDevice)) {
            ltmp2_batch_destroy(b);
            return bfail(nullptr, LTMP2_EDEVICE, "schedule upload failed");
          }
          g.sched[it][r].push_back(std::move(rd));
        }
      }
    // largest slab tile allowed by shared memory for this group
    const int km = sched_kmax(g.sched);
    g.sx = b->prec == LTMP2_FP64 ? grid_ops<double>(g.n)->pair_sx_max(km)
                                 : grid_ops<float>(g.n)->pair_sx_max(km);
  }
  *out = b;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_batch_energy(ltmp2_batch* b, double* e_direct,
                                           double* e_exchange) {
  if (!b) return bfail(nullptr, LTMP2_EINVAL, "batch is NULL");
  if (b->failed) return bfail(b, LTMP2_ESTATE, "batch failed earlier: " + b->err);
  ltmp2_status s;
  if (b->calls == 0 || b->timing) {
    for (Group& g : b->groups)
      if (!g.tuned && (s = tune_group(b, g))) return s;
    if ((s = run_all(b))) return s;  // eager evaluation (first call, or timed)
  } else {
    if (!b->exec) {
      if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed))
        return bfail(b, LTMP2_EDEVICE, "graph capture could not start");
      s = run_all(b);
      hipGraph_t gr = nullptr;
      const hipError_t e = hipStreamEndCapture(b->stream, &gr);
      if (s) return s;
      if (e != hipSuccess || !gr) return bfail(b, LTMP2_EDEVICE, "graph capture failed");
      b->graph = gr;
      if (hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0) != hipSuccess)
        return bfail(b, LTMP2_EDEVICE, "graph instantiation failed");
    }
    if (hipGraphLaunch(b->exec, b->stream) != hipSuccess)
      return bfail(b, LTMP2_EDEVICE, "graph launch failed");
  }
  ++b->calls;
  std::vector<std::vector<double>> pt(b->cells.size());
  for (size_t k = 0; k < b->cells.size(); ++k) {
    ltmp2_ctx* c = b->cells[k];
    pt[k].resize(2 * size_t(c->ntau));
    if (hipMemcpyAsync(pt[k].data(), c->d_scal, sizeof(double) * pt[k].size(),
                       hipMemcpyDeviceToHost, b->stream))
      return bfail(b, LTMP2_EDEVICE, "result copy failed");
  }
  if (hipStreamSynchronize(b->stream)) return bfail(b, LTMP2_EDEVICE, "batch evaluation failed");
  for (size_t k = 0; k < b->cells.size(); ++k) {
    ltmp2_ctx* c = b->cells[k];
    double ed = 0.0, ex = 0.0;
    for (int t = 0; t < c->ntau; ++t) {
      ed += c->w[t] * pt[k][2 * t];
      ex += c->w[t] * pt[k][2 * t + 1];
    }
    if (!std::isfinite(ed) || !std::isfinite(ex)) return bfail(b, LTMP2_ENUMERIC, "non-finite");
    if (e_direct) e_direct[k] = ed;
    if (e_exchange) e_exchange[k] = ex;
  }
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_batch_set_timing(ltmp2_batch* b, int on) {
  if (!b) return LTMP2_EINVAL;
  collect_batch_timing(b);
  b->timing = on != 0;
  b->pair_ms = 0.0;
  b->pair_n = 0;
  for (ltmp2_ctx* c : b->cells) (void)ltmp2_set_timing(c, on);
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_batch_get_timing(ltmp2_batch* b, int stage, double* ms,
                                               long* launches) {
  if (!b || stage < 0 || stage > 6) return LTMP2_EINVAL;
  collect_batch_timing(b);
  double t = 0.0;
  long n = 0;
  if (stage == 5) {
    t = b->pair_ms;
    n = b->pair_n;
  } else {
    for (ltmp2_ctx* c : b->cells) {
      double tc = 0.0;
      long nc = 0;
      (void)ltmp2_get_timing(c, stage, &tc, &nc);
      t += tc;
      n += nc;
    }
  }
  if (ms) *ms = t;
  if (launches) *launches = n;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_batch_info(const ltmp2_batch* b, ltmp2_batch_stats* st) {
  if (!b || !st) return LTMP2_EINVAL;
  st->n_cells = int(b->cells.size());
  st->n_groups = int(b->groups.size());
  st->graph_ready = b->exec != nullptr;
  st->device_bytes = b->bytes;
  for (ltmp2_ctx* c : b->cells) st->device_bytes += c->bytes;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_batch_group(const ltmp2_batch* b, int g, int* n_fft, int* n_cells,
                                          int* rounds, int* slab_tile, int* wg_per_cu,
                                          double* tuned_ms) {
  if (!b || g < 0 || g >= int(b->groups.size())) return LTMP2_EINVAL;
  const Group& G = b->groups[g];
  if (n_fft) *n_fft = G.n;
  if (n_cells) *n_cells = int(G.cells.size());
  if (rounds) *rounds = G.rounds;
  if (slab_tile) *slab_tile = G.sx;
  if (wg_per_cu) *wg_per_cu = G.wg_per_cu;
  if (tuned_ms) *tuned_ms = G.tuned_ms;
  return LTMP2_OK;
}

extern "C" ltmp2_status ltmp2_batch_cell(const ltmp2_batch* b, int k, ltmp2_info* info) {
  if (!b || k < 0 || k >= int(b->cells.size())) return LTMP2_EINVAL;
  return ltmp2_get_info(b->cells[k], info);
}

extern "C" void ltmp2_batch_destroy(ltmp2_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  collect_batch_timing(b);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (ltmp2_ctx* c : b->cells) ltmp2_destroy(c);
  for (void* p : b->owned) (void)hipFree(p);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

extern "C" const char* ltmp2_batch_last_error(const ltmp2_batch* b) {
  return b ? b->err.c_str() : g_batch_error.c_str();
}
