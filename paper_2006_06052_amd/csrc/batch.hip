// Several independent systems of uneven size behind one solver
// (mgk_batch_setup / mgk_batch_solve).
//
// Each system keeps its own hierarchy (set up exactly as a single system), and
// the BiCGStab recurrences of all systems run in lockstep.  Every stage of an
// iteration is one persistent launch over a work list covering all systems
// that take part in it:
//   outer SpMV, dots and vector updates: one launch each over all systems;
//   V-cycle: level l's pre-smoothing, residual and restriction for every system
//   deeper than l (l = 0, 1, ...), then the coarsest solves of all systems in
//   one launch, then level l's prolongation and post-smoothing for l
//   descending.  Systems only depend on themselves, so this order gives each
//   system exactly its own V-cycle.
// The engine tile of each grouped stage is picked by timing the grouped launch
// at setup.  A system whose iteration has stopped is skipped by every launch.
#include <type_traits>

#include "internal.hpp"
#include "kernels_batch.hpp"

namespace mgk {

// Launch shapes of a grouped launch: a persistent grid of PERSIST workgroups
// striding through the tiles, or one workgroup per tile (ONE_PER_TILE).
constexpr int PERSIST = 2048, ONE_PER_TILE = 1 << 30;

struct GStage {
  std::vector<GItem> h;
  GItem* d = nullptr;
  int total = 0;
  Tile tile;
  int cap = PERSIST;               // workgroups per launch (tuned for row stages)
  bool cached = false;             // operator loads cached (the operators' own policy)
  bool dia = false;                // every item's operator read in its diagonal layout
};

struct BatchWork {
  std::vector<mgk_solver*> sys;
  Device dev;                      // descriptors, scalars, partials
  int nsys = 0, maxlev = 0, b = 4, storage = MGK_F64;
  // level stages; index [l][v] with v the V-cycle input (0: p -> ph, 1: s -> sh)
  std::vector<GStage> bd[2], res[2], sm[2];
  std::vector<GStage> R, P;
  GStage coarse;
  GStage outer_spmv[2];            // 0: v = A ph, 1: t = A sh
  GStage outer_res;                // r = b - A x (in/f/out set per solve)
  GVec* dvec = nullptr;            // device GVec sets (GV_SETS x nsys)
  std::vector<GVec> hvec;
  int vtotal = 0;
  double* scb = nullptr;
  int* active = nullptr;
  double* part = nullptr;
  int* hact = nullptr;             // pinned ring of active flags
  int act_slot = 0;
  double* hscb = nullptr;          // pinned mirror of scb
  hipEvent_t ev = nullptr;
  ~BatchWork() {
    for (mgk_solver* s : sys) mgk_destroy(s);
    if (hact) (void)hipHostFree(hact);
    if (hscb) (void)hipHostFree(hscb);
    if (ev) (void)hipEventDestroy(ev);
  }
};

constexpr int ACT_SLOTS = 64;
enum VecSet { VS_B = 0, VS_RINIT, VS_COPY_RH, VS_ZERO_P, VS_ZERO_V, VS_P, VS_RV, VS_S, VS_TS,
              VS_XR, VS_TRUE, VS_ZERO_X, GV_SETS };

void batch_free(BatchWork* w) { delete w; }

template <int B, int S>
static int rows_tiles(int nbr) {
  return std::max(1, (nbr + RowMap<B, S>::ROWS - 1) / RowMap<B, S>::ROWS);
}

static int tiles_for(int B, const Tile& t, int nbr) {
  int T = 1;
  auto f = [&](auto BB) {
    constexpr int Bc = decltype(BB)::value;
    tile_switch<Bc>(t, [&](auto SS, auto UU) {
      (void)UU;
      T = rows_tiles<Bc, decltype(SS)::value>(nbr);
    });
  };
  if (B == 1) f(std::integral_constant<int, 1>());
  else if (B == 3) f(std::integral_constant<int, 3>());
  else f(std::integral_constant<int, 4>());
  return T;
}

// Assign tile starts for a row stage with tile t and upload its items.
static void finish_rows(BatchWork& W, GStage& g, int B, const Tile& t, int cap) {
  g.tile = t;
  g.cap = cap;
  int acc = 0;
  for (GItem& it : g.h) {
    it.tile0 = acc;
    acc += tiles_for(B, t, it.nbr);
  }
  g.total = acc;
  if (!g.d) g.d = (GItem*)W.dev.alloc(sizeof(GItem) * std::max<size_t>(1, g.h.size()));
  if (!g.h.empty())
    HIPCK(hipMemcpyAsync(g.d, g.h.data(), sizeof(GItem) * g.h.size(), hipMemcpyHostToDevice,
                         W.dev.stream));
  HIPCK(hipStreamSynchronize(W.dev.stream));
}

static void finish_fixed(BatchWork& W, GStage& g, int per_tile_rows) {
  int acc = 0;
  for (GItem& it : g.h) {
    it.tile0 = acc;
    acc += std::max(1, (it.nbr + per_tile_rows - 1) / per_tile_rows);
  }
  g.total = acc;
  if (!g.d) g.d = (GItem*)W.dev.alloc(sizeof(GItem) * std::max<size_t>(1, g.h.size()));
  if (!g.h.empty())
    HIPCK(hipMemcpyAsync(g.d, g.h.data(), sizeof(GItem) * g.h.size(), hipMemcpyHostToDevice,
                         W.dev.stream));
  HIPCK(hipStreamSynchronize(W.dev.stream));
}

static int pgrid(int total, int cap = PERSIST) { return std::max(1, std::min(total, cap)); }

// ---------------------------------------------------------------- grouped launches

// The (cached, diagonal-layout) variant of a grouped kernel as compile-time flags; the
// diagonal layout exists for 3x3 and 4x4 blocks only.
template <int B, class F>
static void g_variant(const GStage& g, F&& f) {
  using T = std::true_type;
  using N = std::false_type;
  if (B != 1 && g.dia) {
    if (g.cached) f(T(), T());
    else f(N(), T());
  } else {
    if (g.cached) f(T(), N());
    else f(N(), N());
  }
}

template <int B, class TV, class TX, class TY>
static void g_spmv(hipStream_t st, const GStage& g, const int* active, double beta) {
  if (g.h.empty()) return;
  using TA = AccOf<TV>;
  tile_switch<B>(g.tile, [&](auto SS, auto UU) {
    g_variant<B>(g, [&](auto C, auto D) {
      k_g_spmv<B, B, decltype(SS)::value, decltype(UU)::value, TV, TX, TY, TA,
               decltype(C)::value, B != 1 && decltype(D)::value>
          <<<pgrid(g.total, g.cap), WG, 0, st>>>(g.d, (int)g.h.size(), g.total, active, (TA)beta);
    });
  });
}

template <int B, class TV, class TX, class TF>
static void g_residual(hipStream_t st, const GStage& g, const int* active) {
  if (g.h.empty()) return;
  using TA = AccOf<TV>;
  tile_switch<B>(g.tile, [&](auto SS, auto UU) {
    g_variant<B>(g, [&](auto C, auto D) {
      k_g_residual<B, decltype(SS)::value, decltype(UU)::value, TV, TX, TF, TA,
                   decltype(C)::value, B != 1 && decltype(D)::value>
          <<<pgrid(g.total, g.cap), WG, 0, st>>>(g.d, (int)g.h.size(), g.total, active);
    });
  });
}

template <int B, class TV, class TX, class TF, class TO, class TM>
static void g_smooth(hipStream_t st, const GStage& g, const int* active) {
  if (g.h.empty()) return;
  using TA = AccOf<TV>;
  tile_switch<B>(g.tile, [&](auto SS, auto UU) {
    g_variant<B>(g, [&](auto C, auto D) {
      k_g_smooth<B, decltype(SS)::value, decltype(UU)::value, TV, TX, TF, TO, TM, TA,
                 decltype(C)::value, B != 1 && decltype(D)::value>
          <<<pgrid(g.total, g.cap), WG, 0, st>>>(g.d, (int)g.h.size(), g.total, active);
    });
  });
}

// Tune a row stage: time the grouped SpMV of its items for every candidate tile.
template <int B, class TV, class TX>
static void tune_stage(BatchWork& W, GStage& g, int* active) {
  std::vector<Tile> cands;
#define MGK_BCAND(SS, UU) cands.push_back(Tile{SS, UU, 1});
  if (B == 1) {
    MGK_TILES_1(MGK_BCAND)
  } else {
    MGK_TILES_B(MGK_BCAND)
  }
#undef MGK_BCAND
  if (g.h.empty()) return;
  // scratch outputs: the stage's own outputs are overwritten during setup only
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  Tile best = cands[0];
  int best_cap = PERSIST;
  float best_ms = 1e30f;
  for (const Tile& t : cands)
    for (int cap : {PERSIST, ONE_PER_TILE}) {
      finish_rows(W, g, B, t, cap);
      g_spmv<B, TV, TX, TX>(W.dev.stream, g, active, 0.0);
      HIPCK(hipEventRecord(e0, W.dev.stream));
      for (int r = 0; r < 3; ++r) g_spmv<B, TV, TX, TX>(W.dev.stream, g, active, 0.0);
      HIPCK(hipEventRecord(e1, W.dev.stream));
      HIPCK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
        best_cap = cap;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  finish_rows(W, g, B, best, best_cap);
}

// ---------------------------------------------------------------- grouped V-cycle

template <int B, class TV, class TX>
struct GCycle {
  using TM = typename SmootherOf<TV>::type;
  using TA = AccOf<TV>;
  static void run(BatchWork& W, int v) {
    hipStream_t st = W.dev.stream;
    const int* act = W.active;
    const int L = W.maxlev;
    for (int l = 0; l + 1 < L; ++l) {
      if (W.res[l == 0 ? v : 0][l].h.empty()) continue;
      if (l == 0) {
        const GStage& bd = W.bd[v][0];
        if (!bd.h.empty())
          k_g_block_diag<B, TM, double, TX, TA><<<pgrid(bd.total), WG, 0, st>>>(
              bd.d, (int)bd.h.size(), bd.total, act);
        g_residual<B, TV, TX, double>(st, W.res[v][0], act);
      } else {
        const GStage& bd = W.bd[0][l];
        if (!bd.h.empty())
          k_g_block_diag<B, TM, TX, TX, TA><<<pgrid(bd.total), WG, 0, st>>>(
              bd.d, (int)bd.h.size(), bd.total, act);
        g_residual<B, TV, TX, TX>(st, W.res[0][l], act);
      }
      g_spmv<B, TV, TX, TX>(st, W.R[l], act, 0.0);
    }
    const GStage& c = W.coarse;
    k_g_coarse<TX, TX><<<pgrid(c.total), WG, 0, st>>>(c.d, (int)c.h.size(), c.total, act);
    for (int l = L - 2; l >= 0; --l) {
      g_spmv<B, TV, TX, TX>(st, W.P[l], act, 1.0);
      if (l == 0) g_smooth<B, TV, TX, double, double, TM>(st, W.sm[v][0], act);
      else g_smooth<B, TV, TX, TX, TX, TM>(st, W.sm[0][l], act);
    }
  }
};

static void gvcycle(BatchWork& W, int v) {
#define MGK_GV(BB)                                                                   \
  case BB:                                                                           \
    if (W.storage == MGK_F64) GCycle<BB, double, double>::run(W, v);                 \
    else if (W.storage == MGK_F32) GCycle<BB, float, float>::run(W, v);              \
    else GCycle<BB, bf16, float>::run(W, v);                                         \
    break;
  switch (W.b) {
    MGK_GV(1)
    MGK_GV(3)
    MGK_GV(4)
  }
#undef MGK_GV
}

static void gouter(BatchWork& W, const GStage& g) {
  hipStream_t st = W.dev.stream;
  switch (W.b) {
    case 1: g_spmv<1, double, double, double>(st, g, W.active, 0.0); break;
    case 3: g_spmv<3, double, double, double>(st, g, W.active, 0.0); break;
    case 4: g_spmv<4, double, double, double>(st, g, W.active, 0.0); break;
  }
}

static void gouter_res(BatchWork& W) {
  hipStream_t st = W.dev.stream;
  switch (W.b) {
    case 1: g_residual<1, double, double, double>(st, W.outer_res, W.active); break;
    case 3: g_residual<3, double, double, double>(st, W.outer_res, W.active); break;
    case 4: g_residual<4, double, double, double>(st, W.outer_res, W.active); break;
  }
}

// ---------------------------------------------------------------- setup

static void build_stages(BatchWork& W) {
  const int L = W.maxlev;
  for (int v = 0; v < 2; ++v) {
    W.bd[v].assign(L, GStage());
    W.res[v].assign(L, GStage());
    W.sm[v].assign(L, GStage());
  }
  W.R.assign(L, GStage());
  W.P.assign(L, GStage());
  W.coarse = GStage();
  // the fine operators (outer, hierarchy level 0) are read in their diagonal layout when
  // every system has one; a stage is one kernel instantiation, so it is all or none
  bool dia_outer = W.b != 1, dia_l0 = W.b != 1;
  for (mgk_solver* S : W.sys) {
    dia_outer = dia_outer && S->A.dia.k > 0;
    dia_l0 = dia_l0 && S->H.lv[0].A.dia.k > 0;
  }
  auto op = [](GItem it, const DMat& A, bool dia) {
    if (dia) {
      it.val = A.dval;
      it.dia = A.dia;
    }
    return it;
  };
  for (int s = 0; s < W.nsys; ++s) {
    mgk_solver* S = W.sys[s];
    DHier& H = S->H;
    const int nl = (int)H.lv.size();
    for (int l = 0; l + 1 < nl; ++l) {
      DLevel& Lv = H.lv[l];
      DLevel& C = H.lv[l + 1];
      for (int v = 0; v < (l == 0 ? 2 : 1); ++v) {
        const void* rin = l == 0 ? (v == 0 ? (const void*)S->p : (const void*)S->s) : Lv.r;
        void* zout = l == 0 ? (v == 0 ? (void*)S->ph : (void*)S->sh) : Lv.z2;
        W.bd[v][l].h.push_back(GItem{nullptr, nullptr, nullptr, Lv.M, rin, nullptr, Lv.z,
                                     Lv.nbr, 0, s, 0});
        const bool dl = l == 0 && dia_l0;
        W.res[v][l].h.push_back(op(GItem{Lv.A.ptr, Lv.A.col, Lv.A.val, nullptr, Lv.z, rin,
                                         Lv.t, Lv.nbr, 0, s, 0}, Lv.A, dl));
        W.sm[v][l].h.push_back(op(GItem{Lv.A.ptr, Lv.A.col, Lv.A.val, Lv.M, Lv.z, rin, zout,
                                        Lv.nbr, 0, s, 0}, Lv.A, dl));
        W.res[v][l].cached = W.sm[v][l].cached = Lv.A.cached;
        W.res[v][l].dia = W.sm[v][l].dia = dl;
      }
      W.R[l].h.push_back(GItem{Lv.R.ptr, Lv.R.col, Lv.R.val, nullptr, Lv.t, nullptr, C.r,
                               Lv.R.nbr, 0, s, 0});
      const void* zc = l + 1 == nl - 1 ? C.z : C.z2;
      W.P[l].h.push_back(GItem{Lv.P.ptr, Lv.P.col, Lv.P.val, nullptr, zc, nullptr, Lv.z,
                               Lv.P.nbr, 0, s, 0});
      W.R[l].cached = Lv.R.cached;
      W.P[l].cached = Lv.P.cached;
    }
    DLevel& Cl = H.lv[nl - 1];
    W.coarse.h.push_back(GItem{nullptr, nullptr, nullptr, H.cinv, Cl.r, nullptr, Cl.z, H.nc, 0,
                               s, 0});
    W.outer_spmv[0].h.push_back(op(GItem{S->A.ptr, S->A.col, S->A.val, nullptr, S->ph,
                                         nullptr, S->v, S->nbr, 0, s, 0}, S->A, dia_outer));
    W.outer_spmv[1].h.push_back(op(GItem{S->A.ptr, S->A.col, S->A.val, nullptr, S->sh,
                                         nullptr, S->t, S->nbr, 0, s, 0}, S->A, dia_outer));
    W.outer_res.h.push_back(op(GItem{S->A.ptr, S->A.col, S->A.val, nullptr, nullptr, nullptr,
                                     S->r, S->nbr, 0, s, 0}, S->A, dia_outer));
    W.outer_spmv[0].cached = W.outer_spmv[1].cached = W.outer_res.cached = S->A.cached;
    W.outer_spmv[0].dia = W.outer_spmv[1].dia = W.outer_res.dia = dia_outer;
  }
  finish_fixed(W, W.coarse, 1);
  for (int l = 0; l < L; ++l)
    for (int v = 0; v < 2; ++v) finish_fixed(W, W.bd[v][l], WG / W.b);
}

template <int B, class TV, class TX>
static void tune_all(BatchWork& W) {
  for (int l = 0; l < W.maxlev; ++l) {
    // residual and smoother share the tile of A_l
    tune_stage<B, TV, TX>(W, W.res[0][l], W.active);
    for (int v = 0; v < 2; ++v) {
      if (v == 1 && l > 0) continue;
      finish_rows(W, W.res[v][l], B, W.res[0][l].tile, W.res[0][l].cap);
      finish_rows(W, W.sm[v][l], B, W.res[0][l].tile, W.res[0][l].cap);
    }
    tune_stage<B, TV, TX>(W, W.R[l], W.active);
    tune_stage<B, TV, TX>(W, W.P[l], W.active);
  }
  for (int v = 0; v < 2; ++v) tune_stage<B, double, double>(W, W.outer_spmv[v], W.active);
  finish_rows(W, W.outer_res, B, W.outer_spmv[0].tile, W.outer_spmv[0].cap);
}

static void batch_setup_impl(mgk_solver* S, int nsys, const mgk_bsr* const* A, int block_size,
                             int kind, const mgk_params* prm, void* stream) {
  if (nsys < 1 || nsys > 256 || !A || !prm)
    throw Error(MGK_E_INVALID, "batch: need 1..256 systems and non-null arguments");
  if (kind == MGK_SCHUR || kind == MGK_ILU || prm->ilu_smoother)
    throw Error(MGK_E_INVALID, "batch: monolithic AMG kinds with block-diagonal smoothers only");
  if (prm->krylov != MGK_BICGSTAB) throw Error(MGK_E_INVALID, "batch: BiCGStab only");
  BatchWork* W = new BatchWork();
  S->batch = W;
  W->dev.stream = (hipStream_t)stream;
  W->nsys = nsys;
  W->b = block_size;
  W->storage = prm->hier;
  S->prm = *prm;
  S->kind = kind;
  S->b = block_size;
  S->dev.stream = (hipStream_t)stream;
  // every fine operator with at most 8 block diagonals gets a diagonal-layout copy (its
  // row masks skip the padding, so small systems lose nothing to it); layout 1 keeps BSR
  mgk_params sub_prm = *prm;
  sub_prm.layout = prm->layout == 1 ? 1 : 2;
  for (int s = 0; s < nsys; ++s) {
    mgk_solver* sub = nullptr;
    const int rc = mgk_setup(A[s], block_size, (mgk_precond_kind)kind, &sub_prm, stream, &sub);
    if (rc) throw Error(rc, "batch: system " + std::to_string(s) + ": " + g_err);
    W->sys.push_back(sub);
    if (sub->H.lv.size() < 2)
      throw Error(MGK_E_INVALID, "batch: system " + std::to_string(s) +
                                     " has a single level (it is below coarse_enough)");
    W->maxlev = std::max(W->maxlev, (int)sub->H.lv.size());
    S->n += sub->n;
    S->nbr += sub->nbr;
  }
  W->scb = (double*)W->dev.alloc(sizeof(double) * SC_COUNT * nsys);
  W->active = (int*)W->dev.alloc(sizeof(int) * nsys);
  HIPCK(hipHostMalloc((void**)&W->hact, sizeof(int) * nsys * ACT_SLOTS, hipHostMallocDefault));
  HIPCK(hipHostMalloc((void**)&W->hscb, sizeof(double) * SC_COUNT * nsys, hipHostMallocDefault));
  HIPCK(hipEventCreateWithFlags(&W->ev, hipEventDisableTiming));
  std::vector<int> ones(nsys, 1);
  HIPCK(hipMemcpy(W->active, ones.data(), sizeof(int) * nsys, hipMemcpyHostToDevice));
  build_stages(*W);
  switch (block_size) {
#define MGK_TB(BB)                                                                     \
  case BB:                                                                             \
    if (W->storage == MGK_F64) tune_all<BB, double, double>(*W);                       \
    else if (W->storage == MGK_F32) tune_all<BB, float, float>(*W);                    \
    else tune_all<BB, bf16, float>(*W);                                                \
    break;
    MGK_TB(1)
    MGK_TB(3)
    MGK_TB(4)
#undef MGK_TB
  }
  // vector tiles
  W->hvec.assign((size_t)GV_SETS * nsys, GVec());
  int acc = 0;
  for (int s = 0; s < nsys; ++s) {
    const int nt = (int)((W->sys[s]->n + VTILE - 1) / VTILE);
    for (int q = 0; q < GV_SETS; ++q) {
      GVec& g = W->hvec[(size_t)q * nsys + s];
      g.n = (long long)W->sys[s]->n;
      g.tile0 = acc;
      g.ntiles = nt;
      g.sys = s;
    }
    acc += nt;
  }
  W->vtotal = acc;
  W->dvec = (GVec*)W->dev.alloc(sizeof(GVec) * W->hvec.size());
  W->part = (double*)W->dev.alloc(sizeof(double) * 2 * (size_t)acc + 64);
  HIPCK(hipStreamSynchronize(W->dev.stream));
}

// ---------------------------------------------------------------- lockstep BiCGStab

static void push_active(BatchWork& W, const std::vector<int>& act) {
  int* slot = W.hact + (size_t)W.act_slot * W.nsys;
  W.act_slot = (W.act_slot + 1) % ACT_SLOTS;
  std::memcpy(slot, act.data(), sizeof(int) * W.nsys);
  HIPCK(hipMemcpyAsync(W.active, slot, sizeof(int) * W.nsys, hipMemcpyHostToDevice,
                       W.dev.stream));
}

static void gvec(BatchWork& W, int set, int op, bool dots) {
  k_g_vec<<<pgrid(W.vtotal), WG, 0, W.dev.stream>>>(W.dvec + (size_t)set * W.nsys, W.nsys,
                                                    W.vtotal, op, W.active, W.scb,
                                                    dots ? W.part : nullptr);
}

static void gfin(BatchWork& W, int set, int op, int i0 = 0, int i1 = 0) {
  k_g_finalize<<<W.nsys, WG, 0, W.dev.stream>>>(W.dvec + (size_t)set * W.nsys, W.nsys,
                                                W.vtotal, W.part, op, i0, i1, W.active, W.scb);
}

static void gpublish(BatchWork& W) {
  HIPCK(hipMemcpyAsync(W.hscb, W.scb, sizeof(double) * SC_COUNT * W.nsys,
                       hipMemcpyDeviceToHost, W.dev.stream));
  HIPCK(hipEventRecord(W.ev, W.dev.stream));
  HIPCK(hipEventSynchronize(W.ev));
  HIPCK(hipGetLastError());
}

static int batch_bicgstab(mgk_solver* S, const double* const* b, double* const* x, double tol,
                          mgk_info* infos) {
  BatchWork& W = *S->batch;
  const int ns = W.nsys;
  // vector sets for this solve (b and x are the caller's)
  for (int s = 0; s < ns; ++s) {
    mgk_solver* T = W.sys[s];
    auto set = [&](int q, std::initializer_list<double*> ptrs) {
      GVec& g = W.hvec[(size_t)q * ns + s];
      int i = 0;
      for (double* p : ptrs) g.a[i++] = p;
      for (; i < 7; ++i) g.a[i] = nullptr;
    };
    double* bs = const_cast<double*>(b[s]);
    set(VS_B, {bs, bs});
    set(VS_RINIT, {T->r, T->r, T->rh, T->r});
    set(VS_COPY_RH, {T->r, T->rh});
    set(VS_ZERO_P, {T->p});
    set(VS_ZERO_V, {T->v});
    set(VS_P, {T->r, T->v, T->p});
    set(VS_RV, {T->rh, T->v});
    set(VS_S, {T->r, T->v, T->ph, T->s, x[s]});
    set(VS_TS, {T->t, T->s, T->t, T->t});
    set(VS_XR, {T->s, T->t, T->sh, T->rh, x[s], T->r, T->ph});
    set(VS_TRUE, {T->r, T->r});
    set(VS_ZERO_X, {x[s]});
    W.outer_res.h[s].in = x[s];
    W.outer_res.h[s].f = b[s];
  }
  HIPCK(hipMemcpyAsync(W.dvec, W.hvec.data(), sizeof(GVec) * W.hvec.size(),
                       hipMemcpyHostToDevice, W.dev.stream));
  HIPCK(hipMemcpyAsync(W.outer_res.d, W.outer_res.h.data(), sizeof(GItem) * ns,
                       hipMemcpyHostToDevice, W.dev.stream));
  std::vector<int> act(ns, 1), done(ns, 0), iters(ns, 0), restarts(ns, 0);
  push_active(W, act);
  gvec(W, VS_B, GV_DOT, true);
  gfin(W, VS_B, GF_STORE1, SC_TMP);
  gpublish(W);
  auto sc = [&](int s, int idx) { return W.hscb[(size_t)s * SC_COUNT + idx]; };
  std::vector<double> nb(ns), tol2(ns);
  for (int s = 0; s < ns; ++s) {
    nb[s] = std::sqrt(sc(s, SC_TMP));
    tol2[s] = (tol * nb[s]) * (tol * nb[s]);
    act[s] = nb[s] == 0.0;
  }
  push_active(W, act);
  gvec(W, VS_ZERO_X, GV_ZERO, false);   // x = 0 where b = 0
  for (int s = 0; s < ns; ++s) {
    done[s] = nb[s] == 0.0;
    act[s] = !done[s];
  }
  const int maxit = S->prm.maxiter;
  int it = 0;
  std::vector<double> init(SC_COUNT * (size_t)ns, 0.0);
  auto any = [&]() {
    for (int s = 0; s < ns; ++s)
      if (act[s]) return true;
    return false;
  };
  for (int round = 0;; ++round) {
    push_active(W, act);
    gouter_res(W);
    gvec(W, VS_COPY_RH, GV_COPY, false);
    gvec(W, VS_ZERO_P, GV_ZERO, false);
    gvec(W, VS_ZERO_V, GV_ZERO, false);
    // rho = alpha = omega = 1 for the restarting systems (the others keep theirs)
    gpublish(W);
    for (int s = 0; s < ns; ++s) {
      double* q = &W.hscb[(size_t)s * SC_COUNT];
      if (act[s]) q[SC_RHO] = q[SC_ALPHA] = q[SC_OMEGA] = 1.0;
    }
    HIPCK(hipMemcpyAsync(W.scb, W.hscb, sizeof(double) * SC_COUNT * ns, hipMemcpyHostToDevice,
                         W.dev.stream));
    gvec(W, VS_RINIT, GV_DOT, true);
    gfin(W, VS_RINIT, GF_STORE2, SC_RR, SC_RHO1);
    gpublish(W);
    for (int s = 0; s < ns; ++s)
      if (act[s] && sc(s, SC_RR) <= tol2[s]) act[s] = 0;
    push_active(W, act);
    while (any() && it < maxit) {
      bool ch = false;
      for (int s = 0; s < ns; ++s)
        if (act[s] && sc(s, SC_RHO1) == 0.0) act[s] = 0, ch = true;
      if (ch) push_active(W, act);
      if (!any()) break;
      ++it;
      for (int s = 0; s < ns; ++s) iters[s] += act[s];
      gvec(W, VS_P, GV_P, false);
      gvcycle(W, 0);
      gouter(W, W.outer_spmv[0]);
      gvec(W, VS_RV, GV_DOT, true);
      gfin(W, VS_RV, GF_ALPHA);
      gvec(W, VS_S, GV_S, true);
      gfin(W, VS_S, GF_STORE1, SC_SS);
      gpublish(W);
      ch = false;
      std::vector<int> stop(ns, 0);
      for (int s = 0; s < ns; ++s)
        if (act[s] && sc(s, SC_SS) <= tol2[s]) act[s] = 0, stop[s] = 1, ch = true;
      if (ch) {
        push_active(W, stop);
        gvec(W, VS_S, GV_X, false);   // x += alpha phat for the systems that stop at s
        push_active(W, act);
      }
      if (!any()) break;
      gvcycle(W, 1);
      gouter(W, W.outer_spmv[1]);
      gvec(W, VS_TS, GV_DOT, true);
      gfin(W, VS_TS, GF_OMEGA);
      gvec(W, VS_XR, GV_XR, true);
      gfin(W, VS_XR, GF_RHO);
      gpublish(W);
      ch = false;
      for (int s = 0; s < ns; ++s)
        if (act[s] && (sc(s, SC_RR) <= tol2[s] || sc(s, SC_TT) == 0.0)) act[s] = 0, ch = true;
      if (ch) push_active(W, act);
    }
    // true residuals of every unfinished system
    std::vector<int> want(ns);
    for (int s = 0; s < ns; ++s) want[s] = !done[s];
    push_active(W, want);
    gouter_res(W);
    gvec(W, VS_TRUE, GV_DOT, true);
    gfin(W, VS_TRUE, GF_STORE1, SC_RR);
    gpublish(W);
    bool again = false;
    for (int s = 0; s < ns; ++s) {
      if (done[s]) continue;
      const double rel = std::sqrt(sc(s, SC_RR)) / nb[s];
      infos[s].rel_resid = rel;
      if (rel <= tol) {
        done[s] = 1;
        act[s] = 0;
      } else if (it < maxit && restarts[s] < S->prm.max_restarts) {
        act[s] = 1;
        restarts[s]++;
        again = true;
      } else {
        act[s] = 0;
      }
    }
    if (!again) break;
  }
  int worst = MGK_OK;
  for (int s = 0; s < ns; ++s) {
    infos[s].iters = iters[s];
    infos[s].restarts = restarts[s];
    infos[s].status = done[s] ? MGK_OK : MGK_NOT_CONVERGED;
    infos[s].levels = (int)W.sys[s]->H.lv.size();
    if (!done[s]) worst = MGK_NOT_CONVERGED;
  }
  return worst;
}

}  // namespace mgk

extern "C" {

int mgk_batch_setup(int32_t nsys, const mgk_bsr* const* A, int32_t block_size,
                    mgk_precond_kind kind, const mgk_params* prm, void* hip_stream,
                    mgk_solver** out) {
  if (!out) {
    mgk::g_err = "mgk_batch_setup: null output";
    return MGK_E_INVALID;
  }
  *out = nullptr;
  std::unique_ptr<mgk_solver> S(new mgk_solver());
  return mgk::guard([&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    mgk::batch_setup_impl(S.get(), nsys, A, block_size, kind, prm, hip_stream);
    S->setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = S.release();
    return MGK_OK;
  });
}

int mgk_batch_solve(mgk_solver* s, const double* const* d_b, double* const* d_x, double rtol,
                    mgk_info* infos) {
  if (!s || !s->batch || !d_b || !d_x || !infos || !(rtol > 0.0)) {
    mgk::g_err = "mgk_batch_solve: needs a solver from mgk_batch_setup and non-null arguments";
    return s && !s->batch ? MGK_E_STATE : MGK_E_INVALID;
  }
  return mgk::guard([&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    const int ns = s->batch->nsys;
    for (int q = 0; q < ns; ++q)
      if (!d_b[q] || !d_x[q]) throw mgk::Error(MGK_E_INVALID, "mgk_batch_solve: null vector");
    std::memset(infos, 0, sizeof(mgk_info) * ns);
    const int rc = mgk::batch_bicgstab(s, d_b, d_x, rtol, infos);
    HIPCK(hipStreamSynchronize(s->dev.stream));
    HIPCK(hipGetLastError());
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int64_t bytes = s->batch->dev.bytes;
    for (mgk_solver* q : s->batch->sys) bytes += q->dev.bytes;
    for (int q = 0; q < ns; ++q) {
      infos[q].setup_ms = s->setup_ms;
      infos[q].solve_ms = ms;
      infos[q].device_bytes = bytes;
    }
    return rc;
  });
}

}  // extern "C"
