// Solve-phase orchestration and the C ABI of libmgk: tile autotuner, upload of
// the hierarchy, BiCGStab, FGMRES, the Schur apply, setup and entry points.
// Shared declarations are in internal.hpp; multi-RHS solves are in multi.hip.
#include "internal.hpp"

namespace mgk {

// ---------------------------------------------------------------- tile autotuner

// Picks the fastest engine tile for one stored operator by timing its SpMV on
// the device (a few launches per candidate, each after the caches were cleared, as
// in a solve, where the operator was last read a whole V-cycle or iteration ago);
// results are cached per matrix shape for the process and, when MGK_TUNE_CACHE
// names a file, in that JSON file across processes.
struct TuneCache {
  std::mutex mu;
  std::map<std::string, Tile> m;
  bool loaded = false;
  static TuneCache& get() {
    static TuneCache c;
    return c;
  }
  void load() {
    if (loaded) return;
    loaded = true;
    const char* path = getenv("MGK_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[256];
    int s, u, r;
    // one entry per line: "key": [s, u, rpl],
    char line[512];
    while (fgets(line, sizeof line, f)) {
      const int got = sscanf(line, " \"%255[^\"]\": [%d, %d, %d]", key, &s, &u, &r);
      if (got >= 3) m[key] = Tile{s, u, got == 4 ? r : 1};
    }
    fclose(f);
  }
  void save() {
    const char* path = getenv("MGK_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto& kv : m)
      fprintf(f, "  \"%s\": [%d, %d, %d]%s\n", kv.first.c_str(), kv.second.s, kv.second.u,
              kv.second.rpl, ++i < m.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
  }
};

static thread_local int g_force_tile = 0;  // mgk_params.force_tile of the setup in progress

// Whether a kernel exists for tile t on block rows of BR (wide: the product may
// use the wide-lane BF16 tiles).
template <int BR>
static bool tile_known(const Tile& t, bool wide) {
  bool known = false;
  auto probe = [&](int ss, int uu, int rr) {
    known |= t.s == ss && t.u == uu && t.rpl == rr;
  };
#define MGK_PROBE(SS, UU) probe(SS, UU, 1);
#define MGK_PROBE_W(SS, UU, RR) probe(SS, UU, RR);
  if (BR == 1) {
    MGK_TILES_1(MGK_PROBE)
  } else {
    MGK_TILES_B(MGK_PROBE)
    if (wide) {
      MGK_TILES_W(MGK_PROBE_W)
    }
  }
#undef MGK_PROBE
#undef MGK_PROBE_W
  return known;
}

// Cache clearing for the tuner: reads a buffer twice the size of the 256 MB memory-side
// cache, so that the timed launch finds neither its operator nor its vectors in L2 or
// that cache (nothing is written, so no dirty lines are left to be written back during
// the timed launch).
static __global__ __launch_bounds__(WG) void k_evict(const u4v* __restrict__ p, size_t n,
                                                     unsigned* __restrict__ sink) {
  unsigned a = 0;
  for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < n; i += (size_t)gridDim.x * WG) {
    const u4v v = p[i];   // ordinary loads: streaming loads would not allocate in the caches
    a ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (a == 0x9e3779b9u) sink[0] = a;   // keeps the loads; the buffer is zero, so never taken
}

struct Evictor {
  static constexpr size_t BYTES = (size_t)512 << 20;
  void* buf = nullptr;
  explicit Evictor(hipStream_t st) {
    // MGK_TUNE_WARM=1: time with warm caches (each launch right after the previous one)
    const char* w = getenv("MGK_TUNE_WARM");
    if (w && atoi(w) == 1) return;
    if (hipMalloc(&buf, BYTES + 256) != hipSuccess) {
      (void)hipGetLastError();
      buf = nullptr;   // tune with warm caches instead
      return;
    }
    HIPCK(hipMemsetAsync(buf, 0, BYTES + 256, st));
  }
  void run(hipStream_t st) const {
    if (!buf) return;
    k_evict<<<2048, WG, 0, st>>>((const u4v*)buf, BYTES / 16,
                                 (unsigned*)((char*)buf + BYTES));
  }
  ~Evictor() {
    if (buf) (void)hipFree(buf);
  }
};

// Time `launch` for each candidate tile (three cold launches each); returns the fastest.
template <class F>
static Tile time_candidates(Device& D, const std::vector<Tile>& cands, F&& launch) {
  Evictor ev(D.stream);
  hipEvent_t e[6];
  for (auto& x : e) HIPCK(hipEventCreate(&x));
  Tile best = cands[0];
  float best_ms = 1e30f;
  for (const Tile& t : cands) {
    launch(t);   // first launch of the instantiation
    for (int r = 0; r < 3; ++r) {
      ev.run(D.stream);
      HIPCK(hipEventRecord(e[2 * r], D.stream));
      launch(t);
      HIPCK(hipEventRecord(e[2 * r + 1], D.stream));
    }
    HIPCK(hipEventSynchronize(e[5]));
    float ms = 0;
    for (int r = 0; r < 3; ++r) {
      float m = 0;
      HIPCK(hipEventElapsedTime(&m, e[2 * r], e[2 * r + 1]));
      ms += m;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  for (auto& x : e) (void)hipEventDestroy(x);
  return best;
}

template <int BR>
static std::vector<Tile> tile_candidates(bool wide) {
  std::vector<Tile> cands;
#define MGK_CAND(SS, UU) cands.push_back(Tile{SS, UU, 1});
#define MGK_CAND_W(SS, UU, RR) cands.push_back(Tile{SS, UU, RR});
  if (BR == 1) {
    MGK_TILES_1(MGK_CAND)
  } else {
    MGK_TILES_B(MGK_CAND)
    if (wide) {
      MGK_TILES_W(MGK_CAND_W)
    }
  }
#undef MGK_CAND
#undef MGK_CAND_W
  return cands;
}

// A forced tile (mgk_params.force_tile) when it applies to this product, else {0,0,0}.
template <int BR>
static Tile forced_tile(bool wide) {
  if (!g_force_tile) return Tile{0, 0, 0};
  // 10000*RPL + 100*S + U.  A wide tile (RPL > 1) applies to the products that have
  // wide kernels; the others take (S, U) when that tile exists for them, else the
  // autotuner's choice.  Any other unknown tile is an error.
  const int rpl = g_force_tile / 10000;
  const Tile t{(g_force_tile / 100) % 100, g_force_tile % 100, wide && rpl > 1 ? rpl : 1};
  if (tile_known<BR>(t, wide)) return t;
  if (!(rpl > 1 && !wide))
    throw Error(MGK_E_INVALID, "force_tile " + std::to_string(g_force_tile) +
                                   " is not a kernel tile for block rows of " +
                                   std::to_string(BR));
  return Tile{0, 0, 0};
}

template <int BR, int BC, class TV, class TX>
static Tile autotune(Device& D, const DMat& M, bool trans) {
  const bool wide = wide_ok<BR, BC, TV>() && !trans;
  const Tile ft = forced_tile<BR>(wide);
  if (ft.s) return ft;
  const int nrows = trans ? M.nbc : M.nbr, ncols = trans ? M.nbr : M.nbc;
  if (nrows == 0 || M.nnzb == 0) return BR == 1 ? Tile{4, 4, 1} : Tile{1, 4, 1};
  char key[200];
  snprintf(key, sizeof key, "b%dx%d_v%d_x%d_t%d_r%d_nnz%lld_dia%d", BR, BC, (int)sizeof(TV),
           (int)sizeof(TX), (int)trans, nrows, (long long)M.nnzb, trans ? 0 : M.dia.k);
  TuneCache& C = TuneCache::get();
  {
    std::lock_guard<std::mutex> g(C.mu);
    C.load();
    auto it = C.m.find(key);
    if (it != C.m.end() && tile_known<BR>(it->second, wide)) return it->second;
  }
  const std::vector<Tile> cands = tile_candidates<BR>(wide);
  TX *x = nullptr, *y = nullptr;
  HIPCK(hipMalloc(&x, sizeof(TX) * (size_t)ncols * (trans ? BR : BC) + 64));
  HIPCK(hipMalloc(&y, sizeof(TX) * (size_t)nrows * (trans ? BC : BR) + 64));
  HIPCK(hipMemsetAsync(x, 0, sizeof(TX) * (size_t)ncols * (trans ? BR : BC), D.stream));
  const Tile best = time_candidates(D, cands, [&](const Tile& t) {
    spmv_s<BR, BC, TV, TX, TX>(D.stream, M, trans, t, x, y, 1.0, 0.0);
  });
  HIPCK(hipStreamSynchronize(D.stream));
  (void)hipFree(x);
  (void)hipFree(y);
  std::lock_guard<std::mutex> g(C.mu);
  C.m[key] = best;
  C.save();
  return best;
}

// Tile of the fused FP64 SpMV-and-dots of the outer operator, timed as that kernel: its
// workgroups cover whole 16-row dot groups, so its best tile can differ from the plain
// product's.
template <int BR>
static Tile autotune_dot(Device& D, const DMat& M) {
  const bool wide = wide_ok<BR, BR, double>();
  const Tile ft = forced_tile<BR>(wide);
  if (ft.s) return ft;
  if (M.nbr == 0 || M.nnzb == 0) return M.tile;
  char key[200];
  snprintf(key, sizeof key, "dot_b%d_r%d_nnz%lld_dia%d", BR, M.nbr, (long long)M.nnzb,
           M.dia.k);
  TuneCache& C = TuneCache::get();
  {
    std::lock_guard<std::mutex> g(C.mu);
    C.load();
    auto it = C.m.find(key);
    if (it != C.m.end() && tile_known<BR>(it->second, wide)) return it->second;
  }
  const std::vector<Tile> cands = tile_candidates<BR>(wide);
  const size_t n = (size_t)M.nbr * BR;
  const size_t ng = ((size_t)M.nbr + dot_rows<BR>() - 1) / dot_rows<BR>();
  double *x = nullptr, *y = nullptr, *w = nullptr, *part = nullptr;
  HIPCK(hipMalloc(&x, 8 * n + 64));
  HIPCK(hipMalloc(&y, 8 * n + 64));
  HIPCK(hipMalloc(&w, 8 * n + 64));
  HIPCK(hipMalloc(&part, 16 * ng + 64));
  HIPCK(hipMemsetAsync(x, 0, 8 * n, D.stream));
  HIPCK(hipMemsetAsync(w, 0, 8 * n, D.stream));
  const Tile best = time_candidates(D, cands, [&](const Tile& t) {
    spmv_dot_s<BR, BR>(D.stream, M, false, t, x, y, 1, w, part);
  });
  HIPCK(hipStreamSynchronize(D.stream));
  (void)hipFree(x);
  (void)hipFree(y);
  (void)hipFree(w);
  (void)hipFree(part);
  std::lock_guard<std::mutex> g(C.mu);
  C.m[key] = best;
  C.save();
  return best;
}

// Tune the tiles of one stored operator for its storage and vector precision.
static void tune_mat(Device& D, DMat& M, int storage, bool with_trans) {
  auto run = [&](auto BRc, auto BCc) {
    constexpr int BR = decltype(BRc)::value, BC = decltype(BCc)::value;
    if (storage == MGK_F64) {
      M.tile = autotune<BR, BC, double, double>(D, M, false);
      if (with_trans && BR == BC) M.ttile = autotune<BR, BC, double, double>(D, M, true);
    } else if (storage == MGK_F32) {
      M.tile = autotune<BR, BC, float, float>(D, M, false);
      if (with_trans && BR == BC) M.ttile = autotune<BR, BC, float, float>(D, M, true);
    } else {
      M.tile = autotune<BR, BC, bf16, float>(D, M, false);
      if (with_trans && BR == BC) M.ttile = autotune<BR, BC, bf16, float>(D, M, true);
    }
  };
  using std::integral_constant;
  if (M.br == 1 && M.bc == 1) run(integral_constant<int, 1>(), integral_constant<int, 1>());
  else if (M.br == 3 && M.bc == 3) run(integral_constant<int, 3>(), integral_constant<int, 3>());
  else if (M.br == 4 && M.bc == 4) run(integral_constant<int, 4>(), integral_constant<int, 4>());
  else if (M.br == 1 && M.bc == 3) run(integral_constant<int, 1>(), integral_constant<int, 3>());
  else if (M.br == 3 && M.bc == 1) run(integral_constant<int, 3>(), integral_constant<int, 1>());
  else throw Error(MGK_E_INVALID, "unsupported block shape");
}

static void fill_desc(const HHierarchy& H, std::vector<mgk_level_desc>& desc) {
  desc.resize(H.levels.size());
  for (size_t l = 0; l < H.levels.size(); ++l) {
    const HLevel& h = H.levels[l];
    mgk_level_desc& ds = desc[l];
    ds.n_brows = h.A.nbr;
    ds.block = H.b;
    ds.nnzb = h.A.nnzb();
    ds.n_agg = h.n_agg;
    ds.dia = 0;
    ds.p_nnzb = h.P.nnzb();
    ds.r_nnzb = h.R.nnzb();
    ds.omega = h.omega;
  }
}

static void describe(DHier& H) { fill_desc(H.host, H.desc); }

static void upload_hierarchy(Device& D, HHierarchy& H, int storage, bool with_transpose,
                             DHier& out, const DMat* share_level0, int dia_mode) {
  out.b = H.b;
  out.storage = storage;
  out.trans_ready = with_transpose;
  const int L = (int)H.levels.size();
  out.lv.resize(L);
  out.desc.resize(L);
  const size_t xs = storage == MGK_F64 ? 8 : 4;
  for (int l = 0; l < L; ++l) {
    HLevel& h = H.levels[l];
    DLevel& d = out.lv[l];
    d.nbr = h.A.nbr;
    d.n = (size_t)h.A.nbr * H.b;
    const bool last = l == L - 1;
    if (l == 0 && share_level0 && storage == MGK_F64 && (!with_transpose || share_level0->tptr))
      d.A = *share_level0;
    else if (!last)
      d.A = upload_mat(D, h.A, storage, with_transpose, dia_mode);
    if (!last) {
      d.P = upload_mat(D, h.P, storage, false);
      d.R = upload_mat(D, h.R, storage, false);
      const bool ilu = !h.ilu.Dinv.empty();
      const std::vector<double>& Mh = ilu ? h.ilu.Dinv : h.M;
      // smoother blocks in the hierarchy's storage precision; ILU pivots' inverses in FP32
      // below FP64
      if (storage == MGK_F64) {
        (ilu ? d.Dinv : d.M) = D.upload(Mh.data(), Mh.size());
      } else if (storage == MGK_BF16 && !ilu) {
        std::vector<uint16_t> m(Mh.size());
        for (size_t q = 0; q < Mh.size(); ++q) m[q] = f32_to_bf16((float)Mh[q]);
        d.M = D.upload(m.data(), m.size());
      } else {
        std::vector<float> m(Mh.begin(), Mh.end());
        (ilu ? d.Dinv : d.M) = D.upload(m.data(), m.size());
      }
      if (ilu) {
        out.ilu = true;
        d.Lf = upload_mat(D, h.ilu.L, storage, false);
        d.Uf = upload_mat(D, h.ilu.U, storage, false);
        tune_mat(D, d.Lf, storage, false);
        tune_mat(D, d.Uf, storage, false);
      }
      if (!(l == 0 && share_level0 && storage == MGK_F64 && d.A.ptr == share_level0->ptr))
        tune_mat(D, d.A, storage, with_transpose);
      tune_mat(D, d.P, storage, false);
      tune_mat(D, d.R, storage, false);
    }
    d.r = D.alloc(d.n * xs);
    d.t = D.alloc(d.n * xs);
    d.z = D.alloc(d.n * xs);
    d.z2 = D.alloc(d.n * xs);
  }
  if (out.ilu) {
    const size_t n0 = out.lv[0].n;
    out.sy = D.alloc(n0 * xs);
    out.sy2 = D.alloc(n0 * xs);
    out.sw = D.alloc(n0 * xs);
    out.sz = D.alloc(n0 * xs);
  }
  fill_desc(H, out.desc);
  for (int l = 0; l < L; ++l) out.desc[l].dia = out.lv[l].A.dia.k;
  out.nc = H.nc;
  out.cinv = D.upload(H.coarse_inv.data(), H.coarse_inv.size());
  if (with_transpose) {
    std::vector<double> t((size_t)H.nc * H.nc);
    for (int i = 0; i < H.nc; ++i)
      for (int j = 0; j < H.nc; ++j) t[(size_t)j * H.nc + i] = H.coarse_inv[(size_t)i * H.nc + j];
    out.cinvT = D.upload(t.data(), t.size());
    HIPCK(hipStreamSynchronize(D.stream));
  }
  HIPCK(hipStreamSynchronize(D.stream));
}

}  // namespace mgk

namespace mgk {

void outer_spmv(mgk_solver* S, const double* x, double* y, bool trans, int dots,
                const double* w1, int* nwg) {
  hipStream_t st = S->dev.stream;
  const bool timed = (S->time_mask & 1) && S->tev_used + 2 <= S->tev.size();
  // the fused kernel's own dispatch records its start and end; the plain product (one or
  // more launches) is bracketed by event records on the stream
  hipEvent_t e0 = timed && dots ? S->tev[S->tev_used] : nullptr;
  hipEvent_t e1 = timed && dots ? S->tev[S->tev_used + 1] : nullptr;
  if (timed && !dots) HIPCK(hipEventRecord(S->tev[S->tev_used], st));
  const Tile sp = trans ? S->A.ttile : (dots ? S->A.dtile : S->A.tile);
  int g = 0;
  switch (S->b) {
    case 1:
      if (dots) g = spmv_dot_s<1, 1>(st, S->A, trans, sp, x, y, dots == 2, w1, S->part, e0, e1);
      else spmv_s<1, 1, double, double, double>(st, S->A, trans, sp, x, y, 1.0, 0.0);
      break;
    case 3:
      if (dots) g = spmv_dot_s<3, 3>(st, S->A, trans, sp, x, y, dots == 2, w1, S->part, e0, e1);
      else spmv_s<3, 3, double, double, double>(st, S->A, trans, sp, x, y, 1.0, 0.0);
      break;
    case 4:
      if (dots) g = spmv_dot_s<4, 4>(st, S->A, trans, sp, x, y, dots == 2, w1, S->part, e0, e1);
      else spmv_s<4, 4, double, double, double>(st, S->A, trans, sp, x, y, 1.0, 0.0);
      break;
  }
  if (nwg) *nwg = g;
  if (timed) {
    if (!dots) HIPCK(hipEventRecord(S->tev[S->tev_used + 1], st));
    HIPCK(hipGetLastError());
    S->tev_used += 2;
  }
}

void outer_residual(mgk_solver* S, const double* b, const double* x, double* r, bool trans) {
  hipStream_t st = S->dev.stream;
  const Tile sp = trans ? S->A.ttile : S->A.tile;
  switch (S->b) {
    case 1: residual_s<1, 1, double, double, double>(st, S->A, trans, sp, b, x, r); break;
    case 3: residual_s<3, 3, double, double, double>(st, S->A, trans, sp, b, x, r); break;
    case 4: residual_s<4, 4, double, double, double>(st, S->A, trans, sp, b, x, r); break;
  }
}

// Schur apply: z = B r for interleaved FP64 vectors: z_u = V_u(r_u);
// z_p = P_S(r_p - B_lo z_u) with P_S a V-cycle on S or its SPAI(0); then, for
// the full factorization, z_u = V_u(r_u - B_up z_p) (eqs. SchurP, SchurU).
template <class TV, class TX>
static void schur_apply_t(mgk_solver* S, const double* r, double* z) {
  hipStream_t st = S->dev.stream;
  const size_t nn = (size_t)S->nbr;
  TX *ru = (TX*)S->ru, *rp = (TX*)S->rp, *tu = (TX*)S->tu, *tp = (TX*)S->tp, *zu = (TX*)S->zu,
     *zp = (TX*)S->zp;
  k_split<TX><<<grid_for(nn), WG, 0, st>>>(nn, r, ru, rp);
  vcycle<TX, TX>(st, S->H, ru, zu, false);
  residual_s<1, 3, TV, TX, TX>(st, S->Blo, false, S->Blo.tile, rp, zu, tp);
  if (S->prm.schur_spai0)
    k_diag_mul<TX><<<grid_for(nn), WG, 0, st>>>(nn, (const TX*)S->Sm, tp, zp);
  else
    vcycle<TX, TX>(st, S->Hp, tp, zp, false);
  if (!S->prm.schur_lower) {
    residual_s<3, 1, TV, TX, TX>(st, S->Bup, false, S->Bup.tile, ru, zp, tu);
    vcycle<TX, TX>(st, S->H, tu, zu, false);
  }
  k_merge<TX><<<grid_for(nn), WG, 0, st>>>(nn, zu, zp, z);
}

// Block ILU preconditioner (MGK_ILU) in the storage precision, FP64 in and out.
template <int B, class TV, class TX>
static void ilu_apply_b(mgk_solver* S, const double* r, double* z) {
  ilu_sweeps<B, TV, TX, double, double>(S->dev.stream, S->Lf, S->Uf, S->Dinv, S->nbr,
                                        S->prm.ilu_sweeps, r, z, (TX*)S->iy, (TX*)S->iy2,
                                        (TX*)S->iw, (TX*)S->iz);
}

template <class TV, class TX>
static void ilu_apply_t(mgk_solver* S, const double* r, double* z) {
  switch (S->b) {
    case 1: ilu_apply_b<1, TV, TX>(S, r, z); break;
    case 3: ilu_apply_b<3, TV, TX>(S, r, z); break;
    case 4: ilu_apply_b<4, TV, TX>(S, r, z); break;
  }
}

static void precond_apply(mgk_solver* S, const double* r, double* z, bool trans);

// One preconditioner application z = B r, bracketed by timing events when requested.
void precond(mgk_solver* S, const double* r, double* z, bool trans) {
  const bool timed = (S->time_mask & 2) && S->pev_used + 2 <= S->pev.size();
  if (timed) HIPCK(hipEventRecord(S->pev[S->pev_used], S->dev.stream));
  precond_apply(S, r, z, trans);
  if (timed) {
    HIPCK(hipEventRecord(S->pev[S->pev_used + 1], S->dev.stream));
    S->pev_used += 2;
  }
}

// The AMG V-cycle of an FP32 or BF16 hierarchy from an FP32 input (the copies p32 / s32).
void precond(mgk_solver* S, const float* r, double* z) {
  const bool timed = (S->time_mask & 2) && S->pev_used + 2 <= S->pev.size();
  if (timed) HIPCK(hipEventRecord(S->pev[S->pev_used], S->dev.stream));
  hipStream_t st = S->dev.stream;
  DHier& H = S->H;
#define MGK_VC32(BB)                                                               \
  case BB:                                                                         \
    if (H.storage == MGK_F32) Cycle<BB, float, float>::run<float, double>(st, H, 0, r, z, false); \
    else Cycle<BB, bf16, float>::run<float, double>(st, H, 0, r, z, false);        \
    break;
  if (H.storage == MGK_F64 || S->kind == MGK_SCHUR || S->kind == MGK_ILU || H.ilu)
    throw Error(MGK_E_STATE, "FP32 preconditioner input needs an FP32/BF16 AMG hierarchy");
  switch (H.b) {
    MGK_VC32(1)
    MGK_VC32(3)
    MGK_VC32(4)
    default: throw Error(MGK_E_INVALID, "unsupported block size");
  }
#undef MGK_VC32
  if (timed) {
    HIPCK(hipEventRecord(S->pev[S->pev_used + 1], S->dev.stream));
    S->pev_used += 2;
  }
}

static void precond_apply(mgk_solver* S, const double* r, double* z, bool trans) {
  if (S->kind == MGK_ILU) {
    if (trans) throw Error(MGK_E_STATE, "transposed ILU preconditioner is not available");
    if (S->prm.hier == MGK_F64) ilu_apply_t<double, double>(S, r, z);
    else if (S->prm.hier == MGK_F32) ilu_apply_t<float, float>(S, r, z);
    else ilu_apply_t<bf16, float>(S, r, z);
    return;
  }
  if (S->kind == MGK_SCHUR) {
    if (trans) throw Error(MGK_E_STATE, "transposed Schur preconditioner is not available");
    if (S->H.storage == MGK_F64) schur_apply_t<double, double>(S, r, z);
    else if (S->H.storage == MGK_F32) schur_apply_t<float, float>(S, r, z);
    else schur_apply_t<bf16, float>(S, r, z);
  } else {
    vcycle<double, double>(S->dev.stream, S->H, r, z, trans);
  }
}

// ---------------------------------------------------------------- BiCGStab

static int red_grid(size_t n) { return grid_for(n); }
static int maxiter_of(const mgk_solver* S) { return S->prm.maxiter; }

void finalize(mgk_solver* S, int count, int two, int op, int i0, int i1, double* sc) {
  if (!sc) sc = S->sc;
  // stages of RED_CHUNK partials each until one workgroup can finish (k_finalize reads at
  // most RED_CHUNK); later stages ping-pong between part2 and the consumed part
  const double* src = S->part;
  double* dst[2] = {S->part2, S->part};
  for (int w = 0; count > RED_CHUNK; w ^= 1) {
    const int nb = (count + RED_CHUNK - 1) / RED_CHUNK;
    k_reduce_stage<<<nb, WG, 0, S->dev.stream>>>(src, count, two, dst[w]);
    src = dst[w];
    count = nb;
  }
  k_finalize<<<1, WG, 0, S->dev.stream>>>(src, count, two, op, i0, i1, sc);
}

// Copy the device scalars to pinned memory and mark the point with event e.
static void publish(mgk_solver* S, int e) {
  HIPCK(hipMemcpyAsync(S->hsc, S->sc, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost,
                       S->dev.stream));
  HIPCK(hipEventRecord(S->ev[e], S->dev.stream));
}

static void wait(mgk_solver* S, int e) {
  HIPCK(hipEventSynchronize(S->ev[e]));
  HIPCK(hipGetLastError());
}

double norm2(mgk_solver* S, const double* a) {
  const size_t n = S->n;
  const int g = red_grid(n);
  k_dot2<<<g, WG, 0, S->dev.stream>>>(n, a, a, nullptr, nullptr, S->part);
  finalize(S, g, 0, FIN_STORE1, SC_TMP);
  publish(S, 3);
  wait(S, 3);
  return std::sqrt(S->hsc[SC_TMP]);
}

static int bicgstab(mgk_solver* S, const double* b, double* x, double tol, bool trans,
                    mgk_info* info) {
  hipStream_t st = S->dev.stream;
  const size_t n = S->n;
  const int g = red_grid(n);
  const double nb = norm2(S, b);
  info->iters = 0;
  info->restarts = 0;
  if (nb == 0.0) {
    k_fill<<<g, WG, 0, st>>>(n, 0.0, x);
    info->rel_resid = 0.0;
    return MGK_OK;
  }
  const double tol2 = (tol * nb) * (tol * nb);
  // FP32 V-cycle inputs where the hierarchy takes them (forward cycles)
  float* p32 = trans ? nullptr : S->p32;
  float* s32 = trans ? nullptr : S->s32;
  int it = 0;
  for (int restart = 0;; ++restart) {
    // r = b - A x; rhat = r; rho = alpha = omega = 1; p = v = 0
    outer_residual(S, b, x, S->r, trans);
    k_copy<<<g, WG, 0, st>>>(n, S->r, S->rh);
    k_fill<<<g, WG, 0, st>>>(n, 0.0, S->p);
    k_fill<<<g, WG, 0, st>>>(n, 0.0, S->v);
    k_dot2<<<g, WG, 0, st>>>(n, S->r, S->r, S->rh, S->r, S->part);
    {
      // sc[RR] = ||r||^2, sc[RHO1] = (rhat, r); rho = alpha = omega = 1
      double init[SC_COUNT] = {0};
      init[SC_RHO] = init[SC_ALPHA] = init[SC_OMEGA] = 1.0;
      std::memcpy(S->hsc, init, sizeof(init));
      HIPCK(hipMemcpyAsync(S->sc, S->hsc, sizeof(init), hipMemcpyHostToDevice, st));
      finalize(S, g, 1, FIN_STORE2, SC_RR, SC_RHO1);
      publish(S, 1);
      wait(S, 1);
    }
    bool done = S->hsc[SC_RR] <= tol2;
    bool pending_v = false;  // the p / V-cycle / v stage of iteration it+1 is queued
    while (!done && it < maxiter_of(S)) {
      if (S->hsc[SC_RHO1] == 0.0) break;  // breakdown: restart
      ++it;
      if (!pending_v) {
        k_bicg_p<<<g, WG, 0, st>>>(n, S->sc, S->r, S->v, S->p, p32);
        if (p32) precond(S, p32, S->ph);
        else precond(S, S->p, S->ph, trans);
        int nw = 0;
        outer_spmv(S, S->ph, S->v, trans, 1, S->rh, &nw);
        finalize(S, nw, 0, FIN_ALPHA);
      }
      pending_v = false;
      k_bicg_s<<<g, WG, 0, st>>>(n, S->sc, S->r, S->v, S->s, s32, S->part);
      finalize(S, g, 0, FIN_STORE1, SC_SS);
      publish(S, 0);
      // speculative: shat = M s; t = A shat (harmless if we stop after s)
      if (s32) precond(S, s32, S->sh);
      else precond(S, S->s, S->sh, trans);
      int nw = 0;
      outer_spmv(S, S->sh, S->t, trans, 2, S->s, &nw);  // partials (s,t), (t,t)
      finalize(S, nw, 1, FIN_OMEGA);
      wait(S, 0);
      if (S->hsc[SC_SS] <= tol2) {   // stop at s: x + alpha phat
        k_bicg_x<<<g, WG, 0, st>>>(n, S->sc, S->ph, x);
        break;
      }
      k_bicg_xr<<<g, WG, 0, st>>>(n, S->sc, S->s, S->t, S->ph, S->sh, S->rh, x, S->r, S->part);
      finalize(S, g, 1, FIN_RHO);
      publish(S, 1);
      if (it < maxiter_of(S)) {
        // speculative next p / V-cycle / v (x untouched)
        k_bicg_p<<<g, WG, 0, st>>>(n, S->sc, S->r, S->v, S->p, p32);
        if (p32) precond(S, p32, S->ph);
        else precond(S, S->p, S->ph, trans);
        int nw2 = 0;
        outer_spmv(S, S->ph, S->v, trans, 1, S->rh, &nw2);
        finalize(S, nw2, 0, FIN_ALPHA);
        pending_v = true;
      }
      wait(S, 1);
      if (S->hsc[SC_TT] == 0.0) break;  // breakdown
      if (S->hsc[SC_RR] <= tol2) done = true;
    }
    // true residual
    outer_residual(S, b, x, S->r, trans);
    const double rn = norm2(S, S->r);
    info->rel_resid = rn / nb;
    info->iters = it;
    info->restarts = restart;
    if (info->rel_resid <= tol) return MGK_OK;
    if (it >= maxiter_of(S) || restart >= S->prm.max_restarts) return MGK_NOT_CONVERGED;
  }
}

}  // namespace mgk

namespace mgk {

// ---------------------------------------------------------------- FGMRES

static void arnoldi_products(mgk_solver* S, int j, double* w, int* nw_unused) {
  (void)nw_unused;
  hipStream_t st = S->dev.stream;
  const size_t n = S->n;
  const int g = red_grid(n);
  // h = V^T w; w -= V h; h2 = V^T w; w -= V h2; hsum = h + h2; ||w||^2
  multidot(st, g, n, j + 1, S->V, n, w, S->part);
  k_multifin<<<1, WG, 0, st>>>(S->part, g, j + 1, S->h, S->hsum, 0);
  k_multiaxpy<<<g, WG, 0, st>>>(n, j + 1, S->V, n, S->h, w, nullptr);
  multidot(st, g, n, j + 1, S->V, n, w, S->part);
  k_multifin<<<1, WG, 0, st>>>(S->part, g, j + 1, S->h, S->hsum, 1);
  k_multiaxpy<<<g, WG, 0, st>>>(n, j + 1, S->V, n, S->h, w, S->part);
  finalize(S, g, 0, FIN_STORE1, SC_TMP);
}

static int fgmres(mgk_solver* S, const double* b, double* x, double tol, mgk_info* info) {
  hipStream_t st = S->dev.stream;
  const size_t n = S->n;
  const int g = red_grid(n);
  const int m = S->m;
  const double nb = norm2(S, b);
  info->iters = 0;
  info->restarts = 0;
  if (nb == 0.0) {
    k_fill<<<g, WG, 0, st>>>(n, 0.0, x);
    info->rel_resid = 0.0;
    return MGK_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1);
  int total = 0;
  for (int cycle = 0;; ++cycle) {
    double* V0 = S->V;
    outer_residual(S, b, x, V0, false);
    const double beta = norm2(S, V0);
    info->rel_resid = beta / nb;
    info->iters = total;
    info->restarts = cycle;
    if (beta / nb <= tol) return MGK_OK;
    if (total >= S->prm.maxiter) return MGK_NOT_CONVERGED;
    k_scal<<<g, WG, 0, st>>>(n, 1.0 / beta, V0, V0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k = 0;
    auto stage = [&](int j) {
      // Z_j = M V_j; V_{j+1} <- A Z_j, orthogonalized and normalized on device
      double* Vj = S->V + (size_t)j * n;
      double* Zj = S->Z + (size_t)j * n;
      double* w = S->V + (size_t)(j + 1) * n;
      precond(S, Vj, Zj, false);
      outer_spmv(S, Zj, w, false);
      arnoldi_products(S, j, w, nullptr);
      HIPCK(hipMemcpyAsync(S->hpin + (size_t)j * (MAXM + 1), S->hsum, sizeof(double) * (j + 1),
                           hipMemcpyDeviceToHost, st));
      HIPCK(hipMemcpyAsync(S->hpin + (size_t)j * (MAXM + 1) + MAXM, S->sc + SC_TMP,
                           sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCK(hipEventRecord(S->ev[j & 1], st));
      k_scale<<<g, WG, 0, st>>>(n, S->sc, SC_TMP, 1, w, w);
    };
    stage(0);
    for (int j = 0; j < m && total < S->prm.maxiter; ++j) {
      if (j + 1 < m && total + 1 < S->prm.maxiter) stage(j + 1);  // speculative next step
      wait(S, j & 1);
      const double* hj = S->hpin + (size_t)j * (MAXM + 1);
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hj[i];
      const double hn = std::sqrt(hj[MAXM]);
      H[(size_t)(j + 1) * m + j] = hn;
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
      const double den = std::hypot(a, c);
      cs[j] = a / den;
      sn[j] = c / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++total;
      k = j + 1;
      if (std::fabs(gv[j + 1]) / nb <= tol || hn == 0.0) break;
    }
    // drain speculative work before reusing the host buffers
    HIPCK(hipStreamSynchronize(st));
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
      double sum = gv[i];
      for (int q = i + 1; q < k; ++q) sum -= H[(size_t)i * m + q] * y[q];
      y[i] = sum / H[(size_t)i * m + i];
    }
    std::memcpy(S->hpin + (size_t)MAXM * (MAXM + 1), y.data(), sizeof(double) * k);
    HIPCK(hipMemcpyAsync(S->yv, S->hpin + (size_t)MAXM * (MAXM + 1), sizeof(double) * k,
                         hipMemcpyHostToDevice, st));
    k_update_x<<<g, WG, 0, st>>>(n, k, S->Z, n, S->yv, x);
  }
}

// ---------------------------------------------------------------- setup

static SetupParams setup_params(const mgk_params& p, int kind) {
  SetupParams sp;
  sp.eps_strong = p.eps_strong;
  sp.coarse_enough = p.coarse_enough;
  sp.max_levels = p.max_levels;
  sp.jacobi_omega = p.jacobi_omega;
  sp.smoother = kind == MGK_AMG_JACOBI ? SM_JACOBI : (p.block_spai0 ? SM_SPAI0_BLOCK : SM_SPAI0_SCALAR);
  sp.smooth_p = p.coarsening == MGK_SMOOTHED_AGGREGATION;
  sp.ilu_smoother = p.ilu_smoother != 0;
  sp.ilu_kind = p.ilu_kind;
  sp.ilut_p = p.ilut_p;
  sp.ilut_tau = p.ilut_tau;
  sp.ilu_sweeps = p.ilu_sweeps;
  return sp;
}

static void alloc_krylov(mgk_solver* S) {
  Device& D = S->dev;
  const size_t n = S->n, nb = n * sizeof(double);
  S->r = (double*)D.alloc(nb);
  S->rh = (double*)D.alloc(nb);
  S->p = (double*)D.alloc(nb);
  S->v = (double*)D.alloc(nb);
  S->ph = (double*)D.alloc(nb);
  S->s = (double*)D.alloc(nb);
  S->sh = (double*)D.alloc(nb);
  S->t = (double*)D.alloc(nb);
  if (S->prm.krylov == MGK_BICGSTAB && S->prm.hier != MGK_F64 && S->kind != MGK_SCHUR &&
      S->kind != MGK_ILU && !S->prm.ilu_smoother) {
    S->p32 = (float*)D.alloc(n * sizeof(float));
    S->s32 = (float*)D.alloc(n * sizeof(float));
  }
  S->sc = (double*)D.alloc(sizeof(double) * SC_COUNT);
  // partials: two dots per workgroup of the finest SpMV, or MAXM dots per
  // reduction workgroup
  // (at least 4 block rows per workgroup, two dots)
  S->part_len = std::max<size_t>((size_t)S->nbr / 2 + 4096, (size_t)MAXM * 1024 + 1024);
  S->part = (double*)D.alloc(sizeof(double) * S->part_len);
  S->part2 = (double*)D.alloc(sizeof(double) * (2 * (S->part_len / RED_CHUNK + 2)));
  HIPCK(hipHostMalloc((void**)&S->hsc, sizeof(double) * SC_COUNT, hipHostMallocDefault));
  for (auto& e : S->ev) HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  S->time_mask = S->prm.time_spmv & 3;
  if (S->prm.time_spmv & 1) {
    S->tev.resize(2 * (2 * (size_t)S->prm.maxiter + 64));
    for (auto& e : S->tev) HIPCK(hipEventCreate(&e));
  }
  if (S->prm.time_spmv & 2) {
    S->pev.resize(2 * (2 * (size_t)S->prm.maxiter + 64));
    for (auto& e : S->pev) HIPCK(hipEventCreate(&e));
  }
  if (S->prm.krylov == MGK_IDRS) S->idr = idr_create(S);
  if (S->prm.krylov == MGK_FGMRES) {
    S->m = std::max(1, std::min<int>(S->prm.fgmres_m, MAXM - 1));
    S->V = (double*)D.alloc(nb * (S->m + 1));
    S->Z = (double*)D.alloc(nb * S->m);
    S->h = (double*)D.alloc(sizeof(double) * MAXM);
    S->hsum = (double*)D.alloc(sizeof(double) * MAXM);
    S->yv = (double*)D.alloc(sizeof(double) * MAXM);
    HIPCK(hipHostMalloc((void**)&S->hpin, sizeof(double) * (MAXM + 1) * (MAXM + 1),
                        hipHostMallocDefault));
  }
}

static void setup_impl(mgk_solver* S, const mgk_bsr* A, int block_size, int kind,
                       const mgk_params* prm, void* stream, bool host_only = false) {
  auto t0 = std::chrono::steady_clock::now();
  if (!A || !prm) throw Error(MGK_E_INVALID, "null matrix or params");
  if (A->block != block_size || (block_size != 1 && block_size != 3 && block_size != 4))
    throw Error(MGK_E_INVALID, "block_size must equal A->block and be 1, 3 or 4");
  if (kind < MGK_AMG_SPAI0 || kind > MGK_ILU) throw Error(MGK_E_INVALID, "unknown kind");
  if (kind == MGK_ILU && (prm->ilu_level < 0 || prm->ilu_level > 1))
    throw Error(MGK_E_INVALID, "MGK_ILU needs ilu_level in {0, 1}");
  if (prm->ilu_sweeps < 0 || prm->ilu_sweeps > 64)
    throw Error(MGK_E_INVALID, "ilu_sweeps must be in 0..64");
  if (prm->ilu_smoother & ~1) throw Error(MGK_E_INVALID, "ilu_smoother is 0 or 1");
  if (prm->ilu_kind & ~1) throw Error(MGK_E_INVALID, "ilu_kind is 0 (ILU(k)) or 1 (ILUT)");
  if (prm->layout < 0 || prm->layout > 2)
    throw Error(MGK_E_INVALID, "layout is 0 (automatic), 1 (BSR only) or 2 (diagonal layout "
                               "whatever the padding)");
  if (prm->ilu_kind == 1 && !(prm->ilut_p >= 0.0 && prm->ilut_p <= 1e6 && prm->ilut_tau >= 0.0 &&
                              std::isfinite(prm->ilut_tau)))
    throw Error(MGK_E_INVALID, "ILUT needs 0 <= ilut_p <= 1e6 and finite ilut_tau >= 0");
  if (prm->schur_scalar_u & ~1) throw Error(MGK_E_INVALID, "schur_scalar_u is 0 or 1");
  if (prm->ilu_smoother && prm->enable_transpose)
    throw Error(MGK_E_INVALID, "the ILU smoother has no transposed cycle (enable_transpose)");
  if (kind == MGK_SCHUR && block_size != 4)
    throw Error(MGK_E_INVALID, "MGK_SCHUR needs interleaved [u,v,w,p] (block size 4)");
  if (prm->hier < MGK_F64 || prm->hier > MGK_BF16) throw Error(MGK_E_INVALID, "unknown storage");
  if (prm->krylov != MGK_BICGSTAB && prm->krylov != MGK_FGMRES && prm->krylov != MGK_IDRS)
    throw Error(MGK_E_INVALID, "unknown Krylov method");
  if (prm->krylov == MGK_IDRS && (prm->idr_s < 1 || prm->idr_s > IDR_MAX_S))
    throw Error(MGK_E_INVALID, "IDR(s) needs 1 <= idr_s <= " + std::to_string(IDR_MAX_S));
  if (prm->coarsening != MGK_SMOOTHED_AGGREGATION && prm->coarsening != MGK_PLAIN_AGGREGATION)
    throw Error(MGK_E_INVALID, "unknown coarsening");
  if ((prm->schur_approx | prm->schur_spai0 | prm->schur_lower) & ~1)
    throw Error(MGK_E_INVALID, "schur_approx, schur_spai0 and schur_lower are 0 or 1");
  if (prm->maxiter < 1 || prm->coarse_enough < 1 || prm->max_levels < 1 || prm->fgmres_m < 1)
    throw Error(MGK_E_INVALID, "maxiter, coarse_enough, max_levels and fgmres_m must be >= 1");
  if (A->n_brows < 1 || !A->rowptr || (!A->col && A->rowptr[A->n_brows] > 0))
    throw Error(MGK_E_INVALID, "empty or null matrix arrays");
  S->prm = *prm;
  g_force_tile = prm->force_tile;
  S->kind = kind;
  S->b = block_size;
  S->nbr = A->n_brows;
  S->n = (size_t)A->n_brows * block_size;
  S->dev.stream = (hipStream_t)stream;
  HBsr& H = S->A_host;
  H.br = H.bc = block_size;
  H.nbr = H.nbc = A->n_brows;
  H.ptr.assign(A->rowptr, A->rowptr + A->n_brows + 1);
  if (H.ptr[0] != 0 || H.ptr.back() < 0) throw Error(MGK_E_INVALID, "invalid row pointer");
  H.col.assign(A->col, A->col + H.ptr.back());
  H.val.assign(A->val, A->val + (size_t)H.ptr.back() * block_size * block_size);
  std::string err;
  if (validate_bsr(H, err)) throw Error(MGK_E_INVALID, err);
  const bool tr = prm->enable_transpose != 0;
  S->host_only = host_only;
  if (host_only) {
    // hierarchy only, kept on the host for inspection; no device work
    const SetupParams sp = setup_params(*prm, kind);
    int rc;
    if (kind == MGK_ILU) {
      if ((rc = prm->ilu_kind == 1
                    ? ilut_factor(H, prm->ilut_p, prm->ilut_tau, S->ilu_host, err)
                    : ilu_factor(H, prm->ilu_level, S->ilu_host, err)))
        throw Error(rc, err);
      S->ilu_kept = true;
    } else if (kind == MGK_SCHUR) {
      SchurParts parts;
      if ((rc = schur_split(H, prm->schur_approx != 0, parts, err))) throw Error(rc, err);
      if (prm->schur_scalar_u) parts.Auu = scalar_form(parts.Auu);
      if ((rc = build_hierarchy(parts.Auu, sp, S->H.host, err))) throw Error(rc, err);
      if (!prm->schur_spai0) {
        if ((rc = build_hierarchy(parts.S, sp, S->Hp.host, err))) throw Error(rc, err);
        S->Hp.keep_host = true;
        describe(S->Hp);
      }
    } else {
      if ((rc = build_hierarchy(H, sp, S->H.host, err))) throw Error(rc, err);
    }
    S->H.keep_host = true;
    describe(S->H);
    S->setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return;
  }
  // diagonal layout: 1 with the padding limit, 2 whatever the padding, 0 never
  const int dia = prm->layout == 0 ? 1 : prm->layout == 2 ? 2 : 0;
  S->A = upload_mat(S->dev, H, MGK_F64, tr, dia);
  S->A.cached = operator_cached(MGK_F64, true);
  tune_mat(S->dev, S->A, MGK_F64, tr);
  switch (S->b) {
    case 1: S->A.dtile = autotune_dot<1>(S->dev, S->A); break;
    case 3: S->A.dtile = autotune_dot<3>(S->dev, S->A); break;
    case 4: S->A.dtile = autotune_dot<4>(S->dev, S->A); break;
  }
  const SetupParams sp = setup_params(*prm, kind);
  int rc;
  if (kind == MGK_ILU) {
    IluFactors f;
    if ((rc = prm->ilu_kind == 1 ? ilut_factor(H, prm->ilut_p, prm->ilut_tau, f, err)
                                 : ilu_factor(H, prm->ilu_level, f, err)))
      throw Error(rc, err);
    S->Lf = upload_mat(S->dev, f.L, prm->hier, false);
    S->Uf = upload_mat(S->dev, f.U, prm->hier, false);
    tune_mat(S->dev, S->Lf, prm->hier, false);
    tune_mat(S->dev, S->Uf, prm->hier, false);
    if (prm->hier == MGK_F64) {
      S->Dinv = S->dev.upload(f.Dinv.data(), f.Dinv.size());
    } else {
      std::vector<float> d(f.Dinv.begin(), f.Dinv.end());
      S->Dinv = S->dev.upload(d.data(), d.size());
    }
    if (prm->keep_host) {
      S->ilu_host = std::move(f);
      S->ilu_kept = true;
    }
    const size_t xs = prm->hier == MGK_F64 ? 8 : 4;
    S->iy = S->dev.alloc(S->n * xs);
    S->iy2 = S->dev.alloc(S->n * xs);
    S->iw = S->dev.alloc(S->n * xs);
    S->iz = S->dev.alloc(S->n * xs);
    HIPCK(hipStreamSynchronize(S->dev.stream));
  } else if (kind == MGK_SCHUR) {
    SchurParts parts;
    if ((rc = schur_split(H, prm->schur_approx != 0, parts, err))) throw Error(rc, err);
    if (prm->schur_scalar_u) parts.Auu = scalar_form(parts.Auu);
    HHierarchy hu, hp;
    if ((rc = build_hierarchy(parts.Auu, sp, hu, err))) throw Error(rc, err);
    upload_hierarchy(S->dev, hu, prm->hier, false, S->H, nullptr, dia);
    S->H.ilu_sweeps = prm->ilu_sweeps;
    if (prm->schur_spai0) {
      std::vector<double> m;
      if ((rc = scalar_spai0(parts.S, m, err))) throw Error(rc, err);
      if (prm->hier == MGK_F64) {
        S->Sm = S->dev.upload(m.data(), m.size());
      } else {
        std::vector<float> mf(m.begin(), m.end());
        S->Sm = S->dev.upload(mf.data(), mf.size());
      }
      HIPCK(hipStreamSynchronize(S->dev.stream));
    } else {
      if ((rc = build_hierarchy(parts.S, sp, hp, err))) throw Error(rc, err);
      upload_hierarchy(S->dev, hp, prm->hier, false, S->Hp, nullptr, dia);
      S->Hp.ilu_sweeps = prm->ilu_sweeps;
    }
    S->Blo = upload_mat(S->dev, parts.Blo, prm->hier, false);
    S->Bup = upload_mat(S->dev, parts.Bup, prm->hier, false);
    tune_mat(S->dev, S->Blo, prm->hier, false);
    tune_mat(S->dev, S->Bup, prm->hier, false);
    const size_t xs = prm->hier == MGK_F64 ? 8 : 4, nn = (size_t)S->nbr;
    S->ru = S->dev.alloc(3 * nn * xs);
    S->tu = S->dev.alloc(3 * nn * xs);
    S->zu = S->dev.alloc(3 * nn * xs);
    S->rp = S->dev.alloc(nn * xs);
    S->tp = S->dev.alloc(nn * xs);
    S->zp = S->dev.alloc(nn * xs);
    if (prm->keep_host) {
      S->H.host = std::move(hu);
      S->Hp.host = std::move(hp);
      S->H.keep_host = S->Hp.keep_host = true;
    }
  } else {
    HHierarchy hh;
    if ((rc = build_hierarchy(H, sp, hh, err))) throw Error(rc, err);
    upload_hierarchy(S->dev, hh, prm->hier, tr, S->H, &S->A, dia);
    S->H.ilu_sweeps = prm->ilu_sweeps;
    if (prm->keep_host) {
      S->H.host = std::move(hh);
      S->H.keep_host = true;
    }
  }
  alloc_krylov(S);
  HIPCK(hipStreamSynchronize(S->dev.stream));
  S->setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}


}  // namespace mgk

// ---------------------------------------------------------------- C ABI



extern "C" {

const char* mgk_last_error(void) { return mgk::g_err.c_str(); }

int mgk_params_default(mgk_params* p) {
  if (!p) return MGK_E_INVALID;
  std::memset(p, 0, sizeof(*p));
  p->krylov = MGK_BICGSTAB;
  p->fgmres_m = 30;
  p->maxiter = 1000;
  p->max_restarts = 5;
  p->hier = MGK_F64;
  p->coarse_enough = 3000;
  p->max_levels = 20;
  p->block_spai0 = 1;
  p->eps_strong = 0.08;
  p->jacobi_omega = 2.0 / 3.0;
  p->keep_host = 0;
  p->enable_transpose = 0;
  p->coarsening = MGK_SMOOTHED_AGGREGATION;
  p->idr_s = 5;
  p->ilu_level = 0;
  p->ilu_sweeps = 2;
  p->ilu_kind = 0;
  p->ilut_p = 2.0;
  p->ilut_tau = 1e-2;
  return MGK_OK;
}

int mgk_stokes_sizes(int32_t n, int32_t* n_brows, int64_t* nnzb) {
  if (n < 3 || n > 1290 || !n_brows || !nnzb) {
    mgk::g_err = "mgk_stokes_sizes: need 3 <= n <= 1290 and non-null outputs";
    return MGK_E_INVALID;
  }
  mgk::stokes_sizes(n, *n_brows, *nnzb);
  return MGK_OK;
}

int mgk_stokes_assemble(int32_t n, const double* theta, int32_t* rowptr, int32_t* col,
                        double* val) {
  if (n < 3 || n > 1290 || !rowptr || !col || !val) {
    mgk::g_err = "mgk_stokes_assemble: need 3 <= n <= 1290 and non-null outputs";
    return MGK_E_INVALID;
  }
  if (theta) {
    const size_t nc = (size_t)(n - 1) * (n - 1) * (n - 1);
    for (size_t e = 0; e < nc; ++e)
      if (!(theta[e] > 0.0) || !std::isfinite(theta[e])) {
        mgk::g_err = "mgk_stokes_assemble: theta must be positive and finite";
        return MGK_E_INVALID;
      }
  }
  mgk::stokes_assemble(n, theta, rowptr, col, val);
  return MGK_OK;
}

int mgk_csr_to_bsr(int32_t nrows, const int32_t* ptr, const int32_t* col, const double* val,
                   int32_t b, int32_t* bptr, int32_t* bcol, double* bval, int64_t* nnzb) {
  return mgk::guard([&]() -> int {
    if (!ptr || !nnzb || (nrows > 0 && ptr[nrows] > 0 && (!col || !val)))
      throw mgk::Error(MGK_E_INVALID, "mgk_csr_to_bsr: null argument");
    mgk::HBsr out;
    std::string err;
    if (mgk::csr_to_bsr(nrows, ptr, col, val, b, out, err)) throw mgk::Error(MGK_E_INVALID, err);
    *nnzb = out.nnzb();
    if (bcol) {
      if (!bptr || !bval) throw mgk::Error(MGK_E_INVALID, "mgk_csr_to_bsr: null output");
      std::memcpy(bptr, out.ptr.data(), sizeof(int32_t) * out.ptr.size());
      std::memcpy(bcol, out.col.data(), sizeof(int32_t) * out.col.size());
      std::memcpy(bval, out.val.data(), sizeof(double) * out.val.size());
    }
    return MGK_OK;
  });
}

int mgk_setup(const mgk_bsr* A, int32_t block_size, mgk_precond_kind kind, const mgk_params* prm,
              void* hip_stream, mgk_solver** out) {
  if (!out) {
    mgk::g_err = "mgk_setup: null output";
    return MGK_E_INVALID;
  }
  *out = nullptr;
  std::unique_ptr<mgk_solver> S(new mgk_solver());
  return mgk::guard([&]() -> int {
    mgk::setup_impl(S.get(), A, block_size, kind, prm, hip_stream);
    *out = S.release();
    return MGK_OK;
  });
}

static int solve_common(mgk_solver* s, const double* d_b, double* d_x, double rtol,
                        mgk_info* info, bool trans) {
  if (!s || !d_b || !d_x || !info || !(rtol > 0.0)) {
    mgk::g_err = "solve: null argument or non-positive rtol";
    return MGK_E_INVALID;
  }
  if (s->batch) {
    mgk::g_err = "a batch solver only answers mgk_batch_solve";
    return MGK_E_STATE;
  }
  if (s->host_only) {
    mgk::g_err = "solve: solver was set up with mgk_setup_host (no device data)";
    return MGK_E_STATE;
  }
  if (trans && (s->kind == MGK_SCHUR || s->kind == MGK_ILU || !s->H.trans_ready)) {
    mgk::g_err = "solve_transposed needs a monolithic AMG solver set up with enable_transpose";
    return MGK_E_STATE;
  }
  return mgk::guard([&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    std::memset(info, 0, sizeof(*info));
    s->tev_used = 0;
    s->pev_used = 0;
    int rc;
    if (!trans && s->prm.krylov == MGK_FGMRES) rc = mgk::fgmres(s, d_b, d_x, rtol, info);
    else if (s->prm.krylov == MGK_IDRS) rc = mgk::idrs(s, d_b, d_x, rtol, trans, info);
    else rc = mgk::bicgstab(s, d_b, d_x, rtol, trans, info);
    HIPCK(hipStreamSynchronize(s->dev.stream));
    HIPCK(hipGetLastError());
    info->status = rc;
    info->levels = (int)s->H.lv.size();
    info->setup_ms = s->setup_ms;
    info->solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->device_bytes = s->dev.bytes;
    double spmv_ms = 0.0;
    for (size_t e = 0; e + 1 < s->tev_used; e += 2) {
      float ms = 0.0f;
      HIPCK(hipEventElapsedTime(&ms, s->tev[e], s->tev[e + 1]));
      spmv_ms += ms;
    }
    info->spmv_ms = spmv_ms;
    info->spmv_calls = (int32_t)(s->tev_used / 2);
    double pc_ms = 0.0;
    for (size_t e = 0; e + 1 < s->pev_used; e += 2) {
      float ms = 0.0f;
      HIPCK(hipEventElapsedTime(&ms, s->pev[e], s->pev[e + 1]));
      pc_ms += ms;
    }
    info->precond_ms = pc_ms;
    info->precond_calls = (int32_t)(s->pev_used / 2);
    const mgk::Tile& ot = s->A.dtile;
    info->outer_tile = 10000 * ot.rpl + 100 * ot.s + ot.u;
    info->outer_dia = s->A.dia.k;
    return rc;
  });
}

int mgk_solve(mgk_solver* s, const double* d_b, double* d_x, double rtol, mgk_info* info) {
  return solve_common(s, d_b, d_x, rtol, info, false);
}

int mgk_solve_transposed(mgk_solver* s, const double* d_g, double* d_lambda, double rtol,
                         mgk_info* info) {
  return solve_common(s, d_g, d_lambda, rtol, info, true);
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free solve

namespace mgk {

// Workspace of mgk_solve_noalloc: the eight BiCGStab vectors, the reduction partials
// (both stages) and the device scalars of one solve with at most NOALLOC_MAX_N scalar
// unknowns, in one file-scope device array (34 MiB) that every GPU the library runs
// on holds until the process ends.  Host code never uses the array's name as an
// address: each device's copy is looked up once with hipGetSymbolAddress and the
// pointer kept per device.
constexpr size_t NOALLOC_MAX_N = (size_t)1 << 19;
constexpr size_t na_round(size_t d) { return (d + 31) & ~(size_t)31; }   // 256-byte regions
// partials: two per workgroup of the fused outer SpMV (at most n / 32 for any block
// size) or MAXM per reduction workgroup, as sized by alloc_krylov for n unknowns
constexpr size_t NOALLOC_PART = na_round(NOALLOC_MAX_N / 2 + 4096);
constexpr size_t NOALLOC_PART2 = na_round(2 * (NOALLOC_PART / RED_CHUNK + 2));
constexpr size_t NOALLOC_DOUBLES =
    8 * NOALLOC_MAX_N + NOALLOC_PART + NOALLOC_PART2 + na_round(SC_COUNT);
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEV = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NOALLOC_MAX_DEV] = {};

// The device address of this device's copy of `scratch` (looked up on the first call
// per device, with that device current).
static double* scratch_ptr(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEV)
    throw Error(MGK_E_INVALID, "solve_noalloc: device ordinal out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(MGK_E_HIP, "solve_noalloc: no device address for the workspace");
    g_scratch_ptr[dev] = (double*)p;
  }
  return g_scratch_ptr[dev];
}

// Points the solver's BiCGStab workspace at the static array for the duration of one
// call and restores the solver's own buffers afterwards (also when the solve throws).
struct ScratchWorkspace {
  mgk_solver* S;
  double* saved[11];
  float* saved32[2];
  size_t saved_len;
  ScratchWorkspace(mgk_solver* s, double* base) : S(s) {
    double** f[11] = {&S->r, &S->rh, &S->p, &S->v, &S->ph, &S->s, &S->sh, &S->t,
                      &S->part, &S->part2, &S->sc};
    for (int i = 0; i < 11; ++i) saved[i] = *f[i];
    // the V-cycle reads p and s themselves (the same cycle as from their FP32 copies)
    saved32[0] = S->p32;
    saved32[1] = S->s32;
    S->p32 = S->s32 = nullptr;
    saved_len = S->part_len;
    double* q = base;
    for (int i = 0; i < 8; ++i, q += NOALLOC_MAX_N) *f[i] = q;
    S->part = q;
    q += NOALLOC_PART;
    S->part2 = q;
    q += NOALLOC_PART2;
    S->sc = q;
    S->part_len = NOALLOC_PART;
  }
  ~ScratchWorkspace() {
    double** f[11] = {&S->r, &S->rh, &S->p, &S->v, &S->ph, &S->s, &S->sh, &S->t,
                      &S->part, &S->part2, &S->sc};
    for (int i = 0; i < 11; ++i) *f[i] = saved[i];
    S->p32 = saved32[0];
    S->s32 = saved32[1];
    S->part_len = saved_len;
  }
};

}  // namespace mgk

extern "C" {

int mgk_solve_noalloc(mgk_solver* s, const double* d_b, double* d_x, double rtol,
                      mgk_info* info) {
  if (!s || !d_b || !d_x || !info || !(rtol > 0.0)) {
    mgk::g_err = "solve_noalloc: null argument or non-positive rtol";
    return MGK_E_INVALID;
  }
  if (s->batch || s->host_only) {
    mgk::g_err = "solve_noalloc: needs a single-system solver with device data";
    return MGK_E_STATE;
  }
  if (s->prm.krylov != MGK_BICGSTAB) {
    mgk::g_err = "solve_noalloc: only BiCGStab solvers (mgk_params.krylov = MGK_BICGSTAB)";
    return MGK_E_STATE;
  }
  if (s->n > mgk::NOALLOC_MAX_N) {
    mgk::g_err = "solve_noalloc: " + std::to_string(s->n) + " unknowns exceed the static "
                 "workspace limit of " + std::to_string(mgk::NOALLOC_MAX_N);
    return MGK_E_INVALID;
  }
  return mgk::guard([&]() -> int {
    int dev = -1, sdev = -1;
    HIPCK(hipGetDevice(&dev));
    HIPCK(hipStreamGetDevice(s->dev.stream, &sdev));
    if (sdev != dev)
      throw mgk::Error(MGK_E_INVALID, "solve_noalloc: the solver's stream belongs to device " +
                                          std::to_string(sdev) + ", the current device is " +
                                          std::to_string(dev));
    mgk::ScratchWorkspace ws(s, mgk::scratch_ptr(dev));
    return solve_common(s, d_b, d_x, rtol, info, false);
  });
}

int mgk_set_timing(mgk_solver* s, int32_t mask) {
  if (!s || mask < 0 || mask > 3) {
    mgk::g_err = "set_timing: null solver or mask outside 0..3";
    return MGK_E_INVALID;
  }
  s->time_mask = mask & s->prm.time_spmv;
  return MGK_OK;
}

int mgk_precond_apply(mgk_solver* s, const double* d_r, double* d_z, int32_t transposed) {
  if (!s || !d_r || !d_z) {
    mgk::g_err = "precond_apply: null argument";
    return MGK_E_INVALID;
  }
  if (s->batch) {
    mgk::g_err = "a batch solver only answers mgk_batch_solve";
    return MGK_E_STATE;
  }
  if (s->host_only) {
    mgk::g_err = "precond_apply: solver has no device data";
    return MGK_E_STATE;
  }
  if (transposed && (s->kind == MGK_SCHUR || s->kind == MGK_ILU || !s->H.trans_ready)) {
    mgk::g_err = "transposed preconditioner needs enable_transpose and a monolithic AMG";
    return MGK_E_STATE;
  }
  return mgk::guard([&]() -> int {
    mgk::precond(s, d_r, d_z, transposed != 0);
    HIPCK(hipStreamSynchronize(s->dev.stream));
    HIPCK(hipGetLastError());
    return MGK_OK;
  });
}

int mgk_spmv(mgk_solver* s, int32_t hier, int32_t level, int32_t which, const void* d_x,
             void* d_y) {
  if (!s || !d_x || !d_y || which < 0 || which > 3) {
    mgk::g_err = "spmv: bad argument";
    return MGK_E_INVALID;
  }
  if (s->batch) {
    mgk::g_err = "a batch solver only answers mgk_batch_solve";
    return MGK_E_STATE;
  }
  if (s->host_only) {
    mgk::g_err = "spmv: solver has no device data";
    return MGK_E_STATE;
  }
  return mgk::guard([&]() -> int {
    hipStream_t st = s->dev.stream;
    if (level < 0) {
      if (which != 0 && which != 3) throw mgk::Error(MGK_E_INVALID, "level -1 has only A and A^T");
      if (which == 3 && !s->A.tptr) throw mgk::Error(MGK_E_STATE, "no transpose index");
      mgk::outer_spmv(s, (const double*)d_x, (double*)d_y, which == 3);
    } else {
      mgk::DHier& H = hier == 1 ? s->Hp : s->H;
      if (hier == 1 && s->kind != MGK_SCHUR) throw mgk::Error(MGK_E_INVALID, "no pressure hierarchy");
      if (level >= (int)H.lv.size() - 1 && !(level == 0 && H.lv.size() == 1 && false))
        if (level >= (int)H.lv.size() - 1)
          throw mgk::Error(MGK_E_INVALID, "level has no stored sparse operators (coarsest)");
      mgk::DLevel& L = H.lv[level];
      const mgk::DMat& M = which == 1 ? L.P : (which == 2 ? L.R : L.A);
      const bool tr = which == 3;
      if (tr && !M.tptr) throw mgk::Error(MGK_E_STATE, "no transpose index");
      const Tile sp = which == 1 ? L.P.tile : (which == 2 ? L.R.tile : (tr ? L.A.ttile : L.A.tile));
#define MGK_LV(BB)                                                                           \
  case BB:                                                                                   \
    if (H.storage == MGK_F64)                                                                \
      mgk::spmv_s<BB, BB, double, double, double>(st, M, tr, sp, (const double*)d_x,         \
                                                   (double*)d_y, 1.0, 0.0);                  \
    else if (H.storage == MGK_F32)                                                           \
      mgk::spmv_s<BB, BB, float, float, float>(st, M, tr, sp, (const float*)d_x,             \
                                                (float*)d_y, 1.0, 0.0);                      \
    else                                                                                     \
      mgk::spmv_s<BB, BB, mgk::bf16, float, float>(st, M, tr, sp, (const float*)d_x,         \
                                                    (float*)d_y, 1.0, 0.0);                  \
    break;
      switch (H.b) {
        MGK_LV(1)
        MGK_LV(3)
        MGK_LV(4)
      }
#undef MGK_LV
    }
    HIPCK(hipGetLastError());
    return MGK_OK;
  });
}

int mgk_level_count(mgk_solver* s, int32_t hier) {
  if (!s) return MGK_E_INVALID;
  if (hier == 1 && s->kind != MGK_SCHUR) return 0;
  return (int)(hier == 1 ? s->Hp : s->H).desc.size();
}

int mgk_level_info(mgk_solver* s, int32_t hier, int32_t level, mgk_level_desc* out) {
  if (!s || !out) return MGK_E_INVALID;
  mgk::DHier& H = hier == 1 ? s->Hp : s->H;
  if (level < 0 || level >= (int)H.desc.size()) {
    mgk::g_err = "level_info: level out of range";
    return MGK_E_INVALID;
  }
  *out = H.desc[level];
  return MGK_OK;
}

int mgk_level_export(mgk_solver* s, int32_t hier, int32_t level, int32_t which, int32_t* rowptr,
                     int32_t* col, double* val, int32_t* agg) {
  if (!s) return MGK_E_INVALID;
  mgk::DHier& H = hier == 1 ? s->Hp : s->H;
  if (!H.keep_host) {
    mgk::g_err = "level_export needs keep_host = 1 at setup";
    return MGK_E_STATE;
  }
  if (level < 0 || level >= (int)H.host.levels.size() || which < 0 || which > 3) {
    mgk::g_err = "level_export: bad level or matrix";
    return MGK_E_INVALID;
  }
  const mgk::HLevel& L = H.host.levels[level];
  if (which == 3) {
    if (L.M.empty()) {
      mgk::g_err = "level_export: this level has no block-diagonal smoother";
      return MGK_E_STATE;
    }
    if (val) std::memcpy(val, L.M.data(), sizeof(double) * L.M.size());
    return MGK_OK;
  }
  const mgk::HBsr& M = which == 0 ? L.A : (which == 1 ? L.P : L.R);
  if (rowptr) std::memcpy(rowptr, M.ptr.data(), sizeof(int32_t) * M.ptr.size());
  if (col) std::memcpy(col, M.col.data(), sizeof(int32_t) * M.col.size());
  if (val) std::memcpy(val, M.val.data(), sizeof(double) * M.val.size());
  if (agg) {
    for (int32_t i = 0; i < L.A.nbr; ++i) agg[i] = L.agg.empty() ? -1 : L.agg[i];
  }
  return MGK_OK;
}

int mgk_ilu_info(mgk_solver* s, int32_t* n_brows, int64_t* l_nnzb, int64_t* u_nnzb) {
  if (!s || !n_brows || !l_nnzb || !u_nnzb) return MGK_E_INVALID;
  if (!s->ilu_kept) {
    mgk::g_err = "ilu_info needs an MGK_ILU solver set up with keep_host = 1 (or host only)";
    return MGK_E_STATE;
  }
  *n_brows = s->ilu_host.L.nbr;
  *l_nnzb = s->ilu_host.L.nnzb();
  *u_nnzb = s->ilu_host.U.nnzb();
  return MGK_OK;
}

int mgk_ilu_export(mgk_solver* s, int32_t which, int32_t* rowptr, int32_t* col, double* val) {
  if (!s || which < 0 || which > 2) return MGK_E_INVALID;
  if (!s->ilu_kept) {
    mgk::g_err = "ilu_export needs an MGK_ILU solver set up with keep_host = 1 (or host only)";
    return MGK_E_STATE;
  }
  const mgk::IluFactors& F = s->ilu_host;
  if (which == 2) {
    if (val) std::memcpy(val, F.Dinv.data(), sizeof(double) * F.Dinv.size());
    return MGK_OK;
  }
  const mgk::HBsr& M = which == 0 ? F.L : F.U;
  if (rowptr) std::memcpy(rowptr, M.ptr.data(), sizeof(int32_t) * M.ptr.size());
  if (col) std::memcpy(col, M.col.data(), sizeof(int32_t) * M.col.size());
  if (val) std::memcpy(val, M.val.data(), sizeof(double) * M.val.size());
  return MGK_OK;
}

int mgk_theta_grad(int32_t n, const double* d_lambda, const double* d_x, double* d_g,
                   void* hip_stream) {
  if (n < 3 || !d_lambda || !d_x || !d_g) {
    mgk::g_err = "theta_grad: bad argument";
    return MGK_E_INVALID;
  }
  return mgk::guard([&]() -> int {
    const size_t nc = (size_t)(n - 1) * (n - 1) * (n - 1);
    mgk::k_theta_grad<<<(unsigned)((nc + mgk::WG - 1) / mgk::WG), mgk::WG, 0,
                        (hipStream_t)hip_stream>>>(n, d_lambda, d_x, d_g);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize((hipStream_t)hip_stream));
    return MGK_OK;
  });
}

int mgk_bsr_grad(mgk_solver* s, const double* d_lambda, const double* d_x, double* d_gval) {
  if (!s || !d_lambda || !d_x || !d_gval || s->host_only || s->batch) {
    mgk::g_err = "bsr_grad: bad argument or solver without device data";
    return MGK_E_INVALID;
  }
  return mgk::guard([&]() -> int {
    hipStream_t st = s->dev.stream;
    const int b = s->b;
    const int per = mgk::WG / (b * b);
    const unsigned g = (unsigned)((s->nbr + per - 1) / per);
    if (b == 1) mgk::k_bsr_grad<1><<<g, mgk::WG, 0, st>>>(s->nbr, s->A.ptr, s->A.col, d_lambda, d_x, d_gval);
    else if (b == 3) mgk::k_bsr_grad<3><<<g, mgk::WG, 0, st>>>(s->nbr, s->A.ptr, s->A.col, d_lambda, d_x, d_gval);
    else mgk::k_bsr_grad<4><<<g, mgk::WG, 0, st>>>(s->nbr, s->A.ptr, s->A.col, d_lambda, d_x, d_gval);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(st));
    return MGK_OK;
  });
}


int mgk_setup_host(const mgk_bsr* A, int32_t block_size, mgk_precond_kind kind,
                   const mgk_params* prm, mgk_solver** out) {
  if (!out) {
    mgk::g_err = "mgk_setup_host: null output";
    return MGK_E_INVALID;
  }
  *out = nullptr;
  std::unique_ptr<mgk_solver> S(new mgk_solver());
  return mgk::guard([&]() -> int {
    mgk::setup_impl(S.get(), A, block_size, kind, prm, nullptr, true);
    *out = S.release();
    return MGK_OK;
  });
}

void mgk_destroy(mgk_solver* s) {
  if (!s) return;
  if (!s->host_only) (void)hipStreamSynchronize(s->dev.stream);
  delete s;
}

}  // extern "C"
