// C ABI of the RIDC library: handle lifetime, pipeline scheduling and batching (host side).
//
// Pipeline schedule (section III, Fig. 1 and Fig. 2; section III-E): at pipeline step s level j
// computes time index m = s - j(j+1)/2.  Level j computing t_{n+1} reads level j-1 at
// t_{max(0,n+1-j)} .. t_{max(n+1,j)}, all produced at step s-1 or earlier, so every active level
// of a step is independent and one launch (1D) or one group of launches (2D) covers them all.
// The integration takes nt + P(P-1)/2 steps, the last P(P-1)/2 being the drain of section
// III-E.  Level j < P-1 keeps its last 2j+3 values in a ring (the window level j+1 still reads
// plus the slot being written); the top level ping-pongs between 2 slots.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <mutex>

#include "ridc2d.h"
#include "ridc_internal.h"

namespace ridc {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

}  // namespace ridc

using namespace ridc;

struct ridc_handle {
  ridc_problem p{};
  hipStream_t stream = nullptr;
  int device = 0;
  int P = 1;
  int64_t npts = 0;  // unknowns (n or n*n)
  double h = 0.0;

  char* pool = nullptr;  // one device allocation holding everything below
  size_t pool_bytes = 0;
  std::vector<double*> ring;  // ring base per level
  std::vector<int> R;         // ring slots per level
  double* W = nullptr;        // weights; level j at W + woff[j] (j rows x (j+1), ascending nodes)
  std::vector<int64_t> woff;
  int* flag = nullptr;        // non-finite flag

  // state of the current integration
  int64_t nt = -1;
  int64_t sigma = 0;
  int64_t total = 0;

  // 1D plan
  PcrPlan pcr;
  int threads = 256;
  std::vector<Lvl1D> proto;   // one item per level (sigma0 = 0, nt of the armed integration)
  std::vector<Blk1D> blocks;  // blocks of a solo launch
  Lvl1D* d_items = nullptr;   // device copies (inside the pool)
  Blk1D* d_blocks = nullptr;
  Solo1D solo{};              // kernel-argument descriptor of a single-instance launch
  int solo_blocks = 0;
  // fused integration (one workgroup per instance) when the levels fit one CU's LDS
  bool fused = false;          // whole-range workgroup in use
  int fused_threads = 512;
  size_t fused_lds = 0;
  Fused1D fused_item{};
  Fused1D* d_fused = nullptr;
  size_t blocks_cap = 0;
  size_t lds = 0;

  // 2D plan
  Plan2D* p2 = nullptr;

  // IMEX levels (ridc_create_ext): pairs, orders, delays, f rings and the level-step items
  bool imex = false;
  ridc_ext ext{};
  std::vector<int> S;           // order of level j: p_0 + .. + p_j (also its window nodes)
  std::vector<int64_t> delay;   // level j computes t_m at pipeline step m + delay[j]
  std::vector<double*> ringF;   // f^S + f^N of the stored values (levels below the top)
  std::vector<ImexLvl> iproto;  // one item per level (sigma0 = 0)
  ImexLvl* d_imex = nullptr;    // device copy (inside the pool)
  int imex_M = 2, imex_T = 64;

  // graph of a whole integration, cached per nt
  hipGraphExec_t gexec = nullptr;
  int64_t graph_nt = -1;
};

namespace {

bool env_flag(const char* name, bool dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return !(v[0] == '0' || v[0] == 'n' || v[0] == 'N' || v[0] == 'f' || v[0] == 'F');
}

int validate(const ridc_problem* p) {
  if (!p) return fail(RIDC_E_INVAL, "problem is NULL");
  if (p->dim != 1 && p->dim != 2) return fail(RIDC_E_INVAL, "dim must be 1 or 2");
  if (p->bc != RIDC_BC_PERIODIC && p->bc != RIDC_BC_DIRICHLET0)
    return fail(RIDC_E_INVAL, "unknown boundary condition");
  if (p->n < 2) return fail(RIDC_E_INVAL, "n must be >= 2");
  if (!(p->length > 0.0) || !std::isfinite(p->length))
    return fail(RIDC_E_INVAL, "length must be > 0");
  if (p->order < 1 || p->order > RIDC_MAX_ORDER)
    return fail(RIDC_E_INVAL, "order must be in 1..12");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(RIDC_E_INVAL, "dt must be > 0");
  if (!(p->nu >= 0.0) || !std::isfinite(p->nu)) return fail(RIDC_E_INVAL, "nu must be >= 0");
  if (!std::isfinite(p->a)) return fail(RIDC_E_INVAL, "a must be finite");
  if (p->fe_kind < RIDC_FE_NONE || p->fe_kind > RIDC_FE_BURGERS)
    return fail(RIDC_E_INVAL, "unknown explicit term");
  if (p->prec < RIDC_PREC_FP64 || p->prec > RIDC_PREC_BF16X3_REFINE)
    return fail(RIDC_E_INVAL, "unknown precision");
  if (p->reserved != 0) return fail(RIDC_E_INVAL, "reserved must be 0");
  if (p->dim == 2) {
    if (p->bc != RIDC_BC_DIRICHLET0)
      return fail(RIDC_E_UNSUPPORTED, "2D supports Dirichlet boundaries only");
    if (p->fe_kind != RIDC_FE_NONE && p->fe_kind != RIDC_FE_LOGISTIC)
      return fail(RIDC_E_UNSUPPORTED, "2D provides pointwise explicit terms only");
    return plan2d_validate(p);
  }
  if (p->prec != RIDC_PREC_FP64) return fail(RIDC_E_UNSUPPORTED, "1D computes in FP64 only");
  if (p->n > (1 << 28)) return fail(RIDC_E_UNSUPPORTED, "1D n above 2^28");
  return RIDC_OK;
}

double grid_h(const ridc_problem* p) {
  return p->bc == RIDC_BC_PERIODIC ? p->length / (double)p->n : p->length / (double)(p->n + 1);
}

int device_max_lds() {
  static int cached = -1;
  if (cached < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      cached = v;
    else
      cached = 65536;
  }
  return cached;
}

// ---------------------------------------------------------------------------------------------
// 1D tiling (result-neutral: every tiling performs the same operations for every output row)
// ---------------------------------------------------------------------------------------------
struct Tile1D {
  int wrap = 1;
  int B = 0;
  int threads = 256;
  int nt_store = 0;   // write new level values with nontemporal stores
  int fused = 0;      // 0: one launch per pipeline step; 512/1024: whole-range workgroup threads
};

std::mutex g_tune_mu;

// Tiling of grouped 1D launches (process-wide, guarded by g_tune_mu): threads per workgroup and
// the most LDS rows one workgroup holds (0: whole cycles whenever they fit).  Until it is set or
// measured, a tiling recorded in the tuning cache applies.
struct BatchTile {
  int threads = 256;
  int rows = 0;
};
BatchTile g_batch_tile;
bool g_batch_tile_set = false;

BatchTile current_batch_tile() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_batch_tile_set) {
    int t = 0, r = 0;
    if (tune_get_batch(&t, &r)) g_batch_tile = BatchTile{t, r};
    g_batch_tile_set = true;
  }
  return g_batch_tile;
}

// ridc_set_tile's (threads, rows, flags) as a tiling, and back
Tile1D tile_from(int threads, int rows, int flags) {
  if (flags & 2) return Tile1D{1, 0, 256, 0, threads};
  return Tile1D{rows == 0 ? 1 : 0, rows, threads, flags & 1, 0};
}
void tile_to(const Tile1D& t, int* threads, int* rows, int* flags) {
  *threads = t.fused ? t.fused : t.threads;
  *rows = t.wrap ? 0 : t.B;
  *flags = t.nt_store | (t.fused ? 2 : 0);
}

// the measured tiling of this system, if the tuning table has one
bool tuned_tile(int64_t n, int bc, int stages, Tile1D* t) {
  int th = 0, r = 0, f = 0;
  if (!tune_get_1d(n, bc, stages, &th, &r, &f)) return false;
  *t = tile_from(th, r, f);
  return true;
}

int64_t halo_rows(const PcrPlan& pcr) {
  return pcr.stages < 30 ? ((int64_t)1 << pcr.stages) - 1 : ((int64_t)1 << 40);
}

// Fused integration plan: P level groups of G threads (whole waves) in one workgroup of 1024,
// two LDS buffers per level holding the whole cycle.
struct FusedPlan {
  bool ok = false, db = false;
  int group = 0, rpt = 0;
  size_t lds = 0;
};

FusedPlan plan_fused(const ridc_problem* p, int threads) {
  FusedPlan f;
  if (p->dim != 1 || p->order > kMaxJ1024 + 1) return f;
  if (threads == 1024 && p->order > 4) return f;   // the 1024-thread kernel covers orders <= 4
  const int P = p->order;
  const int64_t ms = p->bc == RIDC_BC_PERIODIC ? p->n : p->n + 2;
  const size_t maxl = (size_t)device_max_lds();
  const int G = (threads / P) / 64 * 64;
  if (G >= 64 && (size_t)P * 2 * ms * sizeof(double) <= maxl) {
    f.ok = f.db = true;
    f.group = G;
    f.lds = (size_t)P * 2 * ms * sizeof(double);
  }
  return f;
}

bool tile_fits(const ridc_problem* p, const PcrPlan& pcr, const Tile1D& t) {
  if (t.fused) return (t.fused == 512 || t.fused == 1024) && plan_fused(p, t.fused).ok;
  const int64_t M = p->bc == RIDC_BC_PERIODIC ? p->n : 2 * p->n + 2;
  const int64_t ms = p->bc == RIDC_BC_PERIODIC ? p->n : p->n + 2;
  if (t.threads != 64 && t.threads != 128 && t.threads != 256 && t.threads != 512 &&
      t.threads != 1024)
    return false;
  if (t.threads == 1024 && p->order > kMaxJ1024 + 1) return false;
  if (t.wrap) return 2 * sizeof(double) * (size_t)ms <= (size_t)device_max_lds();
  const int64_t H = halo_rows(pcr);
  if (pcr.exact || H >= M || t.B < 1 || t.B + H > p->n) return false;
  return 2 * sizeof(double) * (size_t)(t.B + 2 * H) <= (size_t)device_max_lds();
}

// allow_fused: a tuned whole-range workgroup may be chosen (otherwise one launch per step)
int choose_tile_1d(const ridc_problem* p, const PcrPlan& pcr, Tile1D* out,
                   bool allow_fused = true) {
  Tile1D t;
  if (tuned_tile(p->n, p->bc, pcr.stages, &t) && (allow_fused || !t.fused) &&
      tile_fits(p, pcr, t)) {
    *out = t;
    return RIDC_OK;
  }
  const int64_t H = halo_rows(pcr);
  // default for long systems with a short PCR halo: chunks, as many as give about 256
  // workgroups per step over the levels (one per CU: a single system's step is bound by
  // latency, not bytes), at least 128 rows each, 1024 threads where the order allows
  // (measured at n = 8192, order 4: 128-row chunks of 1024 threads run a step in 5.3 us,
  // 1024-row chunks of 256 threads in 10.8).  The whole-range workgroup is left to
  // measurement: ridc_autotune, ridc_set_tile.
  if (p->n >= 2048 && H <= 512) {
    const int64_t per_level = std::max<int64_t>(1, 256 / p->order);
    int64_t B = (p->n / per_level) / 64 * 64;
    B = std::min<int64_t>(1024, std::max<int64_t>(128, B));
    const int threads = p->order <= kMaxJ1024 + 1 ? 1024 : 256;
    Tile1D chunk{0, (int)B, threads};
    if (tile_fits(p, pcr, chunk)) {
      *out = chunk;
      return RIDC_OK;
    }
  }
  Tile1D chunk{0, 1024, 256};
  Tile1D wrap{1, 0, 256};
  if (tile_fits(p, pcr, wrap)) {
    *out = wrap;
    return RIDC_OK;
  }
  if (tile_fits(p, pcr, chunk)) {
    *out = chunk;
    return RIDC_OK;
  }
  return fail(RIDC_E_UNSUPPORTED, "1D system does not fit one workgroup's LDS");
}

int plan_1d(const ridc_problem* p, PcrPlan* pcr, Tile1D* tile) {
  const double h = grid_h(p);
  const double r = p->dt * p->nu / (h * h);
  const int64_t M = p->bc == RIDC_BC_PERIODIC ? p->n : 2 * p->n + 2;
  if (!pcr_plan(r, M, pcr))
    return fail(RIDC_E_UNSUPPORTED, "PCR did not converge within the stage cap");
  return choose_tile_1d(p, *pcr, tile);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kMinChunk = 128;

struct Layout {
  size_t rings = 0, weights = 0, flag = 0, items = 0, blocks = 0, ws2d = 0, total = 0;
  int64_t nblocks = 0;
};

void plan_layout(const ridc_problem* p, const Tile1D* tile, Layout* L) {
  const int P = p->order;
  const int64_t npts = p->dim == 1 ? p->n : p->n * p->n;
  int64_t slots = 0;
  for (int j = 0; j < P; ++j) slots += ring_slots(j, P);
  L->rings = align256(sizeof(double) * (size_t)(slots * npts));
  int64_t nw = 0;
  for (int j = 1; j < P; ++j) nw += (int64_t)j * (j + 1);
  L->weights = align256(sizeof(double) * (size_t)std::max<int64_t>(nw, 1));
  L->flag = 256;
  if (p->dim == 1) {
    // room for the finest tiling the autotuner may pick (chunks of kMinChunk rows)
    const int64_t nchunks = std::max<int64_t>(tile->wrap ? 1 : (p->n + tile->B - 1) / tile->B,
                                              (p->n + kMinChunk - 1) / kMinChunk);
    L->nblocks = nchunks * P;
    L->items = align256(sizeof(Lvl1D) * P) + align256(sizeof(Fused1D));
    L->blocks = align256(sizeof(Blk1D) * (size_t)L->nblocks);
  } else {
    L->ws2d = align256(plan2d_workspace_bytes(p));
  }
  L->total = L->rings + L->weights + L->flag + L->items + L->blocks + L->ws2d;
}

// Kernel-argument descriptor of a single instance's level step (k_step1d_solo): level rings and
// their slot counts, per-level weight tables (W[0] unused), the device PCR tables, the tiling.
void fill_solo(const ridc_problem& p, double h, const PcrPlan& pcr, const Tile1D& tile,
               double* const* ring, const int* R, const double* const* W, const double* gamma,
               const int32_t* shift, int64_t nt, Solo1D* out) {
  Solo1D a{};
  for (int j = 0; j < p.order; ++j) {
    a.ring[j] = ring[j];
    a.W[j] = j > 0 ? W[j] : nullptr;
    a.R[j] = R[j];
  }
  a.gamma = gamma;
  a.shift = shift;
  a.nt = nt;
  a.nchunks = tile.wrap ? 1 : (int)((p.n + tile.B - 1) / tile.B);
  a.n = (int32_t)p.n;
  a.M = (int32_t)(p.bc == RIDC_BC_PERIODIC ? p.n : 2 * p.n + 2);
  a.bc = p.bc;
  a.fe = p.fe_kind;
  a.stages = pcr.stages;
  a.wrap = tile.wrap;
  a.B = tile.wrap ? 0 : tile.B;
  a.H = tile.wrap ? 0 : (int)halo_rows(pcr);
  a.nt_store = tile.nt_store;
  a.dt = p.dt;
  a.ce = explicit_coeff(p.fe_kind, p.a, h);
  a.nu_h2 = p.nu / (h * h);
  a.inv_divisor = 1.0 / pcr.divisor;
  *out = a;
}

void build_items_1d(ridc_handle* h, const Tile1D& tile) {
  const ridc_problem& p = h->p;
  const int P = h->P;
  h->proto.assign(P, Lvl1D{});
  const int64_t M = p.bc == RIDC_BC_PERIODIC ? p.n : 2 * p.n + 2;
  const int H = tile.wrap ? 0 : (int)halo_rows(h->pcr);
  const int nchunks = tile.wrap ? 1 : (int)((p.n + tile.B - 1) / tile.B);
  for (int j = 0; j < P; ++j) {
    Lvl1D& it = h->proto[j];
    it.own = h->ring[j];
    it.prev = j > 0 ? h->ring[j - 1] : nullptr;
    it.W = j > 0 ? h->W + h->woff[j] : nullptr;
    it.nt = 0;
    it.sigma0 = 0;
    it.n = (int32_t)p.n;
    it.j = j;
    it.R_own = h->R[j];
    it.R_prev = j > 0 ? h->R[j - 1] : 1;
    it.bc = p.bc;
    it.fe = p.fe_kind;
    it.stages = h->pcr.stages;
    it.wrap = tile.wrap;
    it.M = (int32_t)M;
    it.B = tile.wrap ? 0 : tile.B;
    it.H = H;
    it.nchunks = nchunks;
    it.dt = p.dt;
    it.ce = explicit_coeff(p.fe_kind, p.a, h->h);
    it.nu_h2 = p.nu / (h->h * h->h);
    it.inv_divisor = 1.0 / h->pcr.divisor;
    for (int k = 0; k < h->pcr.stages; ++k) {
      it.gamma[k] = h->pcr.gamma[k];
      it.shift[k] = (int32_t)h->pcr.shift[k];
    }
  }
  h->blocks.clear();
  for (int j = 0; j < P; ++j)
    for (int c = 0; c < nchunks; ++c) h->blocks.push_back(Blk1D{j, c});
  size_t lds = 0;
  for (auto& it : h->proto) lds = std::max(lds, lds_bytes_1d(it));
  h->lds = lds;
  h->threads = tile.threads;
  (void)prepare_1d_step(h->threads, P, h->lds);
  std::vector<const double*> W(P, nullptr);
  for (int j = 1; j < P; ++j) W[j] = h->W + h->woff[j];
  fill_solo(p, h->h, h->pcr, tile, h->ring.data(), h->R.data(), W.data(),
            (const double*)((const char*)h->d_items + offsetof(Lvl1D, gamma)),
            (const int32_t*)((const char*)h->d_items + offsetof(Lvl1D, shift)),
            h->nt < 0 ? 0 : h->nt, &h->solo);
  h->solo_blocks = P * nchunks;
}

// Grouped launch tables for ridc_advance over several 1D handles (one set per thread and
// device).  Two events guard their reuse: `done` follows the upload of the pinned staging copy
// (the host waits for it before rewriting the staging), and `used` follows the last launch that
// read the device tables (an upload on another stream waits for it on the device, so that the
// tables are never rewritten under a kernel still reading them).
struct BatchArena {
  int device = -1;
  Lvl1D* d_items = nullptr;
  Blk1D* d_blocks = nullptr;
  size_t cap_items = 0, cap_blocks = 0;
  Lvl1D* h_items = nullptr;
  Blk1D* h_blocks = nullptr;
  Fused1D* d_fused = nullptr;
  Fused1D* h_fused = nullptr;
  size_t cap_fused = 0;
  CopyItem* d_copy = nullptr;
  CopyItem* h_copy = nullptr;
  size_t cap_copy = 0;
  ImexLvl* d_imex = nullptr;
  ImexLvl* h_imex = nullptr;
  size_t cap_imex = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  hipEvent_t used = nullptr;
  hipStream_t used_stream = nullptr;
  bool in_use = false;
};

thread_local BatchArena g_arena;

// Mark the tables as read by work enqueued on `stream` so far (call after the launches).
int arena_release(hipStream_t stream) {
  RIDC_HIP_TRY(hipEventRecord(g_arena.used, stream));
  g_arena.used_stream = stream;
  g_arena.in_use = true;
  return RIDC_OK;
}

// Before a table is freed for a larger one: every launch reading it has finished.
int arena_drain() {
  if (g_arena.in_use) RIDC_HIP_TRY(hipEventSynchronize(g_arena.used));
  g_arena.in_use = false;
  return RIDC_OK;
}

int arena_reserve_fused(size_t n) {
  // called after arena_reserve (device, events and pending upload handled there)
  if (n > g_arena.cap_fused) {
    int rc = arena_drain();
    if (rc != RIDC_OK) return rc;
    if (g_arena.d_fused) (void)hipFree(g_arena.d_fused);
    if (g_arena.h_fused) (void)hipHostFree(g_arena.h_fused);
    g_arena.d_fused = nullptr;
    g_arena.h_fused = nullptr;
    const size_t cap = std::max<size_t>(n, 2 * g_arena.cap_fused);
    if (hipMalloc(&g_arena.d_fused, cap * sizeof(Fused1D)) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch fused table");
    if (hipHostMalloc(&g_arena.h_fused, cap * sizeof(Fused1D), hipHostMallocDefault) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch fused staging");
    g_arena.cap_fused = cap;
  }
  return RIDC_OK;
}

int arena_reserve_imex(size_t n) {
  // called after arena_reserve (device, events and pending upload handled there)
  if (n > g_arena.cap_imex) {
    int rc = arena_drain();
    if (rc != RIDC_OK) return rc;
    if (g_arena.d_imex) (void)hipFree(g_arena.d_imex);
    if (g_arena.h_imex) (void)hipHostFree(g_arena.h_imex);
    g_arena.d_imex = nullptr;
    g_arena.h_imex = nullptr;
    const size_t cap = std::max<size_t>(n, 2 * g_arena.cap_imex);
    if (hipMalloc(&g_arena.d_imex, cap * sizeof(ImexLvl)) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch IMEX table");
    if (hipHostMalloc(&g_arena.h_imex, cap * sizeof(ImexLvl), hipHostMallocDefault) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch IMEX staging");
    g_arena.cap_imex = cap;
  }
  return RIDC_OK;
}

// Make the tables (at least nitems items and nblocks blocks) ready for an upload on `stream`.
int arena_reserve(size_t nitems, size_t nblocks, hipStream_t stream) {
  int dev = 0;
  RIDC_HIP_TRY(hipGetDevice(&dev));
  if (g_arena.device != dev) {
    g_arena = BatchArena{};  // tables of another device are left to process teardown
    g_arena.device = dev;
  }
  if (!g_arena.done) RIDC_HIP_TRY(hipEventCreateWithFlags(&g_arena.done, hipEventDisableTiming));
  if (!g_arena.used) RIDC_HIP_TRY(hipEventCreateWithFlags(&g_arena.used, hipEventDisableTiming));
  if (g_arena.pending) {
    RIDC_HIP_TRY(hipEventSynchronize(g_arena.done));
    g_arena.pending = false;
  }
  // launches of another stream may still read the tables this upload overwrites
  if (g_arena.in_use && g_arena.used_stream != stream)
    RIDC_HIP_TRY(hipStreamWaitEvent(stream, g_arena.used, 0));
  if ((nitems > g_arena.cap_items || nblocks > g_arena.cap_blocks) && arena_drain() != RIDC_OK)
    return RIDC_E_HIP;
  if (nitems > g_arena.cap_items) {
    if (g_arena.d_items) (void)hipFree(g_arena.d_items);
    if (g_arena.h_items) (void)hipHostFree(g_arena.h_items);
    g_arena.d_items = nullptr;
    g_arena.h_items = nullptr;
    const size_t cap = std::max<size_t>(nitems, 2 * g_arena.cap_items);
    if (hipMalloc(&g_arena.d_items, cap * sizeof(Lvl1D)) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch item table");
    if (hipHostMalloc(&g_arena.h_items, cap * sizeof(Lvl1D), hipHostMallocDefault) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch item staging");
    g_arena.cap_items = cap;
  }
  if (nblocks > g_arena.cap_blocks) {
    if (g_arena.d_blocks) (void)hipFree(g_arena.d_blocks);
    if (g_arena.h_blocks) (void)hipHostFree(g_arena.h_blocks);
    g_arena.d_blocks = nullptr;
    g_arena.h_blocks = nullptr;
    const size_t cap = std::max<size_t>(nblocks, 2 * g_arena.cap_blocks);
    if (hipMalloc(&g_arena.d_blocks, cap * sizeof(Blk1D)) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch block table");
    if (hipHostMalloc(&g_arena.h_blocks, cap * sizeof(Blk1D), hipHostMallocDefault) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch block staging");
    g_arena.cap_blocks = cap;
  }
  return RIDC_OK;
}

int64_t pipeline_steps(int64_t nt, int P) { return nt > 0 ? nt + (int64_t)P * (P - 1) / 2 : 0; }

// Pipeline steps of an integration of nt steps on this handle, and the first step at which
// every level is active.
int64_t handle_steps(const ridc_handle* h, int64_t nt) {
  if (h->imex) return nt > 0 ? nt + h->delay[h->P - 1] : 0;
  return pipeline_steps(nt, h->P);
}
int64_t first_full_step(const ridc_handle* h) {
  return h->imex ? h->delay[h->P - 1] + 1 : (int64_t)h->P * (h->P - 1) / 2 + 1;
}

// IMEX handles: the first launch of an integration also writes f of every level's initial
// value (the windows' node t_0).
int launch_imex_steps(ridc_handle* h, int64_t first, int64_t last) {
  const bool per = h->p.bc == RIDC_BC_PERIODIC;
  if (first == 1)
    RIDC_HIP_TRY(launch_imex1d(h->d_imex, h->P, h->imex_M, h->imex_T, per, 0, true, h->stream));
  for (int64_t s = first; s <= last; ++s)
    RIDC_HIP_TRY(launch_imex1d(h->d_imex, h->P, h->imex_M, h->imex_T, per, s, false,
                               h->stream));
  return RIDC_OK;
}

// The step count travels in the kernel arguments (single instance) or in the batch tables, so
// arming a 1D handle touches host state only; the device item copy holds the PCR coefficients.
void arm_solo_items(ridc_handle* h) {
  h->solo.nt = h->nt;
  for (auto& it : h->proto) it.nt = h->nt;
}

int launch_solo_steps_1d(ridc_handle* h, int64_t first, int64_t last) {
  for (int64_t s = first; s <= last; ++s)
    RIDC_HIP_TRY(launch_1d_solo(h->solo, h->solo_blocks, h->threads, h->P, h->lds, s,
                                h->stream));
  return RIDC_OK;
}

// Pipeline steps first..last of one handle in one fused launch.
int launch_fused_steps(ridc_handle* h, int64_t first, int64_t last) {
  Fused1D F = h->fused_item;
  F.nt = h->nt;
  F.sigma0 = 0;
  F.sigma_first = first - 1;
  F.sigma_last = last;
  RIDC_HIP_TRY(launch_fused_1d(nullptr, &F, 1, h->P, h->fused_threads, h->fused_lds, h->stream));
  return RIDC_OK;
}

int run_solo_steps(ridc_handle* h, int64_t first, int64_t last) {
  if (h->imex) return launch_imex_steps(h, first, last);
  if (h->p.dim == 1 && h->fused) return launch_fused_steps(h, first, last);
  if (h->p.dim == 1) return launch_solo_steps_1d(h, first, last);
  Plan2D* pl = h->p2;
  const int64_t before = first - 1;
  return plan2d_advance(&pl, 1, &before, last - first + 1, h->stream);
}

int check_handles(ridc_handle* const* hs, int32_t count) {
  if (count < 0 || (count > 0 && !hs)) return fail(RIDC_E_INVAL, "bad handle list");
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i]) return fail(RIDC_E_INVAL, "NULL handle in list");
    if (hs[i]->stream != hs[0]->stream)
      return fail(RIDC_E_INVAL, "batched handles must share one stream");
  }
  return RIDC_OK;
}

int apply_tile_1d(ridc_handle* h, const Tile1D& t) {
  if (!tile_fits(&h->p, h->pcr, t)) return fail(RIDC_E_INVAL, "tile does not fit this system");
  if (t.fused) {
    const FusedPlan fp = plan_fused(&h->p, t.fused);
    h->fused = true;
    h->fused_threads = t.fused;
    h->fused_lds = fp.lds;
    h->fused_item.group = fp.group;
    if (h->gexec) {
      (void)hipGraphExecDestroy(h->gexec);
      h->gexec = nullptr;
    }
    h->graph_nt = -1;
    return RIDC_OK;
  }
  h->fused = false;
  const size_t nchunks = t.wrap ? 1 : (size_t)((h->p.n + t.B - 1) / t.B);
  if (nchunks * h->P > h->blocks_cap) return fail(RIDC_E_INVAL, "tile finer than the minimum chunk");
  build_items_1d(h, t);
  h->solo.nt = h->nt < 0 ? 0 : h->nt;
  RIDC_HIP_TRY(hipMemcpyAsync(h->d_blocks, h->blocks.data(), sizeof(Blk1D) * h->blocks.size(),
                              hipMemcpyHostToDevice, h->stream));
  for (auto& it : h->proto) it.nt = h->nt < 0 ? 0 : h->nt;
  RIDC_HIP_TRY(hipMemcpyAsync(h->d_items, h->proto.data(), sizeof(Lvl1D) * h->proto.size(),
                              hipMemcpyHostToDevice, h->stream));
  RIDC_HIP_TRY(hipStreamSynchronize(h->stream));   // the host tables are rebuilt by later calls
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  h->graph_nt = -1;
  return RIDC_OK;
}

// Time `reps` steady-state steps of the handle with tile t (the rings hold zeros).
int time_tile_1d(ridc_handle* h, const Tile1D& t, int reps, float* ms) {
  int rc = apply_tile_1d(h, t);
  if (rc != RIDC_OK) return rc;
  if (t.fused) {
    const int64_t saved = h->nt;
    h->nt = (int64_t)1 << 40;
    const int64_t first = (int64_t)h->P * (h->P - 1) / 2 + 1;
    hipEvent_t a, b;
    RIDC_HIP_TRY(hipEventCreate(&a));
    RIDC_HIP_TRY(hipEventCreate(&b));
    rc = launch_fused_steps(h, first, first + 4);                // warm-up
    if (rc == RIDC_OK) {
      (void)hipEventRecord(a, h->stream);
      rc = launch_fused_steps(h, first + 5, first + 4 + reps);
      (void)hipEventRecord(b, h->stream);
    }
    if (rc == RIDC_OK && hipEventSynchronize(b) == hipSuccess) (void)hipEventElapsedTime(ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    h->nt = saved;
    return rc;
  }
  for (auto& it : h->proto) it.nt = (int64_t)1 << 40;
  h->solo.nt = (int64_t)1 << 40;
  RIDC_HIP_TRY(hipMemcpyAsync(h->d_items, h->proto.data(), sizeof(Lvl1D) * h->proto.size(),
                              hipMemcpyHostToDevice, h->stream));
  hipEvent_t a, b;
  RIDC_HIP_TRY(hipEventCreate(&a));
  RIDC_HIP_TRY(hipEventCreate(&b));
  const int64_t first = (int64_t)h->P * (h->P - 1) / 2 + 1;   // every level active
  rc = launch_solo_steps_1d(h, first, first + 4);               // warm-up
  if (rc == RIDC_OK) {
    (void)hipEventRecord(a, h->stream);
    rc = launch_solo_steps_1d(h, first + 5, first + 4 + reps);
    (void)hipEventRecord(b, h->stream);
  }
  if (rc == RIDC_OK && hipEventSynchronize(b) == hipSuccess) (void)hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

// Tiling of a grouped 1D launch: every system of the batch shares the thread count; a system
// whose stored cycle has more than `rows` rows (rows > 0) is cut into chunks of at most `rows`
// LDS rows including halos.  Tilings do not change results.
Tile1D batch_tile_for(const ridc_handle* h, const BatchTile& bt, int threads) {
  const ridc_problem& p = h->p;
  const int64_t ms = p.bc == RIDC_BC_PERIODIC ? p.n : p.n + 2;
  const Tile1D wrap{1, 0, threads};
  const bool wrap_ok = tile_fits(&p, h->pcr, wrap);
  if (wrap_ok && (bt.rows <= 0 || ms <= bt.rows)) return wrap;
  const int64_t H = halo_rows(h->pcr);
  if (bt.rows > 0 && bt.rows > 2 * H) {
    const int64_t B = (bt.rows - 2 * H) / 64 * 64;
    const Tile1D c{0, (int)std::min<int64_t>(B, 1 << 20), threads};
    if (B >= 64 && tile_fits(&p, h->pcr, c)) return c;
  }
  if (wrap_ok) return wrap;
  for (int B : {4096, 2048, 1024, 512, 256, kMinChunk}) {
    const Tile1D c{0, B, threads};
    if (tile_fits(&p, h->pcr, c)) return c;
  }
  return Tile1D{-1, 0, threads};
}

struct BatchStage {
  int nblocks = 0, threads = 256, maxP = 1;
  size_t lds = 0;
};

// Fill and upload the item and block tables of one grouped launch over the 1D handles hs.
// Normal use: each handle's own step = launch step + its current sigma.  timing: every level
// active from its start-up step on and never finishing (the rings are scratch).
int stage_batch_1d(const std::vector<ridc_handle*>& hs, const BatchTile& bt, bool timing,
                   hipStream_t stream, BatchStage* out) {
  BatchStage st;
  for (auto* h : hs) st.maxP = std::max(st.maxP, h->P);
  st.threads = bt.threads;
  if (st.threads == 1024 && st.maxP > kMaxJ1024 + 1) st.threads = 512;
  std::vector<Tile1D> tiles(hs.size());
  size_t nitems = 0, nblocks = 0;
  for (size_t i = 0; i < hs.size(); ++i) {
    tiles[i] = batch_tile_for(hs[i], bt, st.threads);
    if (tiles[i].wrap < 0) return fail(RIDC_E_UNSUPPORTED, "no batch tiling fits a system");
    const int64_t nch = tiles[i].wrap ? 1 : (hs[i]->p.n + tiles[i].B - 1) / tiles[i].B;
    nitems += hs[i]->P;
    nblocks += (size_t)(nch * hs[i]->P);
  }
  int rc = arena_reserve(nitems, nblocks, stream);
  if (rc != RIDC_OK) return rc;
  std::vector<std::pair<int64_t, Blk1D>> order;
  order.reserve(nblocks);
  size_t ii = 0;
  for (size_t i = 0; i < hs.size(); ++i) {
    ridc_handle* h = hs[i];
    const Tile1D& t = tiles[i];
    const int64_t H = t.wrap ? 0 : halo_rows(h->pcr);
    const int nch = t.wrap ? 1 : (int)((h->p.n + t.B - 1) / t.B);
    const int64_t ms = h->p.bc == RIDC_BC_PERIODIC ? h->p.n : h->p.n + 2;
    const int64_t rows = t.wrap ? ms : t.B + 2 * H;
    for (int j = 0; j < h->P; ++j) {
      Lvl1D it = h->proto[j];
      it.nt = timing ? ((int64_t)1 << 40) : h->nt;
      it.sigma0 = timing ? 0 : -h->sigma;
      it.wrap = t.wrap;
      it.B = t.wrap ? 0 : t.B;
      it.H = (int32_t)H;
      it.nchunks = nch;
      g_arena.h_items[ii + j] = it;
      st.lds = std::max(st.lds, lds_bytes_1d(it));
      for (int c = 0; c < nch; ++c) order.push_back({rows, Blk1D{(int32_t)(ii + j), c}});
    }
    ii += h->P;
  }
  // the longest workgroups first
  std::stable_sort(order.begin(), order.end(),
                   [](const auto& a, const auto& b) { return a.first > b.first; });
  for (size_t b = 0; b < order.size(); ++b) g_arena.h_blocks[b] = order[b].second;
  st.nblocks = (int)order.size();
  RIDC_HIP_TRY(prepare_1d_step(st.threads, st.maxP, st.lds));
  RIDC_HIP_TRY(hipMemcpyAsync(g_arena.d_items, g_arena.h_items, sizeof(Lvl1D) * nitems,
                              hipMemcpyHostToDevice, stream));
  RIDC_HIP_TRY(hipMemcpyAsync(g_arena.d_blocks, g_arena.h_blocks, sizeof(Blk1D) * order.size(),
                              hipMemcpyHostToDevice, stream));
  RIDC_HIP_TRY(hipEventRecord(g_arena.done, stream));
  g_arena.pending = true;
  *out = st;
  return RIDC_OK;
}

// Validate and arm a handle for nsteps time steps (host state and 2D plan; the rings are
// filled by the caller).
int arm_handle(ridc_handle* h, const double* u0_dev, int64_t nsteps) {
  if (!h || !u0_dev) return fail(RIDC_E_INVAL, "NULL handle or u0");
  if (nsteps < 0) return fail(RIDC_E_INVAL, "nsteps must be >= 0");
  const int64_t least = h->imex ? (h->P > 1 ? h->S[h->P - 1] - 1 : 0) : h->P - 1;
  if (nsteps > 0 && nsteps < least)
    return fail(RIDC_E_INVAL, "nsteps must be 0 or at least the start-up window of the top "
                "corrector (order-1 nodes)");
  h->nt = nsteps;
  h->sigma = 0;
  h->total = handle_steps(h, nsteps);
  if (h->imex) {
    for (auto& it : h->iproto) it.nt = nsteps;
    RIDC_HIP_TRY(hipMemcpyAsync(h->d_imex, h->iproto.data(), sizeof(ImexLvl) * h->P,
                                hipMemcpyHostToDevice, h->stream));
    // the host items are rewritten by the next arm: wait for this upload
    RIDC_HIP_TRY(hipStreamSynchronize(h->stream));
    return RIDC_OK;
  }
  if (h->p.dim == 1) {
    arm_solo_items(h);
    return RIDC_OK;
  }
  return plan2d_arm(h->p2, nsteps, h->stream);
}

// Run a list of vector copies (optionally checking the copied values), the list going through
// the batch arena's pinned staging; one launch per 65535 items (the grid's y extent).
int stage_copies(const std::vector<CopyItem>& c, hipStream_t stream) {
  if (c.empty()) return RIDC_OK;
  int rc = arena_reserve(0, 0, stream);
  if (rc != RIDC_OK) return rc;
  if (c.size() > g_arena.cap_copy) {
    rc = arena_drain();
    if (rc != RIDC_OK) return rc;
    if (g_arena.d_copy) (void)hipFree(g_arena.d_copy);
    if (g_arena.h_copy) (void)hipHostFree(g_arena.h_copy);
    g_arena.d_copy = nullptr;
    g_arena.h_copy = nullptr;
    const size_t cap = std::max<size_t>(c.size(), 2 * g_arena.cap_copy);
    if (hipMalloc(&g_arena.d_copy, cap * sizeof(CopyItem)) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch copy table");
    if (hipHostMalloc(&g_arena.h_copy, cap * sizeof(CopyItem), hipHostMallocDefault) != hipSuccess)
      return fail(RIDC_E_NOMEM, "batch copy staging");
    g_arena.cap_copy = cap;
  }
  int64_t most = 0;
  for (size_t i = 0; i < c.size(); ++i) {
    g_arena.h_copy[i] = c[i];
    most = std::max(most, c[i].n);
  }
  RIDC_HIP_TRY(hipMemcpyAsync(g_arena.d_copy, g_arena.h_copy, sizeof(CopyItem) * c.size(),
                              hipMemcpyHostToDevice, stream));
  RIDC_HIP_TRY(hipEventRecord(g_arena.done, stream));
  g_arena.pending = true;
  for (size_t off = 0; off < c.size(); off += 65535) {
    const int cnt = (int)std::min<size_t>(65535, c.size() - off);
    RIDC_HIP_TRY(launch_copy_items(g_arena.d_copy + off, cnt, most, stream));
  }
  return arena_release(stream);
}

// ---------------------------------------------------------------------------------------------
// IMEX levels (ridc_create_ext): Thm 2's ARK-based RIDC and Newton for a nonlinear stiff term
// ---------------------------------------------------------------------------------------------
struct ImexPlan {
  std::vector<ImexPair> pair;   // per level
  std::vector<int> S;           // order of level j = window nodes of corrector j
  std::vector<int64_t> delay;
  std::vector<int> R;           // ring slots of the values (and of f, below the top)
  size_t rings = 0, frings = 0, weights = 0, work = 0, items = 0, total = 0;
  int M = 2, T = 64;
};

int validate_ext(const ridc_problem* p, const ridc_ext* e, ImexPlan* out) {
  int rc = validate(p);
  if (rc != RIDC_OK) return rc;
  if (!e) return fail(RIDC_E_INVAL, "ext is NULL");
  if (p->dim != 1) return fail(RIDC_E_UNSUPPORTED, "IMEX levels and stiff reactions are 1D");
  if (p->n > (int64_t)kImexMaxThreads * kImexMaxRows)
    return fail(RIDC_E_UNSUPPORTED, "IMEX levels take n <= 8192");
  if (e->reserved != 0) return fail(RIDC_E_INVAL, "ext.reserved must be 0");
  if (e->fs_kind < RIDC_FS_DIFFUSION || e->fs_kind > RIDC_FS_CUBIC)
    return fail(RIDC_E_INVAL, "unknown stiff term");
  if (e->fs_kind != RIDC_FS_DIFFUSION && p->bc != RIDC_BC_DIRICHLET0)
    return fail(RIDC_E_UNSUPPORTED, "a stiff reaction needs a Dirichlet grid");
  if (!std::isfinite(e->kappa)) return fail(RIDC_E_INVAL, "kappa must be finite");
  if (e->newton_maxit < 0 || e->newton_maxit > 1000)
    return fail(RIDC_E_INVAL, "newton_maxit must be in 0..1000");
  ImexPlan pl;
  const int P = p->order;
  int acc = 0;
  for (int j = 0; j < P; ++j) {
    ImexPair pr;
    if (!imex_pair(e->pair[j], &pr)) return fail(RIDC_E_INVAL, "unknown pair of a level");
    // stage 0 explicit at c = 0, every later stage implicit (true of every pair of section II)
    if (pr.AS[0][0] != 0.0 || pr.c6[0] != 0) return fail(RIDC_E_UNSUPPORTED, "pair shape");
    for (int i = 1; i < pr.s; ++i)
      if (pr.AS[i][i] == 0.0) return fail(RIDC_E_UNSUPPORTED, "pair shape");
    acc += pr.order;
    pl.pair.push_back(pr);
    pl.S.push_back(acc);
  }
  if (acc > kMaxOrder) return fail(RIDC_E_UNSUPPORTED, "the top level's order exceeds 12");
  pl.delay.assign(P, 0);
  for (int j = 1; j < P; ++j) pl.delay[j] = pl.delay[j - 1] + pl.S[j] - 1;
  pl.R.resize(P);
  for (int j = 0; j < P; ++j) pl.R[j] = j + 1 < P ? 2 * pl.S[j + 1] - 1 : 2;
  const size_t vec = sizeof(double) * (size_t)p->n;
  for (int j = 0; j < P; ++j) {
    pl.rings += vec * pl.R[j];
    if (j + 1 < P) pl.frings += vec * pl.R[j];
    if (j > 0)
      pl.weights += sizeof(double) * (size_t)(pl.S[j] - 1) * pl.pair[j].s * 2 * pl.S[j];
    pl.work += vec * (2 * pl.pair[j].s + 1);
  }
  pl.rings = align256(pl.rings);
  pl.frings = align256(pl.frings);
  pl.weights = align256(std::max<size_t>(pl.weights, 8));
  pl.work = align256(pl.work);
  pl.items = align256(sizeof(ImexLvl) * P);
  pl.total = pl.rings + pl.frings + pl.weights + pl.work + pl.items + 256;   // + flag
  imex_shape(p->n, &pl.M, &pl.T);
  if (out) *out = pl;
  return RIDC_OK;
}

// One grouped launch per pipeline step for IMEX handles of one shape class (rows per thread,
// threads, boundary kind): every level of every handle in one table, each handle's own step
// = launch step + its current sigma.  Handles at their first step also get the launch that
// writes f of the initial values (harmless for the others: f of a stored value, rewritten).
int advance_imex(const std::vector<ridc_handle*>& hs, int64_t max_steps, hipStream_t stream) {
  std::vector<ridc_handle*> rest = hs;
  while (!rest.empty()) {
    const ridc_handle* k = rest[0];
    std::vector<ridc_handle*> grp, other;
    for (auto* h : rest)
      (h->imex_M == k->imex_M && h->imex_T == k->imex_T && h->p.bc == k->p.bc ? grp : other)
          .push_back(h);
    rest.swap(other);
    size_t nitems = 0;
    for (auto* h : grp) nitems += h->P;
    int rc = arena_reserve(1, 1, stream);
    if (rc != RIDC_OK) return rc;
    rc = arena_reserve_imex(nitems);
    if (rc != RIDC_OK) return rc;
    size_t q = 0;
    bool init = false;
    int64_t steps = 0;
    for (auto* h : grp) {
      init = init || h->sigma == 0;
      steps = std::max(steps, std::min(max_steps, h->total - h->sigma));
      for (int j = 0; j < h->P; ++j) {
        ImexLvl L = h->iproto[j];
        L.nt = h->nt;
        L.sigma0 = -h->sigma;
        g_arena.h_imex[q++] = L;
      }
    }
    RIDC_HIP_TRY(hipMemcpyAsync(g_arena.d_imex, g_arena.h_imex, sizeof(ImexLvl) * nitems,
                                hipMemcpyHostToDevice, stream));
    RIDC_HIP_TRY(hipEventRecord(g_arena.done, stream));
    g_arena.pending = true;
    const bool per = k->p.bc == RIDC_BC_PERIODIC;
    if (init)
      RIDC_HIP_TRY(launch_imex1d(g_arena.d_imex, (int)nitems, k->imex_M, k->imex_T, per, 0, true,
                                 stream));
    for (int64_t st = 1; st <= steps; ++st)
      RIDC_HIP_TRY(launch_imex1d(g_arena.d_imex, (int)nitems, k->imex_M, k->imex_T, per, st,
                                 false, stream));
    rc = arena_release(stream);
    if (rc != RIDC_OK) return rc;
    for (auto* h : grp) h->sigma += std::min(max_steps, h->total - h->sigma);
  }
  return RIDC_OK;
}

// Average duration (us) of `reps` consecutive whole steps (every stage) of one plan from step s.
int time_2d_steps(Plan2D* pl, int64_t s, int reps, hipStream_t stream, double* us) {
  Plan2D* pls[1] = {pl};
  int64_t before = s - 1;
  int rc = plan2d_advance(pls, 1, &before, 1, stream);       // warm
  if (rc != RIDC_OK) return rc;
  hipEvent_t a, b;
  RIDC_HIP_TRY(hipEventCreate(&a));
  RIDC_HIP_TRY(hipEventCreate(&b));
  before = s;
  (void)hipEventRecord(a, stream);
  rc = plan2d_advance(pls, 1, &before, reps, stream);
  (void)hipEventRecord(b, stream);
  hipError_t e = hipEventSynchronize(b);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != RIDC_OK) return rc;
  if (e != hipSuccess) return fail(RIDC_E_HIP, std::string("step timing: ") + hipGetErrorString(e));
  *us = 1e3 * (double)ms / reps;
  return RIDC_OK;
}

// 2D: the transform-pass shape of the handle's (n, precision), from the tuning table or
// measured: every shape the plan allows times whole steps with every level active (10 at
// n <= 1024, fewer above so that the measurement stays near a tenth of a second per shape; on
// zeroed rings; a shape can change the first pass of a solve and the later ones differently),
// best of three rounds; the fastest is kept and recorded.  Leaves the handle unarmed.
// Outputs: threads per block of the chosen shape, 0, and the shape bits.
int autotune_2d(ridc_handle* h, int32_t* threads_out, int32_t* rows_out, int32_t* flags_out) {
  Plan2D* pl = h->p2;
  const int prec = h->p.prec;
  int tile = 0;
  if (!tune_get_2d(h->p.n, prec, &tile) || plan2d_set_tile(pl, tile) != RIDC_OK) {
    std::vector<int> cands;
    plan2d_tile_candidates(pl, &cands);
    tile = cands[0];
    if (cands.size() > 1) {
      int64_t slots = 0;
      for (int j = 0; j < h->P; ++j) slots += h->R[j];
      RIDC_HIP_TRY(hipMemsetAsync(h->ring[0], 0, sizeof(double) * (size_t)(slots * h->npts),
                                  h->stream));
      int rc = plan2d_arm(pl, (int64_t)1 << 30, h->stream);
      if (rc != RIDC_OK) return rc;
      const int64_t s = (int64_t)h->P * (h->P - 1) / 2 + 1;   // every level active
      const double scale = 1024.0 / (double)h->p.n;
      const int steps = (int)std::max(1.0, std::min(10.0, 10.0 * scale * scale * scale));
      // three interleaved rounds, each candidate's best round counts (shapes within a few
      // per cent of each other would otherwise trade places with the run-to-run spread)
      std::vector<double> t(cands.size(), 1e300);
      for (int round = 0; round < 3; ++round)
        for (size_t i = 0; i < cands.size(); ++i) {
          rc = plan2d_set_tile(pl, cands[i]);
          if (rc != RIDC_OK) return rc;
          double us = 0;
          rc = time_2d_steps(pl, s, steps, h->stream, &us);
          if (rc != RIDC_OK) return rc;
          t[i] = std::min(t[i], us);
        }
      size_t bi = 0;
      for (size_t i = 1; i < cands.size(); ++i)
        if (t[i] < t[bi]) bi = i;
      tile = cands[bi];
    }
    tune_put_2d(h->p.n, prec, tile);
    int rc = plan2d_set_tile(pl, tile);
    if (rc != RIDC_OK) return rc;
  }
  h->nt = -1;
  h->sigma = h->total = 0;
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  h->graph_nt = -1;
  if (threads_out) *threads_out = (tile & kPassWide64) ? 256 : 512;
  if (rows_out) *rows_out = 0;
  if (flags_out) *flags_out = tile;
  return RIDC_OK;
}

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

const char* ridc_version(void) { return "ridc-gfx950 0.1"; }

const char* ridc_last_error(void) { return ridc::g_last_error.c_str(); }

int ridc_quadrature_weights(int32_t j, int32_t r, double* out) {
  if (!out) return fail(RIDC_E_INVAL, "out is NULL");
  if (!quadrature_weights(j, r, out)) return fail(RIDC_E_INVAL, "need 1 <= j < 12, 0 <= r < j");
  return RIDC_OK;
}

int ridc_pcr_plan(double r, int64_t m, int32_t* stages, double* divisor) {
  PcrPlan pl;
  if (!pcr_plan(r, m, &pl)) return fail(RIDC_E_INVAL, "bad PCR parameters");
  if (stages) *stages = pl.stages;
  if (divisor) *divisor = pl.divisor;
  return RIDC_OK;
}

size_t ridc_footprint_bytes(const ridc_problem* p) {
  if (validate(p) != RIDC_OK) return 0;
  Layout L;
  if (p->dim == 1) {
    PcrPlan pcr;
    Tile1D tile;
    if (plan_1d(p, &pcr, &tile) != RIDC_OK) return 0;
    plan_layout(p, &tile, &L);
  } else {
    plan_layout(p, nullptr, &L);
  }
  return L.total;
}

int ridc_create(const ridc_problem* p, void* hip_stream, ridc_handle** out) {
  if (!out) return fail(RIDC_E_INVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc != RIDC_OK) return rc;
  auto* h = new ridc_handle();
  h->p = *p;
  h->stream = (hipStream_t)hip_stream;
  h->P = p->order;
  h->npts = p->dim == 1 ? p->n : p->n * p->n;
  h->h = grid_h(p);
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(RIDC_E_HIP, "hipGetDevice failed");
  }
  Tile1D tile;
  if (p->dim == 1) {
    rc = plan_1d(p, &h->pcr, &tile);
    if (rc != RIDC_OK) {
      delete h;
      return rc;
    }
  }
  Layout L;
  plan_layout(p, &tile, &L);
  if (hipMalloc(&h->pool, L.total) != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    return fail(RIDC_E_NOMEM, "device allocation of " + std::to_string(L.total) + " bytes failed");
  }
  h->pool_bytes = L.total;
  char* cur = h->pool;
  double* rings = (double*)cur;
  cur += L.rings;
  h->W = (double*)cur;
  cur += L.weights;
  h->flag = (int*)cur;
  cur += L.flag;
  h->ring.resize(h->P);
  h->R.resize(h->P);
  double* rp = rings;
  for (int j = 0; j < h->P; ++j) {
    h->R[j] = ring_slots(j, h->P);
    h->ring[j] = rp;
    rp += (int64_t)h->R[j] * h->npts;
  }
  // weights: level j, rows r = 0..j-1, ascending nodes
  std::vector<double> w;
  h->woff.assign(h->P, 0);
  for (int j = 1; j < h->P; ++j) {
    h->woff[j] = (int64_t)w.size();
    for (int r = 0; r < j; ++r) {
      double row[kMaxOrder + 1];
      quadrature_weights(j, r, row);
      w.insert(w.end(), row, row + j + 1);
    }
  }
  if (!w.empty() &&
      hipMemcpy(h->W, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    ridc_destroy(h);
    return fail(RIDC_E_HIP, "weight upload failed");
  }
  if (hipMemset(h->flag, 0, sizeof(int)) != hipSuccess) {
    ridc_destroy(h);
    return fail(RIDC_E_HIP, "flag init failed");
  }
  if (p->dim == 1) {
    h->d_items = (Lvl1D*)cur;
    cur += L.items;
    h->d_fused = (Fused1D*)((char*)h->d_items + align256(sizeof(Lvl1D) * h->P));
    h->d_blocks = (Blk1D*)cur;
    cur += L.blocks;
    h->blocks_cap = (size_t)L.nblocks;
    build_items_1d(h, tile);
    h->fused = tile.fused != 0;
    h->fused_threads = tile.fused ? tile.fused : 512;
    const FusedPlan fp = plan_fused(p, h->fused_threads);
    h->fused_lds = fp.lds;
    {
      Fused1D& F = h->fused_item;
      F = Fused1D{};
      for (int j = 0; j < h->P; ++j) {
        F.ring[j] = h->ring[j];
        F.W[j] = j > 0 ? h->W + h->woff[j] : nullptr;
        F.R[j] = h->R[j];
      }
      F.gamma = h->solo.gamma;
      F.shift = h->solo.shift;
      F.P = h->P;
      F.group = fp.group;
      F.n = (int32_t)p->n;
      F.M = h->solo.M;
      F.bc = p->bc;
      F.fe = p->fe_kind;
      F.stages = h->pcr.stages;
      F.dt = p->dt;
      F.ce = h->solo.ce;
      F.nu_h2 = h->solo.nu_h2;
      F.inv_divisor = 1.0 / h->pcr.divisor;
    }
    if (hipMemcpy(h->d_blocks, h->blocks.data(), sizeof(Blk1D) * h->blocks.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_items, h->proto.data(), sizeof(Lvl1D) * h->proto.size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
      ridc_destroy(h);
      return fail(RIDC_E_HIP, "item table upload failed");
    }
  } else {
    rc = plan2d_create(p, h->h, h->ring.data(), h->R.data(), h->W, h->woff.data(), cur, L.ws2d,
                       h->stream, &h->p2);
    if (rc != RIDC_OK) {
      ridc_destroy(h);
      return rc;
    }
    // untuned split-BF16 plans take the 32-wide k-slices for the first pass of a solve where
    // they are a choice (whole steps at n = 1024: 229-232 against 233-239 us)
    int tuned = 0;
    if (p->prec == RIDC_PREC_BF16X3_REFINE && !tune_get_2d(p->n, p->prec, &tuned)) {
      std::vector<int> c;
      plan2d_tile_candidates(h->p2, &c);
      if (std::find(c.begin(), c.end(), kPassNarrowK) != c.end())
        (void)plan2d_set_tile(h->p2, kPassNarrowK);
    }
  }
  *out = h;
  return RIDC_OK;
}

size_t ridc_footprint_bytes_ext(const ridc_problem* p, const ridc_ext* e) {
  ImexPlan pl;
  if (validate_ext(p, e, &pl) != RIDC_OK) return 0;
  return pl.total;
}

int ridc_stage_weights(int32_t S, int32_t r, int32_t pair, int32_t stage, double* interp,
                       double* quad) {
  ImexPair pr;
  if (!interp || !quad) return fail(RIDC_E_INVAL, "NULL output");
  if (!imex_pair(pair, &pr)) return fail(RIDC_E_INVAL, "unknown pair");
  if (stage < 0 || stage >= pr.s) return fail(RIDC_E_INVAL, "stage out of range");
  if (!stage_weights(S, r, pr.c6[stage], interp, quad))
    return fail(RIDC_E_INVAL, "need 2 <= S <= 12 and 0 <= r <= S-2");
  return RIDC_OK;
}

int ridc_create_ext(const ridc_problem* p, const ridc_ext* e, void* hip_stream,
                    ridc_handle** out) {
  if (!out) return fail(RIDC_E_INVAL, "out is NULL");
  *out = nullptr;
  ImexPlan pl;
  int rc = validate_ext(p, e, &pl);
  if (rc != RIDC_OK) return rc;
  auto* h = new ridc_handle();
  h->p = *p;
  h->ext = *e;
  h->imex = true;
  h->stream = (hipStream_t)hip_stream;
  h->P = p->order;
  h->npts = p->n;
  h->h = grid_h(p);
  h->S = pl.S;
  h->delay = pl.delay;
  h->R = pl.R;
  h->imex_M = pl.M;
  h->imex_T = pl.T;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(RIDC_E_HIP, "hipGetDevice failed");
  }
  if (hipMalloc(&h->pool, pl.total) != hipSuccess) {
    (void)hipGetLastError();
    delete h;
    return fail(RIDC_E_NOMEM, "device allocation of " + std::to_string(pl.total) + " bytes failed");
  }
  h->pool_bytes = pl.total;
  const int P = h->P;
  const int64_t n = p->n;
  char* cur = h->pool;
  double* rp = (double*)cur;
  cur += pl.rings;
  double* fp = (double*)cur;
  cur += pl.frings;
  double* wp = (double*)cur;
  cur += pl.weights;
  double* kp = (double*)cur;
  cur += pl.work;
  h->d_imex = (ImexLvl*)cur;
  cur += pl.items;
  h->flag = (int*)cur;
  h->ring.assign(P, nullptr);
  h->ringF.assign(P, nullptr);
  for (int j = 0; j < P; ++j) {
    h->ring[j] = rp;
    rp += (int64_t)h->R[j] * n;
    if (j + 1 < P) {
      h->ringF[j] = fp;
      fp += (int64_t)h->R[j] * n;
    }
  }
  // corrector weights: [row r][stage i][interp S, quad S], exact rationals rounded once
  std::vector<double> w;
  std::vector<int64_t> woff(P, 0);
  for (int j = 1; j < P; ++j) {
    woff[j] = (int64_t)w.size();
    const int S = h->S[j];
    for (int r = 0; r <= S - 2; ++r)
      for (int i = 0; i < pl.pair[j].s; ++i) {
        double li[kMaxOrder], qi[kMaxOrder];
        stage_weights(S, r, pl.pair[j].c6[i], li, qi);
        w.insert(w.end(), li, li + S);
        w.insert(w.end(), qi, qi + S);
      }
  }
  if (!w.empty() &&
      hipMemcpy(wp, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    ridc_destroy(h);
    return fail(RIDC_E_HIP, "weight upload failed");
  }
  if (hipMemset(h->flag, 0, sizeof(int)) != hipSuccess) {
    ridc_destroy(h);
    return fail(RIDC_E_HIP, "flag init failed");
  }
  const double hh = h->h;
  h->iproto.assign(P, ImexLvl{});
  for (int j = 0; j < P; ++j) {
    ImexLvl& L = h->iproto[j];
    const ImexPair& pr = pl.pair[j];
    L.own = h->ring[j];
    L.ownF = h->ringF[j];
    L.prev = j > 0 ? h->ring[j - 1] : nullptr;
    L.prevF = j > 0 ? h->ringF[j - 1] : nullptr;
    L.wt = j > 0 ? wp + woff[j] : nullptr;
    L.ks = kp;
    kp += (int64_t)(2 * pr.s + 1) * n;
    L.nt = 0;
    L.sigma0 = 0;
    L.delay = h->delay[j];
    L.n = (int32_t)n;
    L.j = j;
    L.s = pr.s;
    L.S = h->S[j];
    L.R_own = h->R[j];
    L.R_prev = j > 0 ? h->R[j - 1] : 1;
    L.bc = p->bc;
    L.fe = p->fe_kind;
    L.fs = e->fs_kind;
    L.maxit = e->newton_maxit > 0 ? e->newton_maxit : 30;
    L.dt = p->dt;
    L.ce = explicit_coeff(p->fe_kind, p->a, hh);
    L.nu_h2 = p->nu / (hh * hh);
    L.kappa = e->fs_kind == RIDC_FS_DIFFUSION ? 0.0 : e->kappa;
    for (int i = 0; i < kMaxStages; ++i)
      for (int l = 0; l < kMaxStages; ++l) {
        L.AS[i][l] = i < pr.s && l < pr.s ? pr.AS[i][l] : 0.0;
        L.AN[i][l] = i < pr.s && l < pr.s ? pr.AN[i][l] : 0.0;
      }
  }
  if (hipMemcpy(h->d_imex, h->iproto.data(), sizeof(ImexLvl) * P, hipMemcpyHostToDevice) !=
      hipSuccess) {
    ridc_destroy(h);
    return fail(RIDC_E_HIP, "item table upload failed");
  }
  *out = h;
  return RIDC_OK;
}

int ridc_destroy(ridc_handle* h) {
  if (!h) return RIDC_OK;
  (void)hipStreamSynchronize(h->stream);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->p2) plan2d_destroy(h->p2);
  if (h->pool) (void)hipFree(h->pool);
  delete h;
  return RIDC_OK;
}

int ridc_begin(ridc_handle* h, const double* u0_dev, int64_t nsteps) {
  int rc = arm_handle(h, u0_dev, nsteps);
  if (rc != RIDC_OK) return rc;
  // every level starts from the initial data (section III-E, Fig. 2): slot 0 of each ring
  for (int j = 0; j < h->P; ++j)
    RIDC_HIP_TRY(hipMemcpyAsync(h->ring[j], u0_dev, sizeof(double) * h->npts,
                                hipMemcpyDeviceToDevice, h->stream));
  return RIDC_OK;
}

int64_t ridc_remaining(const ridc_handle* h) {
  if (!h || h->nt < 0) return -1;
  return h->total - h->sigma;
}

int ridc_advance(ridc_handle* const* hs, int32_t count, int64_t max_steps) {
  int rc = check_handles(hs, count);
  if (rc != RIDC_OK) return rc;
  if (max_steps < 0) return fail(RIDC_E_INVAL, "max_steps must be >= 0");
  for (int32_t i = 0; i < count; ++i)
    if (hs[i]->nt < 0) return fail(RIDC_E_STATE, "handle not armed (call ridc_begin)");
  if (count == 0 || max_steps == 0) return RIDC_OK;
  hipStream_t stream = hs[0]->stream;
  int64_t steps = 0;
  for (int32_t i = 0; i < count; ++i)
    steps = std::max(steps, std::min(max_steps, hs[i]->total - hs[i]->sigma));
  if (steps == 0) return RIDC_OK;
  if (count == 1) {
    ridc_handle* h = hs[0];
    const int64_t k = std::min(max_steps, h->total - h->sigma);
    rc = run_solo_steps(h, h->sigma + 1, h->sigma + k);
    if (rc != RIDC_OK) return rc;
    h->sigma += k;
    return RIDC_OK;
  }
  // ---- 1D handles: one grouped launch per pipeline step --------------------------------------
  std::vector<ridc_handle*> h1, h2, h3;
  for (int32_t i = 0; i < count; ++i) {
    if (hs[i]->total - hs[i]->sigma <= 0) continue;
    (hs[i]->imex ? h3 : hs[i]->p.dim == 1 ? h1 : h2).push_back(hs[i]);
  }
  if (!h3.empty()) {
    rc = advance_imex(h3, max_steps, stream);
    if (rc != RIDC_OK) return rc;
  }
  // fused-eligible 1D handles: one workgroup each, every requested step in one launch
  {
    std::vector<ridc_handle*> hf, hs;
    // batches keep the GPU busy with one launch per step (measured faster than whole-range
    // workgroups); a handle tuned to the whole-range workgroup keeps it
    for (auto* h : h1) (h->fused ? hf : hs).push_back(h);
    h1.swap(hs);
    if (!hf.empty()) {
      rc = arena_reserve(1, 1, stream);
      if (rc != RIDC_OK) return rc;
      rc = arena_reserve_fused(hf.size());
      if (rc != RIDC_OK) return rc;
      int maxP = 1;
      size_t lds = 0;
      for (size_t i = 0; i < hf.size(); ++i) {
        ridc_handle* h = hf[i];
        maxP = std::max(maxP, h->P);
        const FusedPlan fp = plan_fused(&h->p, 512);
        lds = std::max(lds, fp.lds);
        Fused1D F = h->fused_item;
        F.group = fp.group;
        F.nt = h->nt;
        F.sigma0 = 0;
        F.sigma_first = h->sigma;
        F.sigma_last = std::min(h->total, h->sigma + max_steps);
        g_arena.h_fused[i] = F;
      }
      RIDC_HIP_TRY(hipMemcpyAsync(g_arena.d_fused, g_arena.h_fused, sizeof(Fused1D) * hf.size(),
                                  hipMemcpyHostToDevice, stream));
      RIDC_HIP_TRY(hipEventRecord(g_arena.done, stream));
      g_arena.pending = true;
      RIDC_HIP_TRY(launch_fused_1d(g_arena.d_fused, nullptr, (int)hf.size(), maxP, 512, lds,
                                   stream));
      rc = arena_release(stream);
      if (rc != RIDC_OK) return rc;
      for (auto* h : hf) h->sigma = std::min(h->total, h->sigma + max_steps);
    }
  }
  if (!h1.empty()) {
    const BatchTile bt = current_batch_tile();
    BatchStage st;
    rc = stage_batch_1d(h1, bt, false, stream, &st);
    if (rc != RIDC_OK) return rc;
    int64_t steps1 = 0;
    for (auto* h : h1) steps1 = std::max(steps1, std::min(max_steps, h->total - h->sigma));
    for (int64_t s = 1; s <= steps1; ++s)
      RIDC_HIP_TRY(launch_1d_step(g_arena.d_items, g_arena.d_blocks, st.nblocks, st.threads,
                                  st.maxP, st.lds, s, stream));
    rc = arena_release(stream);
    if (rc != RIDC_OK) return rc;
    for (auto* h : h1) h->sigma += std::min(max_steps, h->total - h->sigma);
  }
  // ---- 2D handles: grouped per step by the 2D planner -----------------------------------------
  if (!h2.empty()) {
    std::vector<Plan2D*> plans;
    std::vector<int64_t> before;
    int64_t steps2 = 0;
    for (auto* h : h2) {
      plans.push_back(h->p2);
      before.push_back(h->sigma);
      steps2 = std::max(steps2, std::min(max_steps, h->total - h->sigma));
    }
    rc = plan2d_advance(plans.data(), (int)plans.size(), before.data(), steps2, stream);
    if (rc != RIDC_OK) return rc;
    for (auto* h : h2) h->sigma += std::min(max_steps, h->total - h->sigma);
  }
  return RIDC_OK;
}

int ridc_read(ridc_handle* h, double* uT_dev, double* levels_dev) {
  if (!h) return fail(RIDC_E_INVAL, "NULL handle");
  if (h->nt < 0) return fail(RIDC_E_STATE, "handle not armed");
  if (h->sigma != h->total) return fail(RIDC_E_STATE, "pipeline steps remain");
  const size_t bytes = sizeof(double) * h->npts;
  const int top = h->P - 1;
  const double* src = h->ring[top] + (h->nt % h->R[top]) * h->npts;
  if (uT_dev) {
    RIDC_HIP_TRY(hipMemcpyAsync(uT_dev, src, bytes, hipMemcpyDeviceToDevice, h->stream));
    RIDC_HIP_TRY(launch_nonfinite_check(uT_dev, h->npts, h->flag, h->stream));
  }
  if (levels_dev) {
    for (int j = 0; j < h->P; ++j)
      RIDC_HIP_TRY(hipMemcpyAsync(levels_dev + (int64_t)j * h->npts,
                                  h->ring[j] + (h->nt % h->R[j]) * h->npts, bytes,
                                  hipMemcpyDeviceToDevice, h->stream));
  }
  return RIDC_OK;
}

int ridc_sync(ridc_handle* h) {
  if (!h) return fail(RIDC_E_INVAL, "NULL handle");
  RIDC_HIP_TRY(hipStreamSynchronize(h->stream));
  int f = 0;
  RIDC_HIP_TRY(hipMemcpy(&f, h->flag, sizeof(int), hipMemcpyDeviceToHost));
  if (f) {
    RIDC_HIP_TRY(hipMemset(h->flag, 0, sizeof(int)));
    return fail(RIDC_E_NONFINITE, "result holds a NaN or Inf");
  }
  return RIDC_OK;
}

int ridc_integrate(ridc_handle* h, const double* u0_dev, int64_t nsteps, double* uT_dev,
                   double* levels_dev) {
  int rc = ridc_begin(h, u0_dev, nsteps);
  if (rc != RIDC_OK) return rc;
  const bool use_graph = h->stream != nullptr && h->total > 0 && env_flag("RIDC_GRAPH", true);
  if (use_graph) {
    if (h->graph_nt != nsteps) {
      if (h->gexec) {
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
      }
      h->graph_nt = -1;
      hipGraph_t g = nullptr;
      RIDC_HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      rc = run_solo_steps(h, 1, h->total);
      hipError_t e = hipStreamEndCapture(h->stream, &g);
      if (rc != RIDC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return fail(RIDC_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(RIDC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
      h->graph_nt = nsteps;
    }
    RIDC_HIP_TRY(hipGraphLaunch(h->gexec, h->stream));
    h->sigma = h->total;
  } else {
    rc = ridc_advance(&h, 1, h->total);
    if (rc != RIDC_OK) return rc;
  }
  return ridc_read(h, uT_dev, levels_dev);
}

int ridc_integrate_restarts(ridc_handle* h, const double* u0_dev, int64_t nsteps,
                            int32_t segments, double* uT_dev) {
  if (!h || !u0_dev || !uT_dev) return fail(RIDC_E_INVAL, "NULL argument");
  if (segments < 1 || nsteps < 0 || nsteps % segments != 0)
    return fail(RIDC_E_INVAL, "nsteps must be a non-negative multiple of segments");
  const int64_t seg = nsteps / segments;
  // each segment restarts from the previous top level, held in uT (u0 and uT may alias: every
  // segment loads its start value into the rings before anything writes uT)
  const double* src = u0_dev;
  for (int32_t k = 0; k < segments; ++k) {
    int rc = ridc_integrate(h, src, seg, uT_dev, nullptr);
    if (rc != RIDC_OK) return rc;
    src = uT_dev;
  }
  return RIDC_OK;
}

int ridc_integrate_noalloc(const ridc_problem* p, void* hip_stream, const double* u0_dev,
                           int64_t nsteps, double* uT_dev, int* nonfinite_dev) {
  int rc = validate(p);
  if (rc != RIDC_OK) return rc;
  if (p->dim != 1) return fail(RIDC_E_UNSUPPORTED, "the allocation-free integration is 1D only");
  if (p->order > kNoAllocMaxOrder)
    return fail(RIDC_E_UNSUPPORTED, "the allocation-free integration covers orders up to 6");
  if (!u0_dev || !uT_dev) return fail(RIDC_E_INVAL, "NULL u0 or uT");
  if (nsteps < 0) return fail(RIDC_E_INVAL, "nsteps must be >= 0");
  if (nsteps > 0 && nsteps < p->order - 1)
    return fail(RIDC_E_INVAL, "nsteps must be 0 or >= order-1 (start-up quadrature)");
  const int P = p->order;
  const int64_t n = p->n;
  int64_t slots = 0;
  for (int j = 0; j < P; ++j) slots += ring_slots(j, P);
  const size_t need = kNoAllocRingsOffset + sizeof(double) * (size_t)(slots * n);
  if (need > kNoAllocScratchBytes)
    return fail(RIDC_E_UNSUPPORTED, "needs " + std::to_string(need) + " bytes of scratch; the "
                "allocation-free integration holds " + std::to_string(kNoAllocScratchBytes));
  PcrPlan pcr;
  Tile1D tile;
  const double h = grid_h(p);
  const int64_t M = p->bc == RIDC_BC_PERIODIC ? n : 2 * n + 2;
  if (!pcr_plan(p->dt * p->nu / (h * h), M, &pcr))
    return fail(RIDC_E_UNSUPPORTED, "PCR did not converge within the stage cap");
  rc = choose_tile_1d(p, pcr, &tile, /*allow_fused=*/false);
  if (rc != RIDC_OK) return rc;
  void* base = nullptr;
  rc = noalloc_scratch(&base);
  if (rc != RIDC_OK) return rc;
  hipStream_t stream = (hipStream_t)hip_stream;
  const size_t bytes = sizeof(double) * (size_t)n;
  if (nsteps == 0) {
    RIDC_HIP_TRY(hipMemcpyAsync(uT_dev, u0_dev, bytes, hipMemcpyDeviceToDevice, stream));
    if (nonfinite_dev) RIDC_HIP_TRY(launch_nonfinite_check(uT_dev, n, nonfinite_dev, stream));
    return RIDC_OK;
  }
  // the scratch array: tables, then the level rings (layout as in a handle's pool)
  char* b = static_cast<char*>(base);
  NoAllocTables t{};
  double* W[kNoAllocMaxOrder] = {};
  double* ring[kNoAllocMaxOrder] = {};
  int R[kNoAllocMaxOrder] = {};
  double* wdev = reinterpret_cast<double*>(b + kNoAllocWeightsOffset);
  for (int j = 1; j < P; ++j) {
    W[j] = wdev + t.nw;
    for (int r = 0; r < j; ++r) {
      quadrature_weights(j, r, t.w + t.nw);
      t.nw += j + 1;
    }
  }
  t.stages = pcr.stages;
  for (int k = 0; k < pcr.stages; ++k) {
    t.gamma[k] = pcr.gamma[k];
    t.shift[k] = (int32_t)pcr.shift[k];
  }
  double* rp = reinterpret_cast<double*>(b + kNoAllocRingsOffset);
  for (int j = 0; j < P; ++j) {
    R[j] = ring_slots(j, P);
    ring[j] = rp;
    rp += (int64_t)R[j] * n;
  }
  RIDC_HIP_TRY(launch_noalloc_tables(t, base, stream));
  // every level starts from the initial data (section III-E, Fig. 2): slot 0 of each ring
  for (int j = 0; j < P; ++j)
    RIDC_HIP_TRY(hipMemcpyAsync(ring[j], u0_dev, bytes, hipMemcpyDeviceToDevice, stream));
  Solo1D a{};
  fill_solo(*p, h, pcr, tile, ring, R, W,
            reinterpret_cast<const double*>(b + kNoAllocGammaOffset),
            reinterpret_cast<const int32_t*>(b + kNoAllocShiftOffset), nsteps, &a);
  Lvl1D probe{};
  probe.n = (int32_t)n;
  probe.bc = p->bc;
  probe.wrap = tile.wrap;
  probe.B = a.B;
  probe.H = a.H;
  const size_t lds = lds_bytes_1d(probe);
  RIDC_HIP_TRY(prepare_1d_step(tile.threads, P, lds));
  const int64_t total = pipeline_steps(nsteps, P);
  for (int64_t s = 1; s <= total; ++s)
    RIDC_HIP_TRY(launch_1d_solo(a, P * a.nchunks, tile.threads, P, lds, s, stream));
  const int top = P - 1;
  RIDC_HIP_TRY(hipMemcpyAsync(uT_dev, ring[top] + (nsteps % R[top]) * n, bytes,
                              hipMemcpyDeviceToDevice, stream));
  if (nonfinite_dev) RIDC_HIP_TRY(launch_nonfinite_check(uT_dev, n, nonfinite_dev, stream));
  return RIDC_OK;
}

int ridc_integrate_batch(ridc_handle* const* hs, int32_t count, const double* const* u0,
                         const int64_t* nsteps, double* const* uT) {
  int rc = check_handles(hs, count);
  if (rc != RIDC_OK) return rc;
  if (count > 0 && (!u0 || !nsteps || !uT)) return fail(RIDC_E_INVAL, "NULL array argument");
  if (count == 0) return RIDC_OK;
  // arm every handle, then fill slot 0 of every level ring of every instance in one launch
  // (every level starts from the initial data, section III-E)
  int64_t most = 0;
  std::vector<CopyItem> copies;
  for (int32_t i = 0; i < count; ++i) {
    if (!uT[i]) return fail(RIDC_E_INVAL, "NULL output");
    rc = arm_handle(hs[i], u0[i], nsteps[i]);
    if (rc != RIDC_OK) return rc;
    most = std::max(most, hs[i]->total);
    for (int j = 0; j < hs[i]->P; ++j)
      copies.push_back(CopyItem{u0[i], hs[i]->ring[j], hs[i]->npts, nullptr});
  }
  hipStream_t stream = hs[0]->stream;
  rc = stage_copies(copies, stream);
  if (rc != RIDC_OK) return rc;
  rc = ridc_advance(hs, count, most);
  if (rc != RIDC_OK) return rc;
  // the top level of every instance to its output, checked for non-finite values, in one launch
  copies.clear();
  for (int32_t i = 0; i < count; ++i) {
    ridc_handle* h = hs[i];
    const int top = h->P - 1;
    copies.push_back(CopyItem{h->ring[top] + (h->nt % h->R[top]) * h->npts, uT[i], h->npts,
                              h->flag});
  }
  return stage_copies(copies, stream);
}

int ridc_set_tile(ridc_handle* h, int32_t threads, int32_t rows, int32_t flags) {
  if (!h) return fail(RIDC_E_INVAL, "NULL handle");
  if (h->imex) return fail(RIDC_E_UNSUPPORTED, "IMEX levels have one launch shape per n");
  if (h->p.dim == 2) {
    // the transform-pass shape bits; threads and rows are implied by them
    (void)threads;
    if (rows != 0) return fail(RIDC_E_INVAL, "2D shapes take rows = 0");
    int rc = plan2d_set_tile(h->p2, flags);
    if (rc != RIDC_OK) return rc;
    if (h->gexec) {
      (void)hipGraphExecDestroy(h->gexec);
      h->gexec = nullptr;
    }
    h->graph_nt = -1;
    return RIDC_OK;
  }
  if (rows < 0 || (flags & ~3)) return fail(RIDC_E_INVAL, "bad rows or flags");
  if (flags & 2) {
    if (rows != 0) return fail(RIDC_E_INVAL, "the whole-range workgroup holds whole cycles");
    return apply_tile_1d(h, Tile1D{1, 0, 256, 0, threads});
  }
  Tile1D t{rows == 0 ? 1 : 0, rows, threads, flags & 1, 0};
  return apply_tile_1d(h, t);
}

int ridc_autotune(ridc_handle* h, int32_t* threads_out, int32_t* rows_out, int32_t* flags_out) {
  if (!h) return fail(RIDC_E_INVAL, "NULL handle");
  if (h->imex) return fail(RIDC_E_UNSUPPORTED, "IMEX levels have one launch shape per n");
  if (h->p.dim != 1) return autotune_2d(h, threads_out, rows_out, flags_out);
  {
    // a tiling recorded for this system (this process, or the tuning cache) is taken as is
    Tile1D t;
    if (tuned_tile(h->p.n, h->p.bc, h->pcr.stages, &t) && tile_fits(&h->p, h->pcr, t)) {
      int rc = apply_tile_1d(h, t);
      if (rc != RIDC_OK) return rc;
      int th, r, f;
      tile_to(t, &th, &r, &f);
      if (threads_out) *threads_out = th;
      if (rows_out) *rows_out = r;
      if (flags_out) *flags_out = f;
      return RIDC_OK;
    }
  }
  // the tuning steps overwrite the rings: start from zeros, leave the handle unarmed
  int64_t slots = 0;
  for (int j = 0; j < h->P; ++j) slots += h->R[j];
  RIDC_HIP_TRY(hipMemsetAsync(h->ring[0], 0, sizeof(double) * (size_t)(slots * h->npts), h->stream));
  std::vector<Tile1D> cands;
  for (int ft : {512, 1024}) cands.push_back(Tile1D{1, 0, 256, 0, ft});
  for (int nts : {0, 1})
    for (int T : {256, 512, 1024}) {
      cands.push_back(Tile1D{1, 0, T, nts});
      for (int B : {kMinChunk, 256, 512, 1024, 2048, 4096}) cands.push_back(Tile1D{0, B, T, nts});
    }
  Tile1D best{};
  float best_ms = 1e30f;
  for (const Tile1D& t : cands) {
    if (!tile_fits(&h->p, h->pcr, t)) continue;
    float ms = 0;
    int rc = time_tile_1d(h, t, 40, &ms);
    if (rc != RIDC_OK) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  if (best_ms >= 1e29f) return fail(RIDC_E_UNSUPPORTED, "no tile fits");
  int th, r, f;
  tile_to(best, &th, &r, &f);
  tune_put_1d(h->p.n, h->p.bc, h->pcr.stages, th, r, f);
  h->nt = -1;
  h->sigma = h->total = 0;
  int rc = apply_tile_1d(h, best);
  if (rc != RIDC_OK) return rc;
  if (threads_out) *threads_out = th;
  if (rows_out) *rows_out = r;
  if (flags_out) *flags_out = f;
  return RIDC_OK;
}

int ridc_tune_save(const char* path) { return tune_save(path); }

int ridc_tune_load(const char* path) {
  int rc = tune_load(path);
  if (rc != RIDC_OK) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_batch_tile_set = false;             // a loaded grouped tiling applies from the next launch
  return RIDC_OK;
}

int ridc_tune_clear(void) {
  tune_clear();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_batch_tile = BatchTile{};
  g_batch_tile_set = false;
  return RIDC_OK;
}

int ridc_set_batch_tile(int32_t threads, int32_t rows) {
  if (threads != 256 && threads != 512 && threads != 1024)
    return fail(RIDC_E_INVAL, "batch threads must be 256, 512 or 1024");
  if (rows < 0 || (rows > 0 && rows < 256)) return fail(RIDC_E_INVAL, "batch rows: 0 or >= 256");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_batch_tile = BatchTile{threads, rows};
  g_batch_tile_set = true;
  return RIDC_OK;
}

int ridc_autotune_batch(ridc_handle* const* hs, int32_t count, int32_t* threads_out,
                        int32_t* rows_out) {
  int rc = check_handles(hs, count);
  if (rc != RIDC_OK) return rc;
  std::vector<ridc_handle*> h1;
  for (int32_t i = 0; i < count; ++i)
    if (hs[i]->p.dim == 1 && !hs[i]->imex) h1.push_back(hs[i]);
  BatchTile best = current_batch_tile();
  {
    // a grouped tiling recorded in the tuning table (this process or the cache) is taken as is
    int t = 0, r = 0;
    if (tune_get_batch(&t, &r)) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_batch_tile = BatchTile{t, r};
      g_batch_tile_set = true;
      if (threads_out) *threads_out = t;
      if (rows_out) *rows_out = r;
      return RIDC_OK;
    }
  }
  if (!h1.empty()) {
    hipStream_t stream = h1[0]->stream;
    // the timed steps overwrite the rings: start from zeros, leave the handles unarmed
    for (auto* h : h1) {
      int64_t slots = 0;
      for (int j = 0; j < h->P; ++j) slots += h->R[j];
      RIDC_HIP_TRY(hipMemsetAsync(h->ring[0], 0, sizeof(double) * (size_t)(slots * h->npts),
                                  stream));
      h->nt = -1;
      h->sigma = h->total = 0;
    }
    int maxP = 1;
    for (auto* h : h1) maxP = std::max(maxP, h->P);
    const int64_t first = (int64_t)maxP * (maxP - 1) / 2 + 1;   // every level active
    hipEvent_t a, b;
    RIDC_HIP_TRY(hipEventCreate(&a));
    RIDC_HIP_TRY(hipEventCreate(&b));
    float best_ms = 1e30f;
    constexpr int kReps = 20;
    for (int T : {256, 512, 1024})
      for (int rows : {0, 512, 768, 1024, 1536, 2048, 4096}) {
        const BatchTile bt{T, rows};
        BatchStage st;
        rc = stage_batch_1d(h1, bt, true, stream, &st);
        if (rc != RIDC_OK) break;
        for (int64_t s = first; s < first + 3 && rc == RIDC_OK; ++s)   // warm-up
          if (launch_1d_step(g_arena.d_items, g_arena.d_blocks, st.nblocks, st.threads, st.maxP,
                             st.lds, s, stream) != hipSuccess)
            rc = fail(RIDC_E_HIP, "batch tuning launch failed");
        if (rc != RIDC_OK) break;
        (void)hipEventRecord(a, stream);
        for (int64_t s = first + 3; s < first + 3 + kReps && rc == RIDC_OK; ++s)
          if (launch_1d_step(g_arena.d_items, g_arena.d_blocks, st.nblocks, st.threads, st.maxP,
                             st.lds, s, stream) != hipSuccess)
            rc = fail(RIDC_E_HIP, "batch tuning launch failed");
        (void)hipEventRecord(b, stream);
        if (rc == RIDC_OK) rc = arena_release(stream);
        if (rc != RIDC_OK) break;
        float ms = 0;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
          rc = fail(RIDC_E_HIP, "batch tuning timing failed");
          break;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best = BatchTile{st.threads, rows};
        }
      }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != RIDC_OK) return rc;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_batch_tile = best;
      g_batch_tile_set = true;
    }
    tune_put_batch(best.threads, best.rows);
  }
  if (threads_out) *threads_out = best.threads;
  if (rows_out) *rows_out = best.rows;
  return RIDC_OK;
}

int ridc_batch_kernel_time(ridc_handle* const* hs, int32_t count, int32_t reps,
                           double* us_per_launch, double* bytes_per_launch) {
  int rc = check_handles(hs, count);
  if (rc != RIDC_OK) return rc;
  if (reps < 1 || !us_per_launch) return fail(RIDC_E_INVAL, "bad arguments");
  std::vector<ridc_handle*> h1;
  double bytes = 0;
  for (int32_t i = 0; i < count; ++i) {
    ridc_handle* h = hs[i];
    if (h->p.dim != 1 || h->imex)
      return fail(RIDC_E_UNSUPPORTED, "grouped 1D launches only");
    if (h->nt < 0) return fail(RIDC_E_STATE, "handle not armed");
    if (h->fused) return fail(RIDC_E_UNSUPPORTED, "handle uses the whole-range workgroup");
    const int64_t first_full = (int64_t)h->P * (h->P - 1) / 2 + 1;
    if (h->sigma + 1 < first_full || h->sigma + 1 - first_full + 1 > h->nt)
      return fail(RIDC_E_STATE, "the next pipeline step does not have every level active");
    double b = 0, f = 0;
    rc = ridc_step_cost(h, &b, &f);
    if (rc != RIDC_OK) return rc;
    bytes += b;
    h1.push_back(h);
  }
  if (h1.empty()) return fail(RIDC_E_INVAL, "no handles");
  const BatchTile bt = current_batch_tile();
  hipStream_t stream = h1[0]->stream;
  BatchStage st;
  rc = stage_batch_1d(h1, bt, false, stream, &st);
  if (rc != RIDC_OK) return rc;
  // the handles' next step, launched repeatedly: it recomputes the same values (its inputs are
  // other ring slots), so the handles do not advance
  for (int w = 0; w < 3; ++w)
    RIDC_HIP_TRY(launch_1d_step(g_arena.d_items, g_arena.d_blocks, st.nblocks, st.threads,
                                st.maxP, st.lds, 1, stream));
  hipEvent_t a, b;
  RIDC_HIP_TRY(hipEventCreate(&a));
  RIDC_HIP_TRY(hipEventCreate(&b));
  (void)hipEventRecord(a, stream);
  for (int32_t r = 0; r < reps && rc == RIDC_OK; ++r)
    if (launch_1d_step(g_arena.d_items, g_arena.d_blocks, st.nblocks, st.threads, st.maxP,
                       st.lds, 1, stream) != hipSuccess)
      rc = fail(RIDC_E_HIP, "grouped launch failed");
  (void)hipEventRecord(b, stream);
  if (rc == RIDC_OK) rc = arena_release(stream);
  float ms = 0;
  if (rc == RIDC_OK &&
      (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
    rc = fail(RIDC_E_HIP, "event timing failed");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != RIDC_OK) return rc;
  *us_per_launch = 1e3 * (double)ms / reps;
  if (bytes_per_launch) *bytes_per_launch = bytes;
  return RIDC_OK;
}

int ridc_stencil_time(ridc_handle* h, int32_t reps, double* us_per_launch,
                      double* bytes_per_launch) {
  if (!h || reps < 1 || !us_per_launch) return fail(RIDC_E_INVAL, "bad arguments");
  if (h->p.dim != 2)
    return fail(RIDC_E_UNSUPPORTED, "1D stencils are fused into the level-step kernel");
  if (h->nt < 0) return fail(RIDC_E_STATE, "handle not armed");
  const int64_t s = h->sigma + 1;
  const int64_t first_full = (int64_t)h->P * (h->P - 1) / 2 + 1;
  if (s < first_full || s - first_full + 1 > h->nt)
    return fail(RIDC_E_STATE, "the next pipeline step does not have every level active");
  double bytes = 0;
  int rc = plan2d_time_rhs(h->p2, s, reps, h->stream, us_per_launch, &bytes);
  if (rc != RIDC_OK) return rc;
  if (bytes_per_launch) *bytes_per_launch = bytes;
  return RIDC_OK;
}

int ridc_kernel_time(ridc_handle* h, int32_t reps, double* us_per_launch, double* work_per_launch) {
  if (!h || reps < 1 || !us_per_launch) return fail(RIDC_E_INVAL, "bad arguments");
  if (h->nt < 0) return fail(RIDC_E_STATE, "handle not armed");
  const int64_t s = h->sigma + 1;
  const int64_t first_full = first_full_step(h);
  if (s < first_full || s - first_full + 1 > h->nt)
    return fail(RIDC_E_STATE, "the next pipeline step does not have every level active");
  double bytes = 0, flops = 0;
  int rc = ridc_step_cost(h, &bytes, &flops);
  if (rc != RIDC_OK) return rc;
  if (h->p.dim == 2) {
    rc = plan2d_time_pass(h->p2, s, reps, h->stream, us_per_launch);
    if (rc != RIDC_OK) return rc;
    const int passes = h->p.prec == RIDC_PREC_FP64 ? 4 : 8;
    if (work_per_launch) *work_per_launch = flops / passes;   // one pass over every level
    return RIDC_OK;
  }
  if (h->imex) {
    // `reps` launches of the same step: each recomputes the same values (every level reads
    // only slots that no level of this step writes)
    const bool per = h->p.bc == RIDC_BC_PERIODIC;
    hipEvent_t a, b;
    RIDC_HIP_TRY(hipEventCreate(&a));
    RIDC_HIP_TRY(hipEventCreate(&b));
    hipError_t e = launch_imex1d(h->d_imex, h->P, h->imex_M, h->imex_T, per, s, false, h->stream);
    if (e == hipSuccess) e = hipEventRecord(a, h->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
      e = launch_imex1d(h->d_imex, h->P, h->imex_M, h->imex_T, per, s, false, h->stream);
    if (e == hipSuccess) e = hipEventRecord(b, h->stream);
    float ms = 0;
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(RIDC_E_HIP, std::string("kernel timing: ") + hipGetErrorString(e));
    *us_per_launch = 1e3 * (double)ms / reps;
    if (work_per_launch) *work_per_launch = bytes;
    return RIDC_OK;
  }
  if (h->fused) {
    // the fused kernel runs many steps per launch: time `reps` steps in one launch (the handle
    // runs ahead, so it is left unarmed)
    if (s + reps - 1 > h->total) return fail(RIDC_E_STATE, "fewer pipeline steps left than reps");
    hipEvent_t a, b;
    RIDC_HIP_TRY(hipEventCreate(&a));
    RIDC_HIP_TRY(hipEventCreate(&b));
    (void)hipEventRecord(a, h->stream);
    rc = launch_fused_steps(h, s, s + reps - 1);
    (void)hipEventRecord(b, h->stream);
    float ms = 0;
    hipError_t e = rc == RIDC_OK ? hipEventSynchronize(b) : hipSuccess;
    if (rc == RIDC_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    h->nt = -1;
    if (rc != RIDC_OK) return rc;
    if (e != hipSuccess) return fail(RIDC_E_HIP, std::string("kernel timing: ") + hipGetErrorString(e));
    *us_per_launch = 1e3 * (double)ms / reps;
    if (work_per_launch) *work_per_launch = bytes;
    return RIDC_OK;
  }
  hipEvent_t a, b;
  RIDC_HIP_TRY(hipEventCreate(&a));
  RIDC_HIP_TRY(hipEventCreate(&b));
  rc = launch_solo_steps_1d(h, s, s);                           // warm
  if (rc == RIDC_OK) {
    (void)hipEventRecord(a, h->stream);
    for (int r = 0; r < reps && rc == RIDC_OK; ++r) rc = launch_solo_steps_1d(h, s, s);
    (void)hipEventRecord(b, h->stream);
  }
  float ms = 0;
  hipError_t e = rc == RIDC_OK ? hipEventSynchronize(b) : hipSuccess;
  if (rc == RIDC_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != RIDC_OK) return rc;
  if (e != hipSuccess) return fail(RIDC_E_HIP, std::string("kernel timing: ") + hipGetErrorString(e));
  *us_per_launch = 1e3 * (double)ms / reps;
  if (work_per_launch) *work_per_launch = bytes;
  return RIDC_OK;
}

int ridc_step_cost(const ridc_handle* h, double* hbm_bytes, double* flops) {
  if (!h) return fail(RIDC_E_INVAL, "NULL handle");
  // steady state, all levels active: level 0 reads its value and writes one; level j >= 1 reads
  // its value and the j+1 window values of level j-1 and writes one
  double vectors = 0;
  if (h->imex) {
    // IMEX levels: a level reads its value (and, corrector j, the S_j values and S_j stored f of
    // its window) and writes its value and f (the top level: its value only)
    for (int j = 0; j < h->P; ++j)
      vectors += 1 + (j > 0 ? 2 * h->S[j] : 0) + (j + 1 < h->P ? 2 : 1);
  } else {
    for (int j = 0; j < h->P; ++j) vectors += j == 0 ? 2 : j + 3;
  }
  double b = vectors * sizeof(double) * (double)h->npts;
  double f = 0;
  if (h->p.dim == 2) plan2d_cost(h->p2, &b, &f);
  if (hbm_bytes) *hbm_bytes = b;
  if (flops) *flops = f;
  return RIDC_OK;
}

}  // extern "C"
