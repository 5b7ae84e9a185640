// Host side of libefpi: configuration checks, workspace layout and the
// extern "C" entry points declared in include/efpi.h.  Every entry point only
// enqueues kernels on the context's stream (except those documented as
// synchronous); the library never allocates device memory (its one device array,
// the static scratch of efpi_phase_restrict_static, comes with the code object).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "efpi.h"
#include "efpi_internal.h"

using namespace efpi;

namespace {

thread_local std::string g_err;

efpi_status fail(efpi_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << (l + 1)) <= x) ++l;
  return l;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kDefaultTile = 4096;
constexpr size_t kMaxGraphs = 8;  // captured macro steps kept per context
constexpr int kColdIters = 40;     // Newton iterations of a context's first (cold) solve

// First failure among the enqueue calls of the current entry point; hip_check()
// reports it (or else the runtime's last error) and clears it.
thread_local hipError_t t_enqueue_error = hipSuccess;

void note(hipError_t e) {
  if (e != hipSuccess && t_enqueue_error == hipSuccess) t_enqueue_error = e;
}

}  // namespace

// ------------------------------------------------------------ static scratch --
// The int64 histogram of efpi_phase_restrict_static: a file-scope device array
// that every GPU the library runs on holds until the process ends.  In host code
// its name stands for the variable, not for device memory: the device address is
// looked up once per device (hipGetSymbolAddress at the first efpi_init with that
// device current) and only that address goes to kernels and fills.
static_assert(EFPI_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size in 256-byte units");
static __device__ __align__(256) long long scratch[EFPI_STATIC_SCRATCH_BYTES / sizeof(long long)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
efpi_status scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(EFPI_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  if (dev < 0 || dev >= kMaxDevices) return fail(EFPI_EHIP, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(EFPI_EHIP, std::string("static scratch address: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return EFPI_OK;
}

}  // namespace

struct efpi_ctx {
  efpi_config cfg{};
  std::vector<efpi_replica> reps;
  hipStream_t stream = nullptr;
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  void* scratch = nullptr;  // device address of the static scratch on this device
  int R = 0;
  int tile = kDefaultTile;
  int grid_blocks = 0;
  std::vector<RepDev> h_reps;
  RepDev* d_reps = nullptr;
  uint32_t* d_status = nullptr;
  int64_t* d_item_prefix = nullptr;
  int64_t* d_block_prefix = nullptr;
  int64_t* d_snap_off = nullptr;
  int64_t* d_coarse_off = nullptr;
  int32_t* d_group = nullptr;
  bool kinetic = false;             // kinetic electrons (every replica)
  bool lift_deposit = false;        // the lift deposits the ions' charge itself
  int moments = 2;                  // coarse moments per replica (3: EFPI_FLAG_PRESSURE)
  int max_nodes = 0;                // largest node count of the replicas
  std::vector<RepDev> h_ereps;      // electron descriptors (kinetic contexts)
  RepDev* d_ereps = nullptr;
  int64_t* d_eitem_prefix = nullptr;  // electron work items (sort) per replica
  std::vector<int64_t> h_eitem_prefix;
  int64_t total_eitems = 0;
  double* d_snap = nullptr;
  double* d_coarse = nullptr;
  int32_t* d_sort_hist = nullptr;
  int64_t* d_sort_base = nullptr;
  std::vector<int64_t> h_item_prefix, h_block_prefix, h_snap_off, h_coarse_off;
  std::vector<int32_t> h_group;
  int64_t total_items = 0, total_blocks = 0, snap_total = 0, coarse_total = 0;
  // state
  int cur = 0;             // q buffer holding the latest deposit
  bool other_zero = true;  // q[cur ^ 1] is known to be zero
  bool deposited = false;  // charge matches the current particles
  bool field_valid = false;
  bool phi_valid = false;  // phi holds a solve of this context (a warm start)
  bool fresh = true;       // ion velocities at an integer time level
  bool fresh_e = true;     // electron velocities at an integer time level (kinetic)
  int last_burst_steps = -1;
  // optional event timing of the burst-step particle launches
  bool timing = false;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
  // event pairs (indices into events) around the timed ion and electron launches
  std::vector<std::pair<size_t, size_t>> ion_pairs, el_pairs;
  // captured macro steps, keyed by their arguments and the state they start from
  struct HostState {
    int cur;
    bool other_zero, deposited, field_valid, phi_valid, fresh, fresh_e;
    int last_burst_steps;
  };
  HostState state() const {
    return {cur, other_zero, deposited, field_valid, phi_valid, fresh, fresh_e, last_burst_steps};
  }
  void set_state(const HostState& s) {
    cur = s.cur;
    other_zero = s.other_zero;
    deposited = s.deposited;
    field_valid = s.field_valid;
    phi_valid = s.phi_valid;
    fresh = s.fresh;
    fresh_e = s.fresh_e;
    last_burst_steps = s.last_burst_steps;
  }
  struct MacroGraph {
    const double* in;
    double* out;
    int cur0;            // the captured launches depend only on these three fields
    bool other_zero0;
    bool phi_valid0;
    HostState after;     // state the macro step leaves
    hipGraphExec_t exec;
  };
  std::vector<MacroGraph> graphs;
  ~efpi_ctx() {
    // work still queued may use the events, the captured graphs and the workspace
    note(hipStreamSynchronize(stream));
    for (hipEvent_t e : events) note(hipEventDestroy(e));
    for (MacroGraph& g : graphs) note(hipGraphExecDestroy(g.exec));
  }
};

namespace {

efpi_status check_config(const efpi_config* cfg) {
  if (!cfg) return fail(EFPI_EINVAL, "config is NULL");
  if (cfg->abi_version != EFPI_ABI_VERSION) return fail(EFPI_EINVAL, "abi_version mismatch");
  if (cfg->n_replicas < 1 || cfg->n_replicas > (uint32_t)kMaxShiftReplicas)
    return fail(EFPI_EINVAL, "n_replicas must be in [1, 256]");
  if (!cfg->replicas) return fail(EFPI_EINVAL, "replicas is NULL");
  if (cfg->newton_iters < 1 || cfg->newton_iters_start < 1)
    return fail(EFPI_EINVAL, "newton iteration counts must be >= 1");
  if (!(cfg->newton_tol > 0.0)) return fail(EFPI_EINVAL, "newton_tol must be > 0");
  if (cfg->tile != 0 && (cfg->tile % 1024 != 0 || cfg->tile < 1024 || cfg->tile > 16384))
    return fail(EFPI_EINVAL, "tile must be 0 or a multiple of 1024 in [1024, 16384]");
  if (cfg->grid_blocks < 0) return fail(EFPI_EINVAL, "grid_blocks must be >= 0");
  if ((cfg->flags & ~(EFPI_FLAG_SORT_BUFFER | EFPI_FLAG_PRESSURE)) != 0)
    return fail(EFPI_EINVAL, "unknown flags");
  if ((cfg->flags & EFPI_FLAG_PRESSURE) && cfg->replicas &&
      cfg->replicas[0].closure == EFPI_CLOSURE_KINETIC)
    return fail(EFPI_EINVAL, "EFPI_FLAG_PRESSURE is not supported with kinetic electrons");
  for (uint32_t r = 0; r < cfg->n_replicas; ++r) {
    const efpi_replica& p = cfg->replicas[r];
    char buf[160];
    auto bad = [&](const char* what) {
      std::snprintf(buf, sizeof buf, "replica %u: %s", r, what);
      return fail(EFPI_EINVAL, buf);
    };
    if (!is_pow2(p.n_cells) || p.n_cells < 8 || p.n_cells > 16384)
      return bad("n_cells must be a power of two in [8, 16384]");
    if (p.bc != EFPI_BC_PERIODIC && p.bc != EFPI_BC_WALLS) return bad("unknown bc");
    if (p.closure != EFPI_CLOSURE_BOLTZMANN && p.closure != EFPI_CLOSURE_NOFIELD &&
        p.closure != EFPI_CLOSURE_KINETIC)
      return bad("unsupported closure");
    if ((p.closure == EFPI_CLOSURE_KINETIC) != (cfg->replicas[0].closure == EFPI_CLOSURE_KINETIC))
      return bad("kinetic electrons must be used by every replica of a context or by none");
    if (p.closure == EFPI_CLOSURE_KINETIC) {
      if (p.bc != EFPI_BC_PERIODIC) return bad("kinetic electrons need a periodic domain");
      if (p.n_cells > 8192) return bad("kinetic electrons need n_cells <= 8192");
      if (!(p.qm_e < 0.0) || !std::isfinite(p.qm_e)) return bad("qm_e must be finite and < 0");
      if (!(p.vth_e >= 0.0) || !std::isfinite(p.vth_e)) return bad("vth_e must be >= 0");
      if (p.ppc_e < 1) return bad("ppc_e must be >= 1");
      if ((int64_t)p.n_cells * p.ppc_e > (int64_t(1) << 32))
        return bad("n_cells * ppc_e must fit in 32 bits (Hammersley index)");
      if (p.pad_e != 0) return bad("pad_e must be 0");
      if (p.capacity_e < 1 || p.capacity_e >= (int64_t(1) << 31))
        return bad("capacity_e must be in [1, 2^31 - 1]");
    }
    if (p.ppc < 1) return bad("ppc must be >= 1");
    if ((int64_t)p.n_cells * p.ppc > (int64_t(1) << 32))
      return bad("n_cells * ppc must fit in 32 bits (Hammersley index)");
    if (p.haar_levels < 0 || p.haar_levels > ilog2(p.n_cells)) return bad("haar_levels out of range");
    if (p.burst_steps < 1) return bad("burst_steps must be >= 1");
    if (!(p.length > 0.0) || !std::isfinite(p.length)) return bad("length must be > 0");
    if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return bad("dt must be > 0");
    if (!(p.macro_dt >= p.burst_steps * p.dt * (1.0 - 1e-12)) || !std::isfinite(p.macro_dt))
      return bad("macro_dt must be >= burst_steps * dt");
    if (!(p.vth >= 0.0) || !std::isfinite(p.vth)) return bad("vth must be >= 0");
    if (!(p.n_floor > 0.0)) return bad("n_floor must be > 0");
    if (p.capacity < 1 || p.capacity >= (int64_t(1) << 31)) return bad("capacity must be in [1, 2^31 - 1]");
  }
  return EFPI_OK;
}

// Lay the workspace out; with ctx != nullptr also fill the descriptors.
size_t layout(const efpi_config* cfg, efpi_ctx* ctx, uint8_t* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return base ? base + o : nullptr;
  };
  const int R = (int)cfg->n_replicas;
  uint8_t* p_status = take(sizeof(uint32_t));
  uint8_t* p_reps = take(sizeof(RepDev) * R);
  uint8_t* p_items = take(sizeof(int64_t) * (R + 1));
  uint8_t* p_blocks = take(sizeof(int64_t) * (R + 1));
  uint8_t* p_soff = take(sizeof(int64_t) * R);
  uint8_t* p_coff = take(sizeof(int64_t) * R);
  uint8_t* p_group = take(sizeof(int32_t) * R);
  const bool kinetic = cfg->replicas[0].closure == EFPI_CLOSURE_KINETIC;
  uint8_t* p_ereps = kinetic ? take(sizeof(RepDev) * R) : nullptr;
  uint8_t* p_eitems = kinetic ? take(sizeof(int64_t) * (R + 1)) : nullptr;
  const int nm = (cfg->flags & EFPI_FLAG_PRESSURE) ? 3 : 2;  // coarse moments per replica
  int64_t snap_total = 0, coarse_total = 0;
  for (int r = 0; r < R; ++r) {
    const efpi_replica& p = cfg->replicas[r];
    const int nc = p.n_cells >> p.haar_levels;
    snap_total += (int64_t)(p.burst_steps + 1) * nm * nc;
    coarse_total += nm * nc;
  }
  uint8_t* p_snap = take(sizeof(double) * snap_total);
  uint8_t* p_coarse = take(sizeof(double) * coarse_total);
  uint8_t* p_hist = nullptr;
  uint8_t* p_base = nullptr;
  if (cfg->flags & EFPI_FLAG_SORT_BUFFER) {
    const int tile = cfg->tile > 0 ? cfg->tile : kDefaultTile;
    int64_t items = 0;
    int64_t eitems = 0;
    for (int r = 0; r < R; ++r) {
      items += (cfg->replicas[r].capacity + tile - 1) / tile;
      if (kinetic) eitems += (cfg->replicas[r].capacity_e + tile - 1) / tile;
    }
    // the electron sort runs after the ion sort and reuses the histograms
    p_hist = take(sizeof(int32_t) * 256 * std::max(items, eitems));
    p_base = take(sizeof(int64_t) * 256 * R);
  }
  if (ctx) {
    ctx->d_status = reinterpret_cast<uint32_t*>(p_status);
    ctx->d_reps = reinterpret_cast<RepDev*>(p_reps);
    ctx->d_item_prefix = reinterpret_cast<int64_t*>(p_items);
    ctx->d_block_prefix = reinterpret_cast<int64_t*>(p_blocks);
    ctx->d_snap_off = reinterpret_cast<int64_t*>(p_soff);
    ctx->d_coarse_off = reinterpret_cast<int64_t*>(p_coff);
    ctx->d_group = reinterpret_cast<int32_t*>(p_group);
    ctx->d_snap = reinterpret_cast<double*>(p_snap);
    ctx->d_coarse = reinterpret_cast<double*>(p_coarse);
    ctx->d_sort_hist = reinterpret_cast<int32_t*>(p_hist);
    ctx->d_sort_base = reinterpret_cast<int64_t*>(p_base);
    ctx->snap_total = snap_total;
    ctx->coarse_total = coarse_total;
    ctx->h_reps.assign(R, RepDev{});
    ctx->kinetic = kinetic;
    ctx->moments = nm;
    // the lift's fused deposit holds a block's nodes in LDS: blocks of at most
    // 2^kLiftMaxDepositLevels cells (kinetic contexts deposit both species after
    // the electron load anyway)
    ctx->lift_deposit = !kinetic;
    for (int r = 0; r < R; ++r)
      if (cfg->replicas[r].haar_levels > kLiftMaxDepositLevels) ctx->lift_deposit = false;
    ctx->d_ereps = reinterpret_cast<RepDev*>(p_ereps);
    ctx->d_eitem_prefix = reinterpret_cast<int64_t*>(p_eitems);
    if (kinetic) ctx->h_ereps.assign(R, RepDev{});
  }
  int64_t soff = 0, coff = 0;
  const bool sortbuf = (cfg->flags & EFPI_FLAG_SORT_BUFFER) != 0;
  for (int r = 0; r < R; ++r) {
    const efpi_replica& p = cfg->replicas[r];
    const int n = p.n_cells;
    const int nn = p.bc == EFPI_BC_PERIODIC ? n : n + 1;
    const int nc = n >> p.haar_levels;
    const int64_t cap = p.capacity;
    uint8_t* cell = take(sizeof(int16_t) * cap);
    uint8_t* frac = take(sizeof(float) * cap);
    uint8_t* v = take(sizeof(float) * cap);
    uint8_t* w = take(sizeof(float) * cap);
    uint8_t *cell2 = nullptr, *frac2 = nullptr, *v2 = nullptr, *w2 = nullptr;
    if (sortbuf) {
      cell2 = take(sizeof(int16_t) * cap);
      frac2 = take(sizeof(float) * cap);
      v2 = take(sizeof(float) * cap);
      w2 = take(sizeof(float) * cap);
    }
    uint8_t* np = take(sizeof(int64_t));
    uint8_t* q0 = take(sizeof(int64_t) * (nn + 1));
    uint8_t* q1 = take(sizeof(int64_t) * (nn + 1));
    uint8_t* phi = take(sizeof(double) * (nn + 1));
    uint8_t* e = take(sizeof(float) * (nn + 1));
    uint8_t* en = take(sizeof(float) * (nn + 1));
    uint8_t* rb = take(sizeof(int64_t) * (int64_t)(p.burst_steps + 1) * nm * nc);
    uint8_t* pn = take(sizeof(double) * (nn + 1));
    uint8_t* pu = take(sizeof(double) * (nn + 1));
    uint8_t* pt = nm == 3 ? take(sizeof(double) * (nn + 1)) : nullptr;
    uint8_t* cor = take(sizeof(int32_t) * n);
    uint8_t* br = take(sizeof(int32_t) * (nc + 1));
    uint8_t* aux = take(sizeof(int64_t) * 4);
    // electron store and loading arrays of a kinetic replica
    uint8_t *ecell = nullptr, *efrac = nullptr, *ev = nullptr, *ew = nullptr, *enp = nullptr;
    uint8_t *epn = nullptr, *epu = nullptr, *ecor = nullptr, *ebr = nullptr, *eaux = nullptr;
    uint8_t *ecell2 = nullptr, *efrac2 = nullptr, *ev2 = nullptr, *ew2 = nullptr;
    uint8_t* jfx = nullptr;
    if (kinetic) {
      const int64_t cap_e = p.capacity_e;
      ecell = take(sizeof(int16_t) * cap_e);
      efrac = take(sizeof(float) * cap_e);
      ev = take(sizeof(float) * cap_e);
      ew = take(sizeof(float) * cap_e);
      if (sortbuf) {
        ecell2 = take(sizeof(int16_t) * cap_e);
        efrac2 = take(sizeof(float) * cap_e);
        ev2 = take(sizeof(float) * cap_e);
        ew2 = take(sizeof(float) * cap_e);
      }
      enp = take(sizeof(int64_t));
      epn = take(sizeof(double) * (nn + 1));
      jfx = take(sizeof(int64_t) * (nn + 1));
      epu = take(sizeof(double) * (nn + 1));
      ecor = take(sizeof(int32_t) * n);
      ebr = take(sizeof(int32_t) * (nc + 1));
      eaux = take(sizeof(int64_t) * 4);
    }
    if (ctx) {
      RepDev& d = ctx->h_reps[r];
      d.n_cells = n;
      d.n_nodes = nn;
      d.bc = p.bc;
      d.closure = p.closure;
      d.ppc = p.ppc;
      d.levels = p.haar_levels;
      d.n_coarse = nc;
      d.moments = nm;
      d.burst_steps = p.burst_steps;
      d.coevolving = p.coevolving;
      d.lift_linear = p.lift_linear;
      d.log2n = ilog2(n);
      // field solve: N rows over at most 256 threads up to N = 2048 (M = max(1,
      // N / 256)), then over 512 threads (M = 8 at N = 4096, 16 at 8192, 32 at
      // 16384; at N = 4096, 512 threads of 8 rows took 13.0 us for two Newton
      // iterations against 13.5 us for 256 threads of 16 rows)
      d.field_m = n <= 256 ? 1 : (n <= 2048 ? n / 256 : n / 512);
      d.h = p.length / n;
      d.inv_h = n / p.length;
      d.length = p.length;
      d.vth = p.vth;
      d.dt = p.dt;
      d.macro_dt = p.macro_dt;
      d.n_floor = p.n_floor;
      d.capacity = cap;
      d.cell = reinterpret_cast<int16_t*>(cell);
      d.frac = reinterpret_cast<float*>(frac);
      d.v = reinterpret_cast<float*>(v);
      d.w = reinterpret_cast<float*>(w);
      d.cell2 = reinterpret_cast<int16_t*>(cell2);
      d.frac2 = reinterpret_cast<float*>(frac2);
      d.v2 = reinterpret_cast<float*>(v2);
      d.w2 = reinterpret_cast<float*>(w2);
      d.np = reinterpret_cast<int64_t*>(np);
      d.q[0] = reinterpret_cast<int64_t*>(q0);
      d.q[1] = reinterpret_cast<int64_t*>(q1);
      d.phi = reinterpret_cast<double*>(phi);
      d.e = reinterpret_cast<float*>(e);
      d.en = reinterpret_cast<float*>(en);
      d.rbins = reinterpret_cast<int64_t*>(rb);
      d.snap = ctx->d_snap + soff;
      d.coarse_tmp = ctx->d_coarse + coff;
      d.prof_n = reinterpret_cast<double*>(pn);
      d.prof_u = reinterpret_cast<double*>(pu);
      d.prof_t = reinterpret_cast<double*>(pt);
      d.cell_of_rank = reinterpret_cast<int32_t*>(cor);
      d.block_rank = reinterpret_cast<int32_t*>(br);
      d.aux = reinterpret_cast<int64_t*>(aux);
      d.qm = 1.0;
      d.jfx = reinterpret_cast<int64_t*>(jfx);
      if (kinetic) {
        RepDev& el = ctx->h_ereps[r];
        el = d;
        el.ppc = p.ppc_e;
        el.vth = p.vth_e;
        el.capacity = p.capacity_e;
        el.qm = p.qm_e;
        el.cell = reinterpret_cast<int16_t*>(ecell);
        el.frac = reinterpret_cast<float*>(efrac);
        el.v = reinterpret_cast<float*>(ev);
        el.w = reinterpret_cast<float*>(ew);
        el.cell2 = reinterpret_cast<int16_t*>(ecell2);
        el.frac2 = reinterpret_cast<float*>(efrac2);
        el.v2 = reinterpret_cast<float*>(ev2);
        el.w2 = reinterpret_cast<float*>(ew2);
        el.np = reinterpret_cast<int64_t*>(enp);
        el.prof_n = reinterpret_cast<double*>(epn);
        el.prof_u = reinterpret_cast<double*>(epu);
        el.cell_of_rank = reinterpret_cast<int32_t*>(ecor);
        el.block_rank = reinterpret_cast<int32_t*>(ebr);
        el.aux = reinterpret_cast<int64_t*>(eaux);
      }
    }
    soff += (int64_t)(p.burst_steps + 1) * nm * nc;
    coff += nm * nc;
  }
  return off;
}

efpi_status hip_check(const char* where) {
  hipError_t e = t_enqueue_error;
  t_enqueue_error = hipSuccess;
  const hipError_t last = hipGetLastError();
  if (e == hipSuccess) e = last;
  if (e != hipSuccess) return fail(EFPI_EHIP, std::string(where) + ": " + hipGetErrorString(e));
  return EFPI_OK;
}

efpi_status check_ctx(efpi_ctx* ctx) {
  if (!ctx) return fail(EFPI_EINVAL, "context is NULL");
  return EFPI_OK;
}

efpi_status check_rep(efpi_ctx* ctx, int32_t r) {
  if (!ctx) return fail(EFPI_EINVAL, "context is NULL");
  if (r < 0 || r >= ctx->R) return fail(EFPI_EINVAL, "replica index out of range");
  return EFPI_OK;
}

void deposit_into_next(efpi_ctx* c) {
  if (!c->other_zero) launch_zero_charge(c->d_reps, c->R, c->cur ^ 1, c->stream);
}

void run_newton(efpi_ctx* c, int iters, int cold, int save_en, int zero_bins) {
  launch_newton(c->d_reps, c->R, iters, cold, c->cur, save_en, zero_bins, c->cfg.newton_tol,
                c->d_status, c->stream);
  c->other_zero = true;
  c->field_valid = true;
  c->phi_valid = true;
}

// Field of the current deposit: linear Poisson with kinetic electrons, else Newton.
void run_field(efpi_ctx* c, int iters, int cold, int save_en, int zero_bins) {
  if (c->kinetic) {
    launch_poisson(c->d_reps, c->R, c->cur, save_en, zero_bins, c->d_status, c->stream);
    c->other_zero = true;
    c->field_valid = true;
  } else {
    run_newton(c, iters, cold, save_en, zero_bins);
  }
}

// Charge of the current particles (both species in kinetic contexts) into the
// next buffer, which becomes the current one.
void deposit_all(efpi_ctx* c, bool electrons) {
  deposit_into_next(c);
  launch_particles(c->d_reps, c->d_item_prefix, c->R, c->total_items, c->tile, c->grid_blocks, 0,
                   kDepositOnly, c->cur ^ 1, c->d_status, c->stream);
  if (electrons && c->kinetic)
    launch_electrons(c->d_ereps, c->R, 0, 0, c->cur ^ 1, c->max_nodes, c->stream);
  c->cur ^= 1;
  c->other_zero = false;
  c->deposited = true;
}

// Electrons in Boltzmann equilibrium with the current ions: ion charge, Newton
// solve of eq. 3.15, density exp(phi) with the ions' fine velocity profile, and
// the quiet start with the electron rotation derived on the device from the
// ions' stored rotation.
void load_boltzmann_electrons(efpi_ctx* c) {
  deposit_all(c, false);
  run_newton(c, c->cfg.newton_iters_start, 1, 0, 0);
  launch_electron_profile(c->d_reps, c->d_ereps, c->R, 0, c->cur, c->stream);
  launch_occupancy(c->d_ereps, c->R, -1, c->d_status, c->stream);
  launch_lift_particles(c->d_ereps, c->d_block_prefix, c->R, c->total_blocks, -1, nullptr,
                        c->d_coarse_off, nullptr, c->grid_blocks, c->stream);
}

// New electrons (kinetic contexts): their first push is a half step.
void mark_new_electrons(efpi_ctx* c) {
  c->fresh_e = true;
  c->field_valid = false;
  c->deposited = false;
}

void mark_new_particles(efpi_ctx* c) {
  c->fresh = true;
  c->field_valid = false;
  c->deposited = false;
}

ShiftArg shifts_of(const efpi_ctx* c, const uint32_t* h_shifts) {
  ShiftArg s;
  std::memset(&s, 0, sizeof s);
  for (int r = 0; r < c->R; ++r) s.s[r] = h_shifts ? h_shifts[r] : 0u;
  return s;
}

// Lift of every replica; with h_shifts == nullptr the rotations already stored
// on the device (launch_set_shifts) are used.
efpi_status do_lift(efpi_ctx* c, const double* d_coarse, const uint32_t* h_shifts) {
  const ShiftArg sh = shifts_of(c, h_shifts);
  launch_lift_prep(c->d_reps, c->R, d_coarse, c->d_coarse_off, c->d_status,
                   h_shifts ? &sh : nullptr, c->stream);
  // the lift deposits the new ions' charge into the next buffer as it writes them
  if (c->lift_deposit) deposit_into_next(c);
  launch_lift_particles(c->d_reps, c->d_block_prefix, c->R, c->total_blocks, -1, d_coarse,
                        c->d_coarse_off, nullptr, c->grid_blocks, c->stream,
                        c->lift_deposit ? c->cur ^ 1 : -1, c->d_status, c->moments == 3);
  if (c->kinetic) {
    load_boltzmann_electrons(c);
    mark_new_electrons(c);
  }
  mark_new_particles(c);
  if (c->lift_deposit) {
    c->cur ^= 1;
    c->other_zero = false;
    c->deposited = true;
  }
  return hip_check("lift");
}

hipEvent_t next_event(efpi_ctx* c) {
  if (c->events_used == c->events.size()) {
    hipEvent_t e = nullptr;
    // timing only: no system-scope fence (no cache writeback at the event, which
    // would add to the measured interval and slow the following launch)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    c->events.push_back(e);
  }
  return c->events[c->events_used++];
}

efpi_status do_burst(efpi_ctx* c, int steps, bool restrict_) {
  if (!c->field_valid) {
    if (!c->deposited) deposit_all(c, true);
    // the first solve of a context starts from phi = ln max(rho, 1e-8) (its stored
    // phi is zero, far from the solution where the density vanishes) and takes
    // kColdIters iterations: near a plasma edge the vacuum guess lies 10 and more
    // below the solution, and each Newton correction is clamped to 2
    run_field(c, c->phi_valid ? c->cfg.newton_iters_start : std::max(c->cfg.newton_iters_start, kColdIters),
              c->phi_valid ? 0 : 1, restrict_ ? 1 : 0, restrict_ ? 1 : 0);
  } else if (restrict_) {
    launch_prep_burst(c->d_reps, c->R, c->stream);
  }
  const int passes = restrict_ ? steps + 1 : steps;
  for (int p = 0; p < passes; ++p) {
    const bool push = p < steps;
    int flags = 0;
    if (p == 0 && c->fresh) flags |= kFresh;
    if (restrict_) flags |= kRestrict | (c->moments == 3 ? kMoment3 : 0);
    if (push) {
      flags |= kPush;
      deposit_into_next(c);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing && push) {
      e0 = next_event(c);
      e1 = next_event(c);
      if (e0 && e1) c->ion_pairs.push_back({c->events_used - 2, c->events_used - 1});
    }
    launch_particles(c->d_reps, c->d_item_prefix, c->R, c->total_items, c->tile, c->grid_blocks, p,
                     flags, c->cur ^ 1, c->d_status, c->stream, e0, e1);
    if (push) {
      if (c->kinetic) {
        hipEvent_t f0 = nullptr, f1 = nullptr;
        if (c->timing) {
          f0 = next_event(c);
          f1 = next_event(c);
          if (f0 && f1) c->el_pairs.push_back({c->events_used - 2, c->events_used - 1});
        }
        launch_electrons(c->d_ereps, c->R, 1, (p == 0 && c->fresh_e) ? 1 : 0, c->cur ^ 1,
                         c->max_nodes, c->stream, f0, f1);
      }
      c->cur ^= 1;
      c->other_zero = false;
      c->fresh = false;
      c->fresh_e = false;
      run_field(c, c->cfg.newton_iters, 0, 0, 0);
    }
  }
  if (steps > 0) {
    c->fresh = false;
    c->fresh_e = false;
  }
  if (restrict_) c->last_burst_steps = steps;
  return hip_check("pic_burst");
}

}  // namespace

extern "C" {

efpi_status efpi_workspace_size(const efpi_config* cfg, size_t* h_bytes) {
  const efpi_status st = check_config(cfg);
  if (st != EFPI_OK) return st;
  if (!h_bytes) return fail(EFPI_EINVAL, "h_bytes is NULL");
  *h_bytes = layout(cfg, nullptr, nullptr);
  return EFPI_OK;
}

efpi_status efpi_init(const efpi_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                      efpi_ctx** out) {
  efpi_status st = check_config(cfg);
  if (st != EFPI_OK) return st;
  if (!out) return fail(EFPI_EINVAL, "out is NULL");
  if (!d_workspace) return fail(EFPI_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
    return fail(EFPI_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = layout(cfg, nullptr, nullptr);
  if (bytes < need) return fail(EFPI_ENOMEM, "workspace smaller than efpi_workspace_size");
  void* scratch_ptr = nullptr;
  st = scratch_of_current_device(&scratch_ptr);
  if (st != EFPI_OK) return st;
  efpi_ctx* c = new efpi_ctx();
  c->scratch = scratch_ptr;
  c->cfg = *cfg;
  c->R = (int)cfg->n_replicas;
  c->reps.assign(cfg->replicas, cfg->replicas + c->R);
  c->cfg.replicas = c->reps.data();
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<uint8_t*>(d_workspace);
  c->ws_bytes = bytes;
  c->tile = cfg->tile > 0 ? cfg->tile : kDefaultTile;
  layout(&c->cfg, c, c->ws);
  // work items
  c->h_item_prefix.assign(c->R + 1, 0);
  c->h_block_prefix.assign(c->R + 1, 0);
  c->h_snap_off.assign(c->R, 0);
  c->h_coarse_off.assign(c->R, 0);
  int64_t so = 0, co = 0;
  for (int r = 0; r < c->R; ++r) {
    RepDev& d = c->h_reps[r];
    d.item_begin = c->h_item_prefix[r];
    d.block_begin = c->h_block_prefix[r];
    c->h_item_prefix[r + 1] = c->h_item_prefix[r] + (d.capacity + c->tile - 1) / c->tile;
    c->h_block_prefix[r + 1] = c->h_block_prefix[r] + d.n_coarse;
    c->h_snap_off[r] = so;
    c->h_coarse_off[r] = co;
    so += (int64_t)(d.burst_steps + 1) * d.moments * d.n_coarse;
    co += d.moments * d.n_coarse;
  }
  c->total_items = c->h_item_prefix[c->R];
  if (c->kinetic) {
    c->h_eitem_prefix.assign(c->R + 1, 0);
    for (int r = 0; r < c->R; ++r) {
      RepDev& el = c->h_ereps[r];
      // the lift finds a replica's coarse blocks by the ions' block numbering
      el.block_begin = c->h_reps[r].block_begin;
      el.item_begin = c->h_eitem_prefix[r];
      c->h_eitem_prefix[r + 1] = c->h_eitem_prefix[r] + (el.capacity + c->tile - 1) / c->tile;
    }
    c->total_eitems = c->h_eitem_prefix[c->R];
  }
  c->total_blocks = c->h_block_prefix[c->R];
  c->grid_blocks = cfg->grid_blocks;  // 0: one workgroup per work item
  // ensemble groups: replicas with equal (n_cells, length) share the first one's index
  c->h_group.assign(c->R, 0);
  for (int r = 0; r < c->R; ++r) {
    c->h_group[r] = r;
    for (int q = 0; q < r; ++q)
      if (c->reps[q].n_cells == c->reps[r].n_cells && c->reps[q].length == c->reps[r].length) {
        c->h_group[r] = c->h_group[q];
        break;
      }
  }
  // clear the workspace, then upload descriptors and tables
  launch_fill_u8(c->ws, need, c->stream);
  note(hipMemcpyAsync(c->d_reps, c->h_reps.data(), sizeof(RepDev) * c->R, hipMemcpyHostToDevice, c->stream));
  note(hipMemcpyAsync(c->d_item_prefix, c->h_item_prefix.data(), sizeof(int64_t) * (c->R + 1),
                 hipMemcpyHostToDevice, c->stream));
  note(hipMemcpyAsync(c->d_block_prefix, c->h_block_prefix.data(), sizeof(int64_t) * (c->R + 1),
                 hipMemcpyHostToDevice, c->stream));
  note(hipMemcpyAsync(c->d_snap_off, c->h_snap_off.data(), sizeof(int64_t) * c->R, hipMemcpyHostToDevice,
                 c->stream));
  note(hipMemcpyAsync(c->d_coarse_off, c->h_coarse_off.data(), sizeof(int64_t) * c->R,
                 hipMemcpyHostToDevice, c->stream));
  note(hipMemcpyAsync(c->d_group, c->h_group.data(), sizeof(int32_t) * c->R, hipMemcpyHostToDevice,
                 c->stream));
  for (int r = 0; r < c->R; ++r) c->max_nodes = std::max(c->max_nodes, c->h_reps[r].n_nodes);
  if (c->kinetic) {
    note(hipMemcpyAsync(c->d_ereps, c->h_ereps.data(), sizeof(RepDev) * c->R,
                        hipMemcpyHostToDevice, c->stream));
    note(hipMemcpyAsync(c->d_eitem_prefix, c->h_eitem_prefix.data(), sizeof(int64_t) * (c->R + 1),
                        hipMemcpyHostToDevice, c->stream));
  }
  const hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete c;
    return fail(EFPI_EHIP, std::string("init: ") + hipGetErrorString(e));
  }
  st = hip_check("init");
  if (st != EFPI_OK) {
    delete c;
    return st;
  }
  *out = c;
  return EFPI_OK;
}

void efpi_destroy(efpi_ctx* ctx) { delete ctx; }

efpi_status efpi_set_stream(efpi_ctx* ctx, void* hip_stream) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return EFPI_OK;
}

efpi_status efpi_n_coarse(efpi_ctx* ctx, int32_t replica, int32_t* h_nc) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  if (!h_nc) return fail(EFPI_EINVAL, "h_nc is NULL");
  *h_nc = ctx->h_reps[replica].n_coarse;
  return EFPI_OK;
}

efpi_status efpi_set_particles(efpi_ctx* ctx, int32_t replica, const int16_t* d_cell,
                               const float* d_frac, const float* d_v, const float* d_w, int64_t n) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  if (n < 0 || n > ctx->h_reps[replica].capacity) return fail(EFPI_EINVAL, "n out of [0, capacity]");
  if (n > 0 && (!d_cell || !d_frac || !d_v || !d_w)) return fail(EFPI_EINVAL, "NULL particle array");
  launch_copy_particles(ctx->d_reps, replica, d_cell, d_frac, d_v, d_w, n, 1, nullptr, nullptr,
                        nullptr, nullptr, ctx->stream);
  mark_new_particles(ctx);
  return hip_check("set_particles");
}

efpi_status efpi_get_particles(efpi_ctx* ctx, int32_t replica, int16_t* d_cell, float* d_frac,
                               float* d_v, float* d_w, int64_t* h_n) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  const RepDev& d = ctx->h_reps[replica];
  launch_copy_particles(ctx->d_reps, replica, nullptr, nullptr, nullptr, nullptr, d.capacity, 0,
                        d_cell, d_frac, d_v, d_w, ctx->stream);
  int64_t n = 0;
  note(hipMemcpyAsync(&n, d.np, sizeof n, hipMemcpyDeviceToHost, ctx->stream));
  const hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(EFPI_EHIP, std::string("get_particles: ") + hipGetErrorString(e));
  if (h_n) *h_n = n;
  return hip_check("get_particles");
}

efpi_status efpi_get_grid(efpi_ctx* ctx, int32_t replica, int64_t* d_q, double* d_phi, float* d_e) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  const RepDev& d = ctx->h_reps[replica];
  if (d_q) note(hipMemcpyAsync(d_q, d.q[ctx->cur], sizeof(int64_t) * d.n_nodes, hipMemcpyDeviceToDevice, ctx->stream));
  if (d_phi) launch_phi_copy(ctx->d_reps, replica, d.phi, d_phi, 1, ctx->stream);
  if (d_e) note(hipMemcpyAsync(d_e, d.e, sizeof(float) * d.n_nodes, hipMemcpyDeviceToDevice, ctx->stream));
  return hip_check("get_grid");
}

efpi_status efpi_set_potential(efpi_ctx* ctx, int32_t replica, const double* d_phi) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  if (!d_phi) return fail(EFPI_EINVAL, "d_phi is NULL");
  const RepDev& d = ctx->h_reps[replica];
  launch_phi_copy(ctx->d_reps, replica, d_phi, d.phi, 0, ctx->stream);
  ctx->field_valid = false;
  ctx->phi_valid = true;
  return hip_check("set_potential");
}

efpi_status efpi_load_profile(efpi_ctx* ctx, int32_t replica, const double* d_n, const double* d_u,
                              uint32_t shift) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  if (!d_n || !d_u) return fail(EFPI_EINVAL, "NULL profile");
  launch_set_profile(ctx->d_reps, replica, d_n, d_u, ctx->stream);
  launch_occupancy(ctx->d_reps, ctx->R, replica, ctx->d_status, ctx->stream);
  ShiftArg s;
  std::memset(&s, 0, sizeof s);
  s.s[replica] = shift;
  launch_lift_particles(ctx->d_reps, ctx->d_block_prefix, ctx->R, ctx->h_reps[replica].n_coarse,
                        replica, nullptr, ctx->d_coarse_off, &s, ctx->grid_blocks, ctx->stream);
  mark_new_particles(ctx);
  return hip_check("load_profile");
}

efpi_status efpi_set_electrons(efpi_ctx* ctx, int32_t replica, const int16_t* d_cell,
                               const float* d_frac, const float* d_v, const float* d_w,
                               int64_t n) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  if (!ctx->kinetic) return fail(EFPI_ESTATE, "the context has no kinetic electrons");
  if (!d_cell || !d_frac || !d_v || !d_w) return fail(EFPI_EINVAL, "NULL array");
  if (n < 0 || n > ctx->h_ereps[replica].capacity) return fail(EFPI_EINVAL, "n out of [0, capacity_e]");
  launch_copy_particles(ctx->d_ereps, replica, d_cell, d_frac, d_v, d_w, n, 1, nullptr, nullptr,
                        nullptr, nullptr, ctx->stream);
  mark_new_electrons(ctx);
  return hip_check("set_electrons");
}

efpi_status efpi_get_electrons(efpi_ctx* ctx, int32_t replica, int16_t* d_cell, float* d_frac,
                               float* d_v, float* d_w, int64_t* h_n) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  if (!ctx->kinetic) return fail(EFPI_ESTATE, "the context has no kinetic electrons");
  const RepDev& d = ctx->h_ereps[replica];
  launch_copy_particles(ctx->d_ereps, replica, nullptr, nullptr, nullptr, nullptr, d.capacity, 0,
                        d_cell, d_frac, d_v, d_w, ctx->stream);
  int64_t n = 0;
  note(hipMemcpyAsync(&n, d.np, sizeof n, hipMemcpyDeviceToHost, ctx->stream));
  const hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(EFPI_EHIP, std::string("get_electrons: ") + hipGetErrorString(e));
  if (h_n) *h_n = n;
  return hip_check("get_electrons");
}

efpi_status efpi_load_electrons(efpi_ctx* ctx, int32_t replica, const double* d_n,
                                const double* d_u, uint32_t shift) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  if (!ctx->kinetic) return fail(EFPI_ESTATE, "the context has no kinetic electrons");
  if (!d_n || !d_u) return fail(EFPI_EINVAL, "NULL profile");
  launch_set_profile(ctx->d_ereps, replica, d_n, d_u, ctx->stream);
  launch_occupancy(ctx->d_ereps, ctx->R, replica, ctx->d_status, ctx->stream);
  ShiftArg s;
  std::memset(&s, 0, sizeof s);
  s.s[replica] = shift;
  launch_lift_particles(ctx->d_ereps, ctx->d_block_prefix, ctx->R,
                        ctx->h_reps[replica].n_coarse, replica, nullptr, ctx->d_coarse_off, &s,
                        ctx->grid_blocks, ctx->stream);
  mark_new_electrons(ctx);
  return hip_check("load_electrons");
}

efpi_status efpi_boltzmann_electrons(efpi_ctx* ctx, const uint32_t* h_shifts) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!ctx->kinetic) return fail(EFPI_ESTATE, "the context has no kinetic electrons");
  if (!h_shifts) return fail(EFPI_EINVAL, "h_shifts is NULL");
  if (!ctx->fresh) return fail(EFPI_ESTATE, "load electrons with the ions at an integer time level");
  // the ions' rotation slot carries the rotation the electron profile derives from
  launch_set_shifts(ctx->d_reps, ctx->R, -1, shifts_of(ctx, h_shifts), ctx->stream);
  load_boltzmann_electrons(ctx);
  mark_new_electrons(ctx);
  return hip_check("boltzmann_electrons");
}

efpi_status efpi_reset_electrons(efpi_ctx* ctx, const uint32_t* h_shifts) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!ctx->kinetic) return fail(EFPI_ESTATE, "the context has no kinetic electrons");
  if (!h_shifts) return fail(EFPI_EINVAL, "h_shifts is NULL");
  if (!ctx->fresh && !ctx->field_valid)
    return fail(EFPI_ESTATE, "reset_electrons after a burst needs the current field");
  launch_set_shifts(ctx->d_reps, ctx->R, -1, shifts_of(ctx, h_shifts), ctx->stream);
  // ion momentum with time-centred velocities, from the current field
  for (int r = 0; r < ctx->R; ++r)
    launch_fill_u8(ctx->h_reps[r].jfx, sizeof(int64_t) * ctx->h_reps[r].n_nodes, ctx->stream);
  launch_ion_momentum(ctx->d_reps, ctx->R, ctx->fresh ? 0 : 1, ctx->max_nodes, ctx->stream);
  // ion charge (kept in q[cur] through the Newton solve), eq. 3.15, profile, load
  deposit_all(ctx, false);
  run_newton(ctx, ctx->cfg.newton_iters_start, 1, 0, 0);
  launch_electron_profile(ctx->d_reps, ctx->d_ereps, ctx->R, 1, ctx->cur, ctx->stream);
  launch_occupancy(ctx->d_ereps, ctx->R, -1, ctx->d_status, ctx->stream);
  launch_lift_particles(ctx->d_ereps, ctx->d_block_prefix, ctx->R, ctx->total_blocks, -1, nullptr,
                        ctx->d_coarse_off, nullptr, ctx->grid_blocks, ctx->stream);
  mark_new_electrons(ctx);
  return hip_check("reset_electrons");
}

efpi_status efpi_lift(efpi_ctx* ctx, const double* d_coarse, const uint32_t* h_shifts) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_coarse) return fail(EFPI_EINVAL, "d_coarse is NULL");
  if (!h_shifts) return fail(EFPI_EINVAL, "h_shifts is NULL");
  return do_lift(ctx, d_coarse, h_shifts);
}

efpi_status efpi_deposit(efpi_ctx* ctx) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  deposit_all(ctx, true);
  return hip_check("deposit");
}

efpi_status efpi_solve_field(efpi_ctx* ctx, int32_t iters, int32_t cold) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (iters < 1 || iters > 1000) return fail(EFPI_EINVAL, "iters must be in [1, 1000]");
  if (!ctx->deposited) return fail(EFPI_ESTATE, "solve_field needs a deposit of the current particles");
  run_field(ctx, iters, cold ? 1 : 0, 0, 0);
  return hip_check("solve_field");
}

efpi_status efpi_pic_burst(efpi_ctx* ctx, int32_t steps, int32_t restrict_) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (steps < 0) return fail(EFPI_EINVAL, "steps must be >= 0");
  if (restrict_) {
    for (int r = 0; r < ctx->R; ++r)
      if (steps > ctx->h_reps[r].burst_steps)
        return fail(EFPI_EINVAL, "restricting burst longer than burst_steps");
  }
  return do_burst(ctx, steps, restrict_ != 0);
}

efpi_status efpi_restrict(efpi_ctx* ctx, double* d_snap) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_snap) return fail(EFPI_EINVAL, "d_snap is NULL");
  if (ctx->last_burst_steps < 0) return fail(EFPI_ESTATE, "no restricting burst has run");
  launch_restrict(ctx->d_reps, ctx->R, ctx->last_burst_steps, d_snap, ctx->d_snap_off, ctx->stream);
  return hip_check("restrict");
}

efpi_status efpi_project(efpi_ctx* ctx, const double* d_snap, double* d_coarse_next) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_snap || !d_coarse_next) return fail(EFPI_EINVAL, "NULL array");
  launch_project(ctx->d_reps, ctx->R, d_snap, ctx->d_snap_off, d_coarse_next, ctx->d_coarse_off,
                 ctx->d_status, ctx->stream);
  return hip_check("project");
}

efpi_status efpi_macro_step(efpi_ctx* ctx, const double* d_coarse_in, double* d_coarse_out,
                            const uint32_t* h_shifts) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_coarse_in || !d_coarse_out || !h_shifts) return fail(EFPI_EINVAL, "NULL argument");
  int k = ctx->h_reps[0].burst_steps;
  for (int r = 1; r < ctx->R; ++r)
    if (ctx->h_reps[r].burst_steps != k)
      return fail(EFPI_EINVAL, "macro_step needs equal burst_steps in every replica");
  efpi_status st = do_lift(ctx, d_coarse_in, h_shifts);
  if (st != EFPI_OK) return st;
  st = do_burst(ctx, k, true);
  if (st != EFPI_OK) return st;
  launch_restrict_project(ctx->d_reps, ctx->R, ctx->d_snap, ctx->d_snap_off, d_coarse_out,
                          ctx->d_coarse_off, ctx->d_status, ctx->stream);
  return hip_check("macro_step");
}

efpi_status efpi_macro_step_graph(efpi_ctx* ctx, const double* d_coarse_in, double* d_coarse_out,
                                  const uint32_t* h_shifts) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_coarse_in || !d_coarse_out || !h_shifts) return fail(EFPI_EINVAL, "NULL argument");
  if (!ctx->stream) return fail(EFPI_ESTATE, "graph capture needs a non-null stream");
  if (ctx->timing) return fail(EFPI_ESTATE, "disable timing before using captured macro steps");
  const int k = ctx->h_reps[0].burst_steps;
  for (int r = 1; r < ctx->R; ++r)
    if (ctx->h_reps[r].burst_steps != k)
      return fail(EFPI_EINVAL, "macro_step needs equal burst_steps in every replica");
  // the rotations change every step: they are stored outside the graph
  launch_set_shifts(ctx->d_reps, ctx->R, -1, shifts_of(ctx, h_shifts), ctx->stream);
  efpi_ctx::MacroGraph* g = nullptr;
  for (efpi_ctx::MacroGraph& m : ctx->graphs)
    if (m.in == d_coarse_in && m.out == d_coarse_out && m.cur0 == ctx->cur &&
        m.other_zero0 == ctx->other_zero && m.phi_valid0 == ctx->phi_valid)
      g = &m;
  if (!g) {
    const efpi_ctx::HostState before = ctx->state();
    efpi_ctx::MacroGraph m{d_coarse_in, d_coarse_out, ctx->cur, ctx->other_zero,
                           ctx->phi_valid, before, nullptr};
    hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return fail(EFPI_EHIP, std::string("begin capture: ") + hipGetErrorString(e));
    // the same launches as efpi_macro_step, lift rotations read from the device
    efpi_status st = do_lift(ctx, d_coarse_in, nullptr);
    if (st == EFPI_OK) st = do_burst(ctx, k, true);
    launch_restrict_project(ctx->d_reps, ctx->R, ctx->d_snap, ctx->d_snap_off, d_coarse_out,
                            ctx->d_coarse_off, ctx->d_status, ctx->stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->stream, &graph);
    m.after = ctx->state();
    ctx->set_state(before);  // nothing has run yet
    if (e == hipSuccess && st == EFPI_OK) e = hipGraphInstantiate(&m.exec, graph, nullptr, nullptr, 0);
    if (graph) note(hipGraphDestroy(graph));
    if (st != EFPI_OK) return st;
    if (e != hipSuccess) return fail(EFPI_EHIP, std::string("capture: ") + hipGetErrorString(e));
    if (ctx->graphs.size() >= kMaxGraphs) {  // keep the cache bounded: drop the oldest
      note(hipStreamSynchronize(ctx->stream));  // it may still be running
      note(hipGraphExecDestroy(ctx->graphs.front().exec));
      ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(m);
    g = &ctx->graphs.back();
  }
  const hipError_t e = hipGraphLaunch(g->exec, ctx->stream);
  if (e != hipSuccess) return fail(EFPI_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
  ctx->set_state(g->after);
  return hip_check("macro_step_graph");
}

namespace {
efpi_status check_phase(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph) {
  if (check_rep(ctx, replica) != EFPI_OK) return EFPI_EINVAL;
  if (!ph) return fail(EFPI_EINVAL, "phase parameters are NULL");
  const RepDev& d = ctx->h_reps[replica];
  if (d.bc != EFPI_BC_PERIODIC) return fail(EFPI_EINVAL, "phase restriction needs a periodic replica");
  if (!(ph->v_max > ph->v_min) || !std::isfinite(ph->v_min) || !std::isfinite(ph->v_max))
    return fail(EFPI_EINVAL, "need finite v_min < v_max");
  // jf = 11 fills 64 KB of LDS with the histogram window (four x nodes x 2^11 int64)
  if (ph->jf < 4 || ph->jf > 11) return fail(EFPI_EINVAL, "jf must be in [4, 11]");
  if (ph->jc < 1 || ph->jc > ph->jf) return fail(EFPI_EINVAL, "jc must be in [1, jf]");
  if (ph->n_taps < 2 || ph->n_taps > 16 || (ph->n_taps & 1))
    return fail(EFPI_EINVAL, "n_taps must be even in [2, 16]");
  if ((1 << ph->jc) < ph->n_taps) return fail(EFPI_EINVAL, "2^jc must be >= n_taps");
  if (ph->levels < 0 || (d.n_cells >> ph->levels) < 1)
    return fail(EFPI_EINVAL, "levels out of range");
  // A coarse bin sums at most 2^(levels+1) cells' charge with weights up to
  // 2^levels: with node densities up to 16 that is below 2^40 * 16 * 2 h 4^levels,
  // which must stay below 2^63 for the int64 histogram.
  if (std::ldexp(d.h, 2 * ph->levels) >= 262144.0)
    return fail(EFPI_EINVAL, "h * 4^levels must be below 2^18 (int64 phase histogram range)");
  for (int m = 0; m < ph->n_taps; ++m)
    if (!std::isfinite(ph->taps[m])) return fail(EFPI_EINVAL, "non-finite filter tap");
  return EFPI_OK;
}
}  // namespace

efpi_status efpi_phase_work_size(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                                 size_t* h_bytes) {
  const efpi_status st = check_phase(ctx, replica, ph);
  if (st != EFPI_OK) return st;
  if (!h_bytes) return fail(EFPI_EINVAL, "h_bytes is NULL");
  *h_bytes = sizeof(int64_t) * (size_t)(ctx->h_reps[replica].n_cells >> ph->levels) *
             ((size_t)1 << ph->jf);
  return EFPI_OK;
}

efpi_status efpi_phase_restrict(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                                double tau, int32_t stored_field, void* d_work, double* d_out) {
  const efpi_status st = check_phase(ctx, replica, ph);
  if (st != EFPI_OK) return st;
  if (!d_work || !d_out) return fail(EFPI_EINVAL, "NULL array");
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return fail(EFPI_EINVAL, "d_work must be 256-byte aligned");
  if (!std::isfinite(tau)) return fail(EFPI_EINVAL, "tau must be finite");
  if (!ctx->fresh && !ctx->field_valid)
    return fail(EFPI_ESTATE, "phase restriction after a burst needs the current field");
  if (tau != 0.0 && !stored_field && !ctx->field_valid)
    return fail(EFPI_ESTATE, "the co-evolving frame (tau != 0) needs the current field");
  const RepDev& d = ctx->h_reps[replica];
  launch_phase_restrict(ctx->d_reps, replica, d.n_cells, ph->levels, ph->v_min, ph->v_max, ph->jf,
                        ph->jc, ph->taps, ph->n_taps, tau, ctx->fresh ? 1 : 0,
                        stored_field ? 1 : 0, d.h, static_cast<long long*>(d_work), d_out,
                        ctx->stream);
  return hip_check("phase_restrict");
}

efpi_status efpi_phase_restrict_static(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                                       double tau, int32_t stored_field, double* d_out) {
  size_t need = 0;
  const efpi_status st = efpi_phase_work_size(ctx, replica, ph, &need);
  if (st != EFPI_OK) return st;
  if (need > EFPI_STATIC_SCRATCH_BYTES)
    return fail(EFPI_EINVAL, "histogram of " + std::to_string(need) +
                                 " bytes exceeds the static scratch (" +
                                 std::to_string(EFPI_STATIC_SCRATCH_BYTES) + " bytes)");
  if (!ctx->scratch) return fail(EFPI_ESTATE, "no static scratch on this context's device");
  // the same checks and kernels as with a caller's work buffer; the histogram
  // fill at its start clears what the previous call left in the array
  return efpi_phase_restrict(ctx, replica, ph, tau, stored_field, ctx->scratch, d_out);
}

namespace {
size_t phase_lift_cols_bytes(const RepDev& d, const efpi_phase* ph) {
  return align256(sizeof(double) * (size_t)(d.n_cells >> ph->levels) * ((size_t)1 << ph->jf));
}
size_t phase_lift_cdf_bytes(const RepDev& d, const efpi_phase* ph) {
  return align256(sizeof(double) * (((size_t)1 << ph->jf) + 1) * (size_t)d.n_cells);
}
}  // namespace

efpi_status efpi_phase_lift_work_size(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                                      size_t* h_bytes) {
  const efpi_status st = check_phase(ctx, replica, ph);
  if (st != EFPI_OK) return st;
  if (!h_bytes) return fail(EFPI_EINVAL, "h_bytes is NULL");
  const RepDev& d = ctx->h_reps[replica];
  *h_bytes = phase_lift_cols_bytes(d, ph) + phase_lift_cdf_bytes(d, ph);
  return EFPI_OK;
}

efpi_status efpi_phase_lift(efpi_ctx* ctx, int32_t replica, const efpi_phase* ph,
                            const double* d_coarse, uint32_t shift, void* d_work) {
  const efpi_status st = check_phase(ctx, replica, ph);
  if (st != EFPI_OK) return st;
  if (!d_coarse || !d_work) return fail(EFPI_EINVAL, "NULL array");
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return fail(EFPI_EINVAL, "d_work must be 256-byte aligned");
  const RepDev& d = ctx->h_reps[replica];
  uint8_t* w = static_cast<uint8_t*>(d_work);
  double* cols = reinterpret_cast<double*>(w);
  double* cdf = reinterpret_cast<double*>(w + phase_lift_cols_bytes(d, ph));
  launch_phase_lift(ctx->d_reps, replica, d.n_cells, ph->levels, ph->v_min, ph->v_max, ph->jf,
                    ph->jc, ph->taps, ph->n_taps, d_coarse, cols, cdf, ctx->d_status, shift,
                    ctx->stream);
  mark_new_particles(ctx);
  return hip_check("phase_lift");
}

efpi_status efpi_phase_project(efpi_ctx* ctx, const double* d_snap, int64_t count,
                               int32_t snapshots, double dt, double macro_dt, double* d_out) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_snap || !d_out) return fail(EFPI_EINVAL, "NULL array");
  if (count < 1 || snapshots < 2) return fail(EFPI_EINVAL, "need count >= 1 and snapshots >= 2");
  if (!(dt > 0.0) || !(macro_dt >= (snapshots - 1) * dt * (1.0 - 1e-12)))
    return fail(EFPI_EINVAL, "need dt > 0 and macro_dt >= (snapshots - 1) dt");
  launch_phase_project(d_snap, count, snapshots - 1, dt, macro_dt, d_out, ctx->stream);
  return hip_check("phase_project");
}

efpi_status efpi_store_field(efpi_ctx* ctx) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!ctx->field_valid) {
    if (!ctx->deposited) deposit_all(ctx, true);
    run_field(ctx, ctx->phi_valid ? ctx->cfg.newton_iters_start
                                  : std::max(ctx->cfg.newton_iters_start, kColdIters),
              ctx->phi_valid ? 0 : 1, 1, 0);
  } else {
    launch_prep_burst(ctx->d_reps, ctx->R, ctx->stream);
  }
  return hip_check("store_field");
}

efpi_status efpi_restrict_state(efpi_ctx* ctx, double* d_coarse) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_coarse) return fail(EFPI_EINVAL, "d_coarse is NULL");
  if (!ctx->fresh && !ctx->field_valid)
    return fail(EFPI_ESTATE, "restrict_state needs integer-time velocities or a current field");
  launch_prep_burst(ctx->d_reps, ctx->R, ctx->stream);
  launch_particles(ctx->d_reps, ctx->d_item_prefix, ctx->R, ctx->total_items, ctx->tile,
                   ctx->grid_blocks, -1,
                   kRestrict | (ctx->fresh ? kFresh : 0) | (ctx->moments == 3 ? kMoment3 : 0),
                   ctx->cur ^ 1,
                   ctx->d_status, ctx->stream);
  launch_restrict(ctx->d_reps, ctx->R, 0, d_coarse, ctx->d_coarse_off, ctx->stream);
  ctx->last_burst_steps = -1;
  return hip_check("restrict_state");
}

efpi_status efpi_next_macro_dt(double macro_dt, double err, double tol, double dt_min,
                               double dt_max, double safety, double* h_next) {
  if (!h_next) return fail(EFPI_EINVAL, "h_next is NULL");
  const double v[] = {macro_dt, err, tol, dt_min, dt_max, safety};
  for (double x : v)
    if (!std::isfinite(x)) return fail(EFPI_EINVAL, "non-finite argument");
  if (!(macro_dt > 0.0) || !(tol > 0.0) || !(safety > 0.0) || err < 0.0 || !(dt_min > 0.0) ||
      dt_min > dt_max)
    return fail(EFPI_EINVAL, "need macro_dt, tol, safety > 0, err >= 0, 0 < dt_min <= dt_max");
  // the Euler step's local error grows as Delta t^2: the step that meets tol is
  // Delta t (tol / err)^{1/2}; a safety factor, at most a doubling or a halving
  const double grow = err == 0.0 ? 2.0 : std::min(2.0, std::max(0.5, safety * std::sqrt(tol / err)));
  *h_next = std::min(dt_max, std::max(dt_min, macro_dt * grow));
  return EFPI_OK;
}

efpi_status efpi_set_macro_dt(efpi_ctx* ctx, double macro_dt) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!std::isfinite(macro_dt)) return fail(EFPI_EINVAL, "macro_dt must be finite");
  for (int r = 0; r < ctx->R; ++r) {
    const efpi_replica& p = ctx->reps[r];
    if (!(macro_dt >= p.burst_steps * p.dt * (1.0 - 1e-12)))
      return fail(EFPI_EINVAL, "macro_dt must be >= burst_steps * dt of every replica");
  }
  for (int r = 0; r < ctx->R; ++r) {
    ctx->reps[r].macro_dt = macro_dt;
    ctx->h_reps[r].macro_dt = macro_dt;
  }
  for (RepDev& d : ctx->h_ereps) d.macro_dt = macro_dt;
  if (ctx->kinetic)
    note(hipMemcpyAsync(ctx->d_ereps, ctx->h_ereps.data(), sizeof(RepDev) * ctx->R,
                        hipMemcpyHostToDevice, ctx->stream));
  // kernels (and captured graphs) read the descriptors on the device when they run,
  // so the new step takes effect for the work enqueued after this call
  note(hipMemcpyAsync(ctx->d_reps, ctx->h_reps.data(), sizeof(RepDev) * ctx->R,
                      hipMemcpyHostToDevice, ctx->stream));
  // the host copies must outlive the asynchronous copies above
  note(hipStreamSynchronize(ctx->stream));
  return hip_check("set_macro_dt");
}

efpi_status efpi_project2(efpi_ctx* ctx, const double* d_snap, const double* d_slope_prev,
                          double gap, double* d_slope, double* d_euler, double* d_coarse_next) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_snap || !d_slope || !d_coarse_next) return fail(EFPI_EINVAL, "NULL array");
  if (d_slope_prev && !(gap > 0.0 && std::isfinite(gap)))
    return fail(EFPI_EINVAL, "gap must be finite and > 0 with a previous slope");
  launch_project2(ctx->d_reps, ctx->R, d_snap, ctx->d_snap_off, d_slope_prev, gap, d_slope,
                  d_euler, d_coarse_next, ctx->d_coarse_off, ctx->d_status, ctx->stream);
  return hip_check("project2");
}

efpi_status efpi_ensemble_mean(efpi_ctx* ctx, double* d_coarse) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!d_coarse) return fail(EFPI_EINVAL, "d_coarse is NULL");
  launch_ensemble_mean(ctx->d_reps, ctx->R, ctx->d_group, d_coarse, ctx->d_coarse_off, ctx->stream);
  return hip_check("ensemble_mean");
}

efpi_status efpi_sort(efpi_ctx* ctx) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!(ctx->cfg.flags & EFPI_FLAG_SORT_BUFFER))
    return fail(EFPI_ESTATE, "efpi_sort needs EFPI_FLAG_SORT_BUFFER at init");
  launch_sort(ctx->d_reps, ctx->d_item_prefix, ctx->R, ctx->total_items, ctx->tile,
              ctx->d_sort_hist, ctx->d_sort_base, ctx->grid_blocks, ctx->stream);
  if (ctx->kinetic)
    launch_sort(ctx->d_ereps, ctx->d_eitem_prefix, ctx->R, ctx->total_eitems, ctx->tile,
                ctx->d_sort_hist, ctx->d_sort_base, ctx->grid_blocks, ctx->stream);
  return hip_check("sort");
}

efpi_status efpi_sync(efpi_ctx* ctx, uint32_t* h_bits) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  uint32_t bits = 0;
  hipError_t e = hipMemcpyAsync(&bits, ctx->d_status, sizeof bits, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(EFPI_EHIP, std::string("sync: ") + hipGetErrorString(e));
  launch_fill_u8(ctx->d_status, sizeof(uint32_t), ctx->stream);
  e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(EFPI_EHIP, std::string("sync: ") + hipGetErrorString(e));
  if (h_bits) *h_bits = bits;
  if (bits & EFPI_DEV_NAN) return fail(EFPI_ENUMERIC, "non-finite potential or coarse value");
  if (bits & EFPI_DEV_NEWTON) return fail(EFPI_ENEWTON, "Newton iteration above tolerance");
  if (bits & EFPI_DEV_OVERFLOW) return fail(EFPI_EOVERFLOW, "particle capacity exceeded at lift");
  g_err.clear();
  return EFPI_OK;
}

efpi_status efpi_timing(efpi_ctx* ctx, int32_t enable) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  ctx->timing = enable != 0;
  ctx->events_used = 0;
  ctx->ion_pairs.clear();
  ctx->el_pairs.clear();
  return EFPI_OK;
}

namespace {
// Sum the intervals of the given event pairs and forget them; the event pool is
// reused once neither list holds pairs.
efpi_status read_pairs(efpi_ctx* ctx, std::vector<std::pair<size_t, size_t>>& pairs,
                       double* h_total_ms, int64_t* h_launches) {
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(EFPI_EHIP, std::string("timing_read: ") + hipGetErrorString(e));
  double total = 0.0;
  for (const auto& pr : pairs) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ctx->events[pr.first], ctx->events[pr.second]);
    if (e != hipSuccess) return fail(EFPI_EHIP, std::string("timing_read: ") + hipGetErrorString(e));
    total += ms;
  }
  const int64_t n = (int64_t)pairs.size();
  pairs.clear();
  if (ctx->ion_pairs.empty() && ctx->el_pairs.empty()) ctx->events_used = 0;
  if (h_total_ms) *h_total_ms = total;
  if (h_launches) *h_launches = n;
  return EFPI_OK;
}
}  // namespace

efpi_status efpi_timing_read(efpi_ctx* ctx, double* h_total_ms, int64_t* h_launches) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  return read_pairs(ctx, ctx->ion_pairs, h_total_ms, h_launches);
}

efpi_status efpi_timing_read_electrons(efpi_ctx* ctx, double* h_total_ms, int64_t* h_launches) {
  if (check_ctx(ctx) != EFPI_OK) return EFPI_EINVAL;
  if (!ctx->kinetic) return fail(EFPI_ESTATE, "the context has no kinetic electrons");
  return read_pairs(ctx, ctx->el_pairs, h_total_ms, h_launches);
}

// ------------------------------------------------------ learned projection

efpi_status efpi_nn_workspace_size(int32_t batch, int32_t n_c, size_t* h_bytes) {
  if (!h_bytes) return fail(EFPI_EINVAL, "h_bytes is NULL");
  if (batch < 1 || n_c < 1) return fail(EFPI_EINVAL, "batch and n_c must be >= 1");
  *h_bytes = sizeof(float) * nn::workspace_floats(batch, n_c);
  return EFPI_OK;
}

namespace {
efpi_status check_nn_shape(int32_t batch, int32_t n_c, void* d_ws, size_t ws_bytes) {
  if (batch < 1 || n_c < 1) return fail(EFPI_EINVAL, "batch and n_c must be >= 1");
  if (batch > 65535) return fail(EFPI_EINVAL, "batch must be <= 65535");
  if (!d_ws) return fail(EFPI_EINVAL, "workspace is NULL");
  if (ws_bytes < sizeof(float) * nn::workspace_floats(batch, n_c))
    return fail(EFPI_ENOMEM, "nn workspace smaller than efpi_nn_workspace_size");
  return EFPI_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
}  // namespace

efpi_status efpi_nn_pack(const float* d_params, void* d_pack, void* hip_stream) {
  if (!d_params || !d_pack) return fail(EFPI_EINVAL, "NULL parameter or pack pointer");
  if (!aligned16(d_pack)) return fail(EFPI_EINVAL, "pack must be 16-byte aligned");
  nn::launch_pack(d_params, static_cast<uint16_t*>(d_pack), static_cast<hipStream_t>(hip_stream));
  return hip_check("nn_pack");
}

efpi_status efpi_nn_forward(const float* d_params, const void* d_pack, const float* d_x,
                            float* d_y, int32_t batch, int32_t n_c, int32_t periodic, void* d_ws,
                            size_t ws_bytes, void* hip_stream) {
  if (!d_params || !d_pack || !d_x || !d_y) return fail(EFPI_EINVAL, "NULL pointer");
  if (!aligned16(d_pack)) return fail(EFPI_EINVAL, "pack must be 16-byte aligned");
  const efpi_status st = check_nn_shape(batch, n_c, d_ws, ws_bytes);
  if (st != EFPI_OK) return st;
  nn::launch_forward(d_params, static_cast<const uint16_t*>(d_pack), d_x, d_y, batch, n_c,
                     periodic != 0, static_cast<float*>(d_ws), static_cast<hipStream_t>(hip_stream));
  return hip_check("nn_forward");
}

efpi_status efpi_nn_backward(const void* d_pack, const float* d_x, const float* d_dy,
                             float* d_grad, int32_t batch, int32_t n_c, int32_t periodic,
                             void* d_ws, size_t ws_bytes, void* hip_stream) {
  if (!d_pack || !d_x || !d_dy || !d_grad) return fail(EFPI_EINVAL, "NULL pointer");
  if (!aligned16(d_pack)) return fail(EFPI_EINVAL, "pack must be 16-byte aligned");
  const efpi_status st = check_nn_shape(batch, n_c, d_ws, ws_bytes);
  if (st != EFPI_OK) return st;
  nn::launch_backward(static_cast<const uint16_t*>(d_pack), d_x, d_dy, d_grad, batch, n_c,
                      periodic != 0, static_cast<float*>(d_ws),
                      static_cast<hipStream_t>(hip_stream));
  return hip_check("nn_backward");
}

efpi_status efpi_nn_mse(const float* d_y, const float* d_t, float* d_dy, float* d_loss,
                        int64_t count, void* hip_stream) {
  if (!d_y || !d_t || !d_dy || !d_loss) return fail(EFPI_EINVAL, "NULL pointer");
  if (count < 1) return fail(EFPI_EINVAL, "count must be >= 1");
  nn::launch_mse(d_y, d_t, d_dy, d_loss, count, static_cast<hipStream_t>(hip_stream));
  return hip_check("nn_mse");
}

efpi_status efpi_nn_adam(float* d_params, const float* d_grad, float* d_m, float* d_v,
                         int32_t step, float lr, float beta1, float beta2, float eps,
                         void* d_pack, void* hip_stream) {
  if (!d_params || !d_grad || !d_m || !d_v || !d_pack) return fail(EFPI_EINVAL, "NULL pointer");
  if (!aligned16(d_pack)) return fail(EFPI_EINVAL, "pack must be 16-byte aligned");
  if (step < 1) return fail(EFPI_EINVAL, "step counts from 1");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(EFPI_EINVAL, "Adam hyper-parameters out of range");
  nn::launch_adam(d_params, d_grad, d_m, d_v, step, lr, beta1, beta2, eps,
                  static_cast<uint16_t*>(d_pack), static_cast<hipStream_t>(hip_stream));
  return hip_check("nn_adam");
}

namespace {
efpi_status check_norm(const efpi_nn_norm* n) {
  if (!n) return fail(EFPI_EINVAL, "norm is NULL");
  for (int m = 0; m < 2; ++m)
    if (!(n->sigma[m] > 0.f) || !(n->delta[m] > 0.f) || !std::isfinite(n->mu[m]))
      return fail(EFPI_EINVAL, "norm scales must be positive and finite");
  return EFPI_OK;
}
}  // namespace

efpi_status efpi_nn_features(const double* d_states, int32_t n_states, const int32_t* d_index,
                             int32_t batch, int32_t n_c, const efpi_nn_norm* h_norm, float noise,
                             uint32_t seed, float* d_x, float* d_t, void* hip_stream) {
  if (!d_states || !d_index || !d_x) return fail(EFPI_EINVAL, "NULL pointer");
  if (!(noise >= 0.f) || !std::isfinite(noise)) return fail(EFPI_EINVAL, "noise must be >= 0");
  if (batch < 1 || n_c < 1) return fail(EFPI_EINVAL, "batch and n_c must be >= 1");
  if (n_states < (d_t ? 4 : 3)) return fail(EFPI_EINVAL, "too few states");
  if (check_norm(h_norm) != EFPI_OK) return EFPI_EINVAL;
  nn::launch_features(d_states, n_states, d_index, batch, n_c, *h_norm, noise, seed, d_x, d_t,
                      static_cast<hipStream_t>(hip_stream));
  return hip_check("nn_features");
}

efpi_status efpi_nn_step(const double* d_c_n, const float* d_y, int32_t batch, int32_t n_c,
                         const efpi_nn_norm* h_norm, double* d_c_next, void* hip_stream) {
  if (!d_c_n || !d_y || !d_c_next) return fail(EFPI_EINVAL, "NULL pointer");
  if (batch < 1 || n_c < 1) return fail(EFPI_EINVAL, "batch and n_c must be >= 1");
  if (check_norm(h_norm) != EFPI_OK) return EFPI_EINVAL;
  nn::launch_step(d_c_n, d_y, batch, n_c, *h_norm, d_c_next, static_cast<hipStream_t>(hip_stream));
  return hip_check("nn_step");
}

efpi_status efpi_nn_predict_step(const float* d_params, const void* d_pack,
                                 const double* d_states, int32_t n_c, int32_t periodic,
                                 const efpi_nn_norm* h_norm, double* d_c_next, void* d_ws,
                                 size_t ws_bytes, void* hip_stream) {
  if (!d_params || !d_pack || !d_states || !d_c_next) return fail(EFPI_EINVAL, "NULL pointer");
  if (!aligned16(d_pack)) return fail(EFPI_EINVAL, "pack must be 16-byte aligned");
  const efpi_status st = check_nn_shape(1, n_c, d_ws, ws_bytes);
  if (st != EFPI_OK) return st;
  if (check_norm(h_norm) != EFPI_OK) return EFPI_EINVAL;
  const double* lo = d_states;
  const double* hi = d_states + 6 * (size_t)n_c;
  if (d_c_next + 2 * (size_t)n_c > lo && d_c_next < hi)
    return fail(EFPI_EINVAL, "d_c_next overlaps d_states");
  nn::launch_predict_step(d_params, static_cast<const uint16_t*>(d_pack), d_states, n_c,
                          periodic != 0, *h_norm, d_c_next, static_cast<float*>(d_ws),
                          static_cast<hipStream_t>(hip_stream));
  return hip_check("nn_predict_step");
}

efpi_status efpi_rel_l2(const double* d_a, const double* d_b, int64_t n, double* d_eps,
                        void* hip_stream) {
  if (!d_a || !d_b || !d_eps) return fail(EFPI_EINVAL, "NULL pointer");
  if (n < 1) return fail(EFPI_EINVAL, "n must be >= 1");
  nn::launch_rel_l2(d_a, d_b, n, d_eps, static_cast<hipStream_t>(hip_stream));
  return hip_check("rel_l2");
}

const char* efpi_last_error(void) { return g_err.c_str(); }

}  // extern "C"
