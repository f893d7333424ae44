// Host side of the C ABI declared in include/aderdg.h.
//
// A handle owns, per problem, a device scratch state (ping-pong partner of
// the caller's buffer: a fused step reads neighbour cells of u^n while other
// workgroups write u^{n+1}, so the update cannot be in place) and a device
// clock (time, rotating signal-speed maxima, last dt, status, sweep count).
// Problems sharing (scheme, PDE, N, precision) form a launch group served by
// one kernel launch per step; a workgroup finds its problem by binary search
// on the group's tile prefix.  Nothing here synchronises the host during
// aderdg_step / aderweno_step unless the caller's state pointers changed
// since the previous call (then the group's pointer table is re-uploaded
// after a stream synchronisation).
#include "../../include/aderdg.h"
#include "../../include/aderdg2d.h"
#include "../../include/aderdg3d.h"
#include "../../include/aderdg_lim.h"
#include "../../include/aderdg_lim2d.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "launch.hpp"
#include "launch2d.hpp"
#include "launch3d.hpp"
#include "launch_lim.hpp"
#include "operators.hpp"
#include "rtc.hpp"

using namespace aderdg;

namespace {

constexpr int kPdeUser = 100;   // pde code of a runtime-compiled user model
thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int fail_hip(hipError_t e, const char* what) {
  return fail(ADERDG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int model_nvars(int pde) {
  switch (pde) {
    case ADERDG_PDE_ADVECTION: return 1;
    case ADERDG_PDE_EULER: return 3;
    case ADERDG_PDE_EULER_REACT: return 5;
    case ADERDG_PDE_SWE: return 3;
    default: return -1;
  }
}

std::mutex g_tables_mutex;
std::set<int> g_tables_devices;

// Host copies of the device operator tables (also used to fill the tables of
// runtime-compiled modules).
DevOps g_host_ops[kDevMaxn];
DevOpsF g_host_opsf[kDevMaxn];

int ensure_tables(int device) {
  std::lock_guard<std::mutex> lock(g_tables_mutex);
  if (g_tables_devices.count(device)) return ADERDG_OK;
  DevOps* ops = g_host_ops;
  DevOpsF* opsf = g_host_opsf;
  static DevWeno weno[4];   // WENO degree 2, 4 (finite-volume step), 1 (limiter subgrid), 3
  static DevWeno fvw[3];    // degrees 1, 2, 3 (2-D and 3-D finite volumes)
  std::memset(g_host_ops, 0, sizeof(g_host_ops));
  std::memset(g_host_opsf, 0, sizeof(g_host_opsf));
  std::memset(weno, 0, sizeof(weno));
  for (int N = 0; N < kDevMaxn; ++N) {
    OpTables t;
    if (!build_op_tables(N, t)) return fail(ADERDG_E_DEVICE, "operator construction failed");
    const int n = N + 1;
    for (int i = 0; i < n; ++i) {
      ops[N].xi[i] = t.xi[i];
      ops[N].w[i] = t.w[i];
      ops[N].winv[i] = 1.0 / t.w[i];
      ops[N].psi0[i] = t.psi0[i];
      ops[N].psi1[i] = t.psi1[i];
      for (int j = 0; j < n; ++j) {
        ops[N].ktil[i][j] = t.ktil[i][j];
        ops[N].kappa[i][j] = t.kappa[i][j];
        ops[N].Dw[i][j] = t.Dtil[i][j] / t.w[i];
        opsf[N].ktil[i][j] = (float)t.ktil[i][j];
        opsf[N].kappa[i][j] = (float)t.kappa[i][j];
      }
    }
    for (int s = 0; s < t.Ns; ++s)
      for (int k = 0; k < n; ++k) ops[N].P[s][k] = t.P[s][k];
  }
  for (int wi = 0; wi < 4; ++wi) {
    WenoTables w;
    const int deg = wi < 2 ? 2 * (wi + 1) : wi == 2 ? 1 : 3;
    if (!build_weno_tables(deg, w)) return fail(ADERDG_E_DEVICE, "WENO table construction failed");
    for (int s = 0; s < w.nstencils; ++s)
      for (int i = 0; i < w.n; ++i)
        for (int j = 0; j < w.n; ++j) {
          weno[wi].R[s][i][j] = w.R[s][i][j];
          weno[wi].S[s][i][j] = w.S[s][i][j];
        }
  }
  hipError_t e = upload_tables(ops, opsf, weno);
  if (e != hipSuccess) return fail_hip(e, "upload of operator tables");
  {
    static DevLimR lim[kDevMaxn];
    std::memset(lim, 0, sizeof(lim));
    for (int N = 0; N < kDevMaxn; ++N) {
      OpTables t;
      if (!build_op_tables(N, t)) return fail(ADERDG_E_DEVICE, "operator construction failed");
      for (int k = 0; k <= N; ++k)
        for (int s = 0; s < t.Ns; ++s) lim[N].R[k][s] = t.R[k][s];
    }
    e = upload_lim_tables(lim, &weno[2]);
    if (e != hipSuccess) return fail_hip(e, "upload of limiter tables");
    e = upload_lim2d_tables(lim);
    if (e != hipSuccess) return fail_hip(e, "upload of 2-D limiter tables");
  }
  fvw[0] = weno[2];
  fvw[1] = weno[0];
  fvw[2] = weno[3];
  e = upload_tables_2d(ops, opsf, fvw);
  if (e != hipSuccess) return fail_hip(e, "upload of 2-D operator tables");
  e = upload_tables_3d(ops, opsf, fvw);
  if (e != hipSuccess) return fail_hip(e, "upload of 3-D operator tables");
  g_tables_devices.insert(device);
  return ADERDG_OK;
}

struct Group {
  int scheme, pde, N, prec, inner;
  const RtcModule* rtc = nullptr;   // runtime-compiled user model (else a compiled-in one)
  std::vector<int> pids;
  std::vector<ProbDev> host;
  ProbDev* dev = nullptr;
  int64_t blocks = 0;       // step kernel workgroups
  int64_t lam_blocks = 0;   // lambda kernel workgroups
  std::vector<ProbDev> lam_host;
  ProbDev* lam_dev = nullptr;
  bool any_cfl = false;
  int waves = kDgWaves;     // wavefronts per workgroup of the fused DG step
};

}  // namespace

struct aderdg_handle {
  hipStream_t stream = nullptr;
  int device = 0;
  int nprob = 0;
  std::vector<aderdg_pde_desc> pdes;
  std::vector<aderdg_config> cfgs;
  std::vector<double*> scratch;
  std::vector<int64_t> elems;          // doubles of state per problem
  std::vector<ProbDev> single_host;    // per-problem descriptor for the standalone kernels
  ProbDev* single_dev = nullptr;
  ProbClock* clocks = nullptr;
  double* partials = nullptr;          // conserved-totals partial sums (largest problem)
  const RtcModule* rtc = nullptr;      // user model of a handle made by aderdg_user_init
  std::vector<Group> groups;
};

namespace {

// Stream-ordered release: every buffer goes back to the device's memory pool
// after the work already enqueued on the handle's stream; the host is not
// synchronised.
void release(aderdg_handle* h) {
  if (!h) return;
  hipStream_t st = h->stream;
  for (double* p : h->scratch) if (p) (void)hipFreeAsync(p, st);
  for (Group& g : h->groups) {
    if (g.dev) (void)hipFreeAsync(g.dev, st);
    if (g.lam_dev) (void)hipFreeAsync(g.lam_dev, st);
  }
  if (h->single_dev) (void)hipFreeAsync(h->single_dev, st);
  if (h->clocks) (void)hipFreeAsync(h->clocks, st);
  if (h->partials) (void)hipFreeAsync(h->partials, st);
  delete h;
}

int validate(const aderdg_pde_desc& p, const aderdg_config& c, int k) {
  char buf[256];
  auto bad = [&](const char* what) {
    std::snprintf(buf, sizeof(buf), "problem %d: %s", k, what);
    return fail(ADERDG_E_INVAL, buf);
  };
  const int M = p.pde == kPdeUser ? p.nvars : model_nvars(p.pde);
  if (M < 0) return bad("unknown pde");
  if (p.pde == kPdeUser && (M < 1 || M > kTotMaxVars)) return bad("a user model needs 1 <= nvars <= 5");
  if (p.nvars != M) return bad("nvars does not match the model");
  if (p.pde == kPdeUser && c.scheme != ADERDG_SCHEME_DG) return bad("user models run the DG scheme");
  if (p.pde == kPdeUser && c.inner != ADERDG_INNER_PICARD) return bad("user models use Picard inner iterations");
  if ((p.pde == ADERDG_PDE_EULER || p.pde == ADERDG_PDE_EULER_REACT) && !(p.gamma > 1.0))
    return bad("gamma must be > 1");
  if (p.pde == ADERDG_PDE_SWE && !(p.g > 0.0)) return bad("g must be > 0");
  if (!std::isfinite(p.omega) || !std::isfinite(p.adv_speed)) return bad("non-finite model parameter");
  if (c.scheme != ADERDG_SCHEME_DG && c.scheme != ADERDG_SCHEME_FV) return bad("unknown scheme");
  if (c.scheme == ADERDG_SCHEME_DG && (c.N < 1 || c.N > kMaxN)) return bad("DG degree N must be in 1..9");
  if (c.scheme == ADERDG_SCHEME_FV && c.N != 2 && c.N != 4) return bad("WENO degree N must be 2 or 4");
  if (c.bc != ADERDG_BC_PERIODIC) return bad("only periodic boundaries are supported");
  if (c.ncells < 1) return bad("ncells must be >= 1");
  if (c.scheme == ADERDG_SCHEME_FV && c.ncells < 2 * c.N + 1) return bad("FV needs ncells >= 2N+1");
  if (c.ncells > (int64_t)1 << 34) return bad("ncells too large");
  if (!(std::isfinite(c.x0) && std::isfinite(c.x1) && c.x1 > c.x0)) return bad("need finite x1 > x0");
  if (!(c.fixed_dt > 0.0) && !(c.cfl > 0.0 && c.cfl <= 1.0)) return bad("cfl must be in (0, 1]");
  if (!std::isfinite(c.fixed_dt)) return bad("non-finite fixed_dt");
  if (c.cfl_mode != ADERDG_CFL_SUBCELL && c.cfl_mode != ADERDG_CFL_NODAL) return bad("unknown cfl_mode");
  if (c.precision != ADERDG_FP64 && c.precision != ADERDG_FP32_PREDICTOR) return bad("unknown precision");
  if (!std::isfinite(c.picard_tol)) return bad("non-finite picard_tol");
  if (c.picard_max_iter > 100000) return bad("picard_max_iter too large");
  if (c.inner != ADERDG_INNER_PICARD && c.inner != ADERDG_INNER_NEWTON) return bad("unknown inner solver");
  if (c.inner == ADERDG_INNER_NEWTON && (c.scheme != ADERDG_SCHEME_DG || p.pde != ADERDG_PDE_EULER_REACT))
    return bad("Newton inner iterations serve DG problems of the model with a linear source (EULER_REACT)");
  if (c.reserved != 0) return bad("reserved must be 0");
  return ADERDG_OK;
}

ProbDev probdev_of(const aderdg_pde_desc& p, const aderdg_config& c, int k, double* scratch) {
  ProbDev d;
  std::memset(&d, 0, sizeof(d));
  d.state[0] = nullptr;
  d.state[1] = scratch;
  d.ncells = c.ncells;
  d.x0 = c.x0;
  d.dx = (c.x1 - c.x0) / (double)c.ncells;
  d.cfl = c.cfl;
  d.fixed_dt = c.fixed_dt > 0.0 ? c.fixed_dt : 0.0;
  d.tol = c.picard_tol > 0.0 ? c.picard_tol : (c.precision == ADERDG_FP32_PREDICTOR ? 1e-6 : 1e-14);
  d.max_iter = c.picard_max_iter > 0 ? c.picard_max_iter : 64;
  d.cfl_mode = c.cfl_mode;
  d.pid = k;
  d.pp.gamma = p.gamma;
  d.pp.g = p.g;
  d.pp.omega = p.omega;
  d.pp.a = p.adv_speed;
  return d;
}

ProbDev make_probdev(const aderdg_handle* h, int k) {
  return probdev_of(h->pdes[k], h->cfgs[k], k, h->scratch[k]);
}

int upload_group(aderdg_handle* h, Group& g) {
  hipError_t e = launch_write_probs(g.host.data(), (int)g.host.size(), g.dev, h->stream);
  if (e != hipSuccess) return fail_hip(e, "upload of problem table");
  e = launch_write_probs(g.lam_host.data(), (int)g.lam_host.size(), g.lam_dev, h->stream);
  if (e != hipSuccess) return fail_hip(e, "upload of problem table");
  return ADERDG_OK;
}

// Point the group's tables at the caller's state buffers: when they changed,
// the new pointers are written by a small kernel in stream order (no host
// synchronisation; under stream capture the write is part of the graph).
int bind_states(aderdg_handle* h, Group& g, double* const* u) {
  bool changed = false;
  for (size_t i = 0; i < g.pids.size(); ++i) {
    double* p = u[g.pids[i]];
    if (!p) return fail(ADERDG_E_INVAL, "null state pointer for problem " + std::to_string(g.pids[i]));
    if (g.host[i].state[0] != p) changed = true;
  }
  if (!changed) return ADERDG_OK;
  std::vector<double*> ptrs(g.pids.size());
  for (size_t i = 0; i < g.pids.size(); ++i) {
    ptrs[i] = u[g.pids[i]];
    g.host[i].state[0] = ptrs[i];
    g.lam_host[i].state[0] = ptrs[i];
  }
  hipError_t e = launch_write_state_ptrs(ptrs.data(), (int)ptrs.size(), g.dev, g.lam_dev, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "state pointer kernel");
}

int run_steps(aderdg_handle* h, int scheme, double* const* u, double* t, const double* t_end,
              double* dt, int32_t* status, int32_t nsteps) {
  if (!h) return fail(ADERDG_E_INVAL, "null handle");
  if (!u || !t || !t_end || !dt || !status) return fail(ADERDG_E_INVAL, "null argument");
  if (nsteps < 0) return fail(ADERDG_E_INVAL, "nsteps must be >= 0");
  std::vector<Group*> gs;
  for (Group& g : h->groups)
    if (g.scheme == scheme) gs.push_back(&g);
  for (Group* g : gs) {
    int rc = bind_states(h, *g, u);
    if (rc) return rc;
  }
  hipError_t e = launch_clock_begin(h->clocks, t, h->nprob, h->stream);
  if (e != hipSuccess) return fail_hip(e, "clock kernel");
  if (nsteps > 0) {
    for (Group* g : gs) {
      if (!g->any_cfl) continue;
      StepArgs A{};
      A.probs = g->lam_dev;
      A.nprob = (int)g->pids.size();
      A.clocks = h->clocks;
      A.t_end = t_end;
      e = g->rtc ? rtc_launch(g->rtc->lambda, A, g->lam_blocks, 256, h->stream)
                 : launch_lambda(g->pde, g->N, scheme == ADERDG_SCHEME_DG, A, g->lam_blocks, h->stream);
      if (e != hipSuccess) return fail_hip(e, "lambda kernel");
    }
  }
  for (int s = 0; s < nsteps; ++s) {
    for (Group* g : gs) {
      StepArgs A{};
      A.probs = g->dev;
      A.nprob = (int)g->pids.size();
      A.clocks = h->clocks;
      A.t_end = t_end;
      A.step = s;
      if (g->rtc)
        e = rtc_launch(g->rtc->dg[2], A, g->blocks, kRtcWaves * 64, h->stream);
      else
        e = scheme == ADERDG_SCHEME_DG ? launch_dg(g->pde, g->N, g->prec, 2, A, g->blocks, h->stream,
                                                   g->inner == ADERDG_INNER_NEWTON, g->waves)
                                        : launch_fv(g->pde, g->N, g->prec, A, g->blocks, h->stream);
      if (e != hipSuccess) return fail_hip(e, "step kernel");
    }
  }
  e = launch_clock_end(h->clocks, t, dt, status, h->nprob, nsteps & 1, h->stream);
  if (e != hipSuccess) return fail_hip(e, "clock kernel");
  if (nsteps & 1) {
    for (Group* g : gs)
      for (size_t i = 0; i < g->pids.size(); ++i) {
        const int k = g->pids[i];
        e = launch_copy(h->scratch[k], u[k], h->elems[k], h->stream);
        if (e != hipSuccess) return fail_hip(e, "copy kernel");
      }
  }
  return ADERDG_OK;
}

// A group whose fused step can run with either compiled workgroup size.
bool tunable(const Group& g) {
  return g.scheme == ADERDG_SCHEME_DG && !g.rtc && g.inner == ADERDG_INNER_PICARD;
}

// Tile the group's problems for `waves` wavefronts per workgroup and upload
// the table (stream-ordered).
int set_group_waves(aderdg_handle* h, Group& g, int waves) {
  const int64_t tile = dg_tile_cells(g.N, true, waves);
  int64_t b = 0;
  for (ProbDev& d : g.host) {
    d.tile_begin = b;
    d.tiles = (d.ncells + tile - 1) / tile;
    b += d.tiles;
  }
  if (b >= ((int64_t)1 << 31)) return fail(ADERDG_E_INVAL, "grid too large");
  g.blocks = b;
  g.waves = waves;
  return upload_group(h, g);
}

// Process-wide cache of tuned workgroup sizes: key (device arch, model, N,
// precision, total cells of the group rounded up to a power of 2); also
// kept in the file named by ADERDG_TUNE_FILE (one "key waves" line each).
std::mutex g_tune_mutex;
std::map<std::string, int> g_tune_cache;
bool g_tune_file_read = false;

std::string tune_key(int device, const Group& g) {
  hipDeviceProp_t prop;
  std::string arch = hipGetDeviceProperties(&prop, device) == hipSuccess ? prop.gcnArchName : "unknown";
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  int64_t cells = 0;
  for (const ProbDev& d : g.host) cells += d.ncells;
  int lg = 0;
  while (((int64_t)1 << lg) < cells) ++lg;
  return arch + "/pde" + std::to_string(g.pde) + "/N" + std::to_string(g.N) + "/p" + std::to_string(g.prec) +
         "/c2^" + std::to_string(lg);
}

void tune_file_load() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("ADERDG_TUNE_FILE");
  if (!path) return;
  std::ifstream in(path);
  std::string key;
  int w;
  while (in >> key >> w)
    if (w == kDgWaves || w == kDgWavesAlt) g_tune_cache[key] = w;
}

void tune_file_append(const std::string& key, int w) {
  const char* path = std::getenv("ADERDG_TUNE_FILE");
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  out << key << " " << w << "\n";
}

// Seconds of `steps` fused steps of group g from the states src (copied to
// work first), with `waves` wavefronts per workgroup; -1 on error.
double time_group(aderdg_handle* h, Group& g, int waves, double* const* src, double* const* work,
                  double* t_dev, const double* tend_dev, int32_t steps) {
  if (set_group_waves(h, g, waves)) return -1.0;
  for (size_t i = 0; i < g.pids.size(); ++i) {
    const int k = g.pids[i];
    if (launch_copy(src[k], work[k], h->elems[k], h->stream) != hipSuccess) return -1.0;
  }
  if (bind_states(h, g, work)) return -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
  hipError_t e = launch_clock_begin(h->clocks, t_dev, h->nprob, h->stream);
  StepArgs A{};
  A.clocks = h->clocks;
  A.t_end = tend_dev;
  if (e == hipSuccess && g.any_cfl) {
    A.probs = g.lam_dev;
    A.nprob = (int)g.pids.size();
    e = launch_lambda(g.pde, g.N, true, A, g.lam_blocks, h->stream);
  }
  A.probs = g.dev;
  A.nprob = (int)g.pids.size();
  const int warm = 2;
  for (int s = 0; s < warm + steps && e == hipSuccess; ++s) {
    if (s == warm) e = hipEventRecord(e0, h->stream);
    A.step = s;
    if (e == hipSuccess) e = launch_dg(g.pde, g.N, g.prec, 2, A, g.blocks, h->stream, false, waves);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = -1.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e == hipSuccess ? ms * 1e-3 : -1.0;
}

int init_handle(const aderdg_pde_desc* pdes, const aderdg_config* cfgs, int32_t nprob, void* hip_stream,
                aderdg_handle** out, const std::string* user_model) {
  if (!pdes || !cfgs || !out) return fail(ADERDG_E_INVAL, "null argument");
  if (nprob < 1) return fail(ADERDG_E_INVAL, "nprob must be >= 1");
  for (int k = 0; k < nprob; ++k) {
    if ((pdes[k].pde == kPdeUser) != (user_model != nullptr)) return fail(ADERDG_E_INVAL, "unknown pde");
    int rc = validate(pdes[k], cfgs[k], k);
    if (rc) return rc;
  }
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  int rc = ensure_tables(device);
  if (rc) return rc;
  const RtcModule* rtc = nullptr;
  if (user_model) {
    std::string log;
    const int r = rtc_module(*user_model, pdes[0].nvars, cfgs[0].N, cfgs[0].precision, device, g_host_ops,
                             g_host_opsf, &rtc, &log);
    if (r == -1) return fail(ADERDG_E_INVAL, "user model does not compile:\n" + log);
    if (r) return fail(ADERDG_E_DEVICE, log);
  }

  aderdg_handle* h = new aderdg_handle();
  h->rtc = rtc;
  h->stream = (hipStream_t)hip_stream;
  h->device = device;
  h->nprob = nprob;
  h->pdes.assign(pdes, pdes + nprob);
  h->cfgs.assign(cfgs, cfgs + nprob);
  h->scratch.assign(nprob, nullptr);
  h->elems.assign(nprob, 0);
  // every allocation and table write is stream-ordered on the handle's stream
  hipStream_t st = h->stream;
  for (int k = 0; k < nprob; ++k) {
    const aderdg_config& c = cfgs[k];
    const int64_t per_cell = c.scheme == ADERDG_SCHEME_DG ? (int64_t)(c.N + 1) * pdes[k].nvars : pdes[k].nvars;
    h->elems[k] = per_cell * c.ncells;
    e = hipMallocAsync((void**)&h->scratch[k], sizeof(double) * h->elems[k], st);
    if (e != hipSuccess) { release(h); return fail(ADERDG_E_NOMEM, "scratch allocation"); }
  }
  int64_t nparts = 1;
  for (int k = 0; k < nprob; ++k) {
    const int64_t p = totals_partials(cfgs[k].ncells) * pdes[k].nvars;
    if (p > nparts) nparts = p;
  }
  e = hipMallocAsync((void**)&h->partials, sizeof(double) * nparts, st);
  if (e != hipSuccess) { release(h); return fail(ADERDG_E_NOMEM, "partials allocation"); }
  e = hipMallocAsync((void**)&h->clocks, sizeof(ProbClock) * nprob, st);
  if (e != hipSuccess) { release(h); return fail(ADERDG_E_NOMEM, "clock allocation"); }
  e = launch_zero(h->clocks, sizeof(ProbClock) * nprob, st);
  if (e != hipSuccess) { release(h); return fail_hip(e, "clock init"); }
  // standalone descriptors
  for (int k = 0; k < nprob; ++k) h->single_host.push_back(make_probdev(h, k));
  e = hipMallocAsync((void**)&h->single_dev, sizeof(ProbDev) * nprob, st);
  if (e != hipSuccess) { release(h); return fail(ADERDG_E_NOMEM, "table allocation"); }
  e = launch_write_probs(h->single_host.data(), nprob, h->single_dev, st);
  if (e != hipSuccess) { release(h); return fail_hip(e, "table upload"); }
  // launch groups
  std::map<std::tuple<int, int, int, int, int>, int> index;
  for (int k = 0; k < nprob; ++k) {
    auto key = std::make_tuple(cfgs[k].scheme, pdes[k].pde, cfgs[k].N, cfgs[k].precision, cfgs[k].inner);
    auto it = index.find(key);
    if (it == index.end()) {
      Group g;
      g.scheme = cfgs[k].scheme;
      g.pde = pdes[k].pde;
      g.N = cfgs[k].N;
      g.prec = cfgs[k].precision;
      g.inner = cfgs[k].inner;
      index[key] = (int)h->groups.size();
      h->groups.push_back(g);
      it = index.find(key);
    }
    h->groups[it->second].pids.push_back(k);
  }
  for (Group& g : h->groups) {
    const int64_t tile = g.scheme == ADERDG_SCHEME_DG ? dg_tile_cells(g.N, true) : fv_tile_cells(g.N);
    int64_t b = 0, lb = 0;
    for (int k : g.pids) {
      ProbDev d = make_probdev(h, k);
      d.tile_begin = b;
      d.tiles = (d.ncells + tile - 1) / tile;
      b += d.tiles;
      g.host.push_back(d);
      ProbDev l = d;
      l.tile_begin = lb;
      l.tiles = (d.ncells + 255) / 256;
      lb += l.tiles;
      g.lam_host.push_back(l);
      if (!(cfgs[k].fixed_dt > 0.0)) g.any_cfl = true;
    }
    g.blocks = b;
    g.lam_blocks = lb;
    if (b >= ((int64_t)1 << 31)) { release(h); return fail(ADERDG_E_INVAL, "grid too large"); }
    e = hipMallocAsync((void**)&g.dev, sizeof(ProbDev) * g.host.size(), st);
    if (e != hipSuccess) { release(h); return fail(ADERDG_E_NOMEM, "table allocation"); }
    e = hipMallocAsync((void**)&g.lam_dev, sizeof(ProbDev) * g.lam_host.size(), st);
    if (e != hipSuccess) { release(h); return fail(ADERDG_E_NOMEM, "table allocation"); }
    // state pointers are bound by the first step call
    rc = upload_group(h, g);
    if (rc) { release(h); return rc; }
    g.rtc = rtc;
  }
  *out = h;
  return ADERDG_OK;
}

}  // namespace

extern "C" {

int aderdg_init(const aderdg_pde_desc* pdes, const aderdg_config* cfgs, int32_t nprob,
                void* hip_stream, aderdg_handle** out) {
  g_last_error.clear();
  return init_handle(pdes, cfgs, nprob, hip_stream, out, nullptr);
}

int aderdg_user_init(const char* model_source, int32_t nvars, const double* params,
                     const aderdg_config* cfg, void* hip_stream, aderdg_handle** out) {
  g_last_error.clear();
  if (!model_source || !params || !cfg || !out) return fail(ADERDG_E_INVAL, "null argument");
  aderdg_pde_desc d{};
  d.pde = kPdeUser;
  d.nvars = nvars;
  d.gamma = params[0];
  d.g = params[1];
  d.omega = params[2];
  d.adv_speed = params[3];
  const std::string model(model_source);
  return init_handle(&d, cfg, 1, hip_stream, out, &model);
}

int aderdg_user_compile_check(const char* model_source, int32_t nvars, int32_t N, int32_t precision,
                              char* log, int64_t cap) {
  g_last_error.clear();
  if (!model_source) return fail(ADERDG_E_INVAL, "null argument");
  if (N < 1 || N > kMaxN) return fail(ADERDG_E_INVAL, "N must be in 1..9");
  if (precision != ADERDG_FP64 && precision != ADERDG_FP32_PREDICTOR) return fail(ADERDG_E_INVAL, "unknown precision");
  if (nvars < 1 || nvars > kTotMaxVars) return fail(ADERDG_E_INVAL, "a user model needs 1 <= nvars <= 5");
  std::string text;
  const int r = rtc_compile_check(model_source, nvars, N, precision, &text);
  if (log && cap > 0) {
    const size_t n = text.size() < (size_t)(cap - 1) ? text.size() : (size_t)(cap - 1);
    std::memcpy(log, text.data(), n);
    log[n] = '\0';
  }
  return r ? fail(ADERDG_E_INVAL, "user model does not compile") : ADERDG_OK;
}

int aderdg_set_stream(aderdg_handle* h, void* hip_stream) {
  if (!h) return fail(ADERDG_E_INVAL, "null handle");
  h->stream = (hipStream_t)hip_stream;
  return ADERDG_OK;
}

static int check_standalone(aderdg_handle* h, int32_t k, double t, double dt) {
  if (!h) return fail(ADERDG_E_INVAL, "null handle");
  if (k < 0 || k >= h->nprob) return fail(ADERDG_E_INVAL, "problem index out of range");
  if (h->cfgs[k].scheme != ADERDG_SCHEME_DG) return fail(ADERDG_E_INVAL, "problem is not a DG problem");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return fail(ADERDG_E_INVAL, "need finite t and dt > 0");
  return ADERDG_OK;
}

int aderdg_predict(aderdg_handle* h, int32_t k, const double* u, double t, double dt, void* q_out,
                   int32_t* iters_out) {
  int rc = check_standalone(h, k, t, dt);
  if (rc) return rc;
  if (!u || !q_out) return fail(ADERDG_E_INVAL, "null buffer");
  const aderdg_config& c = h->cfgs[k];
  StepArgs A{};
  A.probs = h->single_dev + k;
  A.nprob = 1;
  A.k = 0;
  A.clocks = h->clocks;
  A.u_in = u;
  A.q = q_out;
  A.iters = iters_out;
  A.t = t;
  A.dt = dt;
  const int64_t tile = dg_tile_cells(c.N, false);
  hipError_t e = h->rtc ? rtc_launch(h->rtc->dg[0], A, (c.ncells + tile - 1) / tile, kRtcWaves * 64, h->stream)
                        : launch_dg(h->pdes[k].pde, c.N, c.precision, 0, A, (c.ncells + tile - 1) / tile,
                                    h->stream, c.inner == ADERDG_INNER_NEWTON);
  if (e != hipSuccess) return fail_hip(e, "predictor kernel");
  return ADERDG_OK;
}

int aderdg_correct(aderdg_handle* h, int32_t k, const double* u, const void* q, double t, double dt,
                   double* u_next) {
  int rc = check_standalone(h, k, t, dt);
  if (rc) return rc;
  if (!u || !q || !u_next) return fail(ADERDG_E_INVAL, "null buffer");
  if ((const void*)u == (const void*)u_next) return fail(ADERDG_E_INVAL, "u_next must not alias u");
  const aderdg_config& c = h->cfgs[k];
  StepArgs A{};
  A.probs = h->single_dev + k;
  A.nprob = 1;
  A.k = 0;
  A.clocks = h->clocks;
  A.u_in = u;
  A.u_out = u_next;
  A.q = const_cast<void*>(q);
  A.t = t;
  A.dt = dt;
  const int64_t tile = dg_tile_cells(c.N, true);
  hipError_t e = h->rtc ? rtc_launch(h->rtc->dg[1], A, (c.ncells + tile - 1) / tile, kRtcWaves * 64, h->stream)
                        : launch_dg(h->pdes[k].pde, c.N, c.precision, 1, A, (c.ncells + tile - 1) / tile,
                                    h->stream);
  if (e != hipSuccess) return fail_hip(e, "corrector kernel");
  return ADERDG_OK;
}

int aderdg_step(aderdg_handle* h, double* const* u, double* t, const double* t_end, double* dt,
                int32_t* status, int32_t nsteps) {
  return run_steps(h, ADERDG_SCHEME_DG, u, t, t_end, dt, status, nsteps);
}

int aderweno_step(aderdg_handle* h, double* const* v, double* t, const double* t_end, double* dt,
                  int32_t* status, int32_t nsteps) {
  return run_steps(h, ADERDG_SCHEME_FV, v, t, t_end, dt, status, nsteps);
}

int aderdg_set_waves(aderdg_handle* h, int32_t waves) {
  g_last_error.clear();
  if (!h) return fail(ADERDG_E_INVAL, "null handle");
  if (waves != kDgWaves && waves != kDgWavesAlt) return fail(ADERDG_E_INVAL, "waves must be 4 or 2");
  for (Group& g : h->groups) {
    if (!tunable(g)) continue;
    int rc = set_group_waves(h, g, waves);
    if (rc) return rc;
  }
  return ADERDG_OK;
}

int aderdg_autotune(aderdg_handle* h, double* const* u, int32_t steps, int32_t* waves_out) {
  g_last_error.clear();
  if (!h || !u) return fail(ADERDG_E_INVAL, "null argument");
  if (steps < 1 || steps > 10000) return fail(ADERDG_E_INVAL, "steps must be in 1..10000");
  for (int k = 0; k < h->nprob; ++k)
    if (!u[k]) return fail(ADERDG_E_INVAL, "null state pointer for problem " + std::to_string(k));
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  tune_file_load();
  hipStream_t st = h->stream;
  // work copies of the states, the clocks saved, a start time and an open end
  std::vector<double*> work(h->nprob, nullptr);
  ProbClock* saved = nullptr;
  double* tt = nullptr;
  auto cleanup = [&]() {
    for (double* p : work) if (p) (void)hipFreeAsync(p, st);
    if (saved) (void)hipFreeAsync(saved, st);
    if (tt) (void)hipFreeAsync(tt, st);
    (void)hipStreamSynchronize(st);
  };
  hipError_t e = hipMallocAsync((void**)&saved, sizeof(ProbClock) * h->nprob, st);
  if (e == hipSuccess) e = hipMallocAsync((void**)&tt, sizeof(double) * 2 * h->nprob, st);
  for (int k = 0; k < h->nprob && e == hipSuccess; ++k) e = hipMallocAsync((void**)&work[k], sizeof(double) * h->elems[k], st);
  if (e != hipSuccess) { cleanup(); return fail(ADERDG_E_NOMEM, "autotune buffers"); }
  std::vector<double> host_t(2 * h->nprob, 0.0);     // start times, then end times
  for (int k = 0; k < h->nprob; ++k) host_t[h->nprob + k] = 1.0e300;
  e = hipMemcpyAsync(saved, h->clocks, sizeof(ProbClock) * h->nprob, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(tt, host_t.data(), sizeof(double) * 2 * h->nprob, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { cleanup(); return fail_hip(e, "autotune set-up"); }
  int rc = ADERDG_OK;
  for (Group& g : h->groups) {
    if (!tunable(g)) continue;
    const std::string key = tune_key(h->device, g);
    auto it = g_tune_cache.find(key);
    int best = kDgWaves;
    if (it != g_tune_cache.end()) {
      best = it->second;
    } else {
      std::vector<double> times;
      for (int w : {kDgWaves, kDgWavesAlt}) {
        double s = time_group(h, g, w, u, work.data(), tt, tt + h->nprob, steps);
        if (s < 0.0) { rc = fail(ADERDG_E_DEVICE, "autotune timing run"); break; }
        times.push_back(s);
      }
      if (rc) break;
      best = times[1] < times[0] ? kDgWavesAlt : kDgWaves;
      g_tune_cache[key] = best;
      tune_file_append(key, best);
    }
    rc = set_group_waves(h, g, best);
    if (rc) break;
  }
  // leave the problems as they were: clocks restored; the state pointers are
  // bound again by the next step call
  e = hipMemcpyAsync(h->clocks, saved, sizeof(ProbClock) * h->nprob, hipMemcpyDeviceToDevice, st);
  cleanup();
  if (rc) return rc;
  if (e != hipSuccess) return fail_hip(e, "autotune restore");
  if (waves_out)
    for (const Group& g : h->groups)
      for (int k : g.pids) waves_out[k] = tunable(g) ? g.waves : kDgWaves;
  return ADERDG_OK;
}

int aderdg_free(aderdg_handle* h) {
  release(h);
  return ADERDG_OK;
}

int aderdg_step_noalloc(const aderdg_pde_desc* pde, const aderdg_config* cfg, double* u, double* t,
                        const double* t_end, double* dt, int32_t* status, int32_t nsteps,
                        void* hip_stream) {
  g_last_error.clear();
  if (!pde || !cfg || !u || !t || !t_end || !dt || !status) return fail(ADERDG_E_INVAL, "null argument");
  if (nsteps < 0) return fail(ADERDG_E_INVAL, "nsteps must be >= 0");
  int rc = validate(*pde, *cfg, 0);
  if (rc) return rc;
  const bool is_dg = cfg->scheme == ADERDG_SCHEME_DG;
  const int64_t per_cell = is_dg ? (int64_t)(cfg->N + 1) * pde->nvars : pde->nvars;
  const int64_t elems = per_cell * cfg->ncells;
  if (elems > (int64_t)kNoallocMaxElems)
    return fail(ADERDG_E_INVAL, "state of " + std::to_string(elems) + " doubles exceeds the " +
                                    std::to_string(kNoallocMaxElems) +
                                    " doubles of the static scratch (64 MiB per device)");
  hipStream_t st = (hipStream_t)hip_stream;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  rc = ensure_tables(device);
  if (rc) return rc;
  void* base = nullptr;
  e = noalloc_scratch(device, &base);
  if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress of the static scratch");
  unsigned char* b = static_cast<unsigned char*>(base);
  double* copy = reinterpret_cast<double*>(b + kNoallocState);
  ProbDev d = probdev_of(*pde, *cfg, 0, copy);
  d.state[0] = u;
  const int64_t tile = is_dg ? dg_tile_cells(cfg->N, true) : fv_tile_cells(cfg->N);
  d.tile_begin = 0;
  d.tiles = (cfg->ncells + tile - 1) / tile;
  ProbDev l = d;
  l.tiles = (cfg->ncells + 255) / 256;
  if (d.tiles >= ((int64_t)1 << 31)) return fail(ADERDG_E_INVAL, "grid too large");
  e = launch_noalloc_setup(d, l, base, st);
  if (e != hipSuccess) return fail_hip(e, "descriptor kernel");
  ProbClock* clk = reinterpret_cast<ProbClock*>(b + kNoallocClock);
  e = launch_clock_begin(clk, t, 1, st);
  if (e != hipSuccess) return fail_hip(e, "clock kernel");
  if (nsteps > 0 && !(cfg->fixed_dt > 0.0)) {
    StepArgs A{};
    A.probs = reinterpret_cast<const ProbDev*>(b + kNoallocLamDesc);
    A.nprob = 1;
    A.clocks = clk;
    A.t_end = t_end;
    e = launch_lambda(pde->pde, cfg->N, is_dg, A, l.tiles, st);
    if (e != hipSuccess) return fail_hip(e, "lambda kernel");
  }
  for (int s = 0; s < nsteps; ++s) {
    StepArgs A{};
    A.probs = reinterpret_cast<const ProbDev*>(b + kNoallocStepDesc);
    A.nprob = 1;
    A.clocks = clk;
    A.t_end = t_end;
    A.step = s;
    e = is_dg ? launch_dg(pde->pde, cfg->N, cfg->precision, 2, A, d.tiles, st, cfg->inner == ADERDG_INNER_NEWTON)
              : launch_fv(pde->pde, cfg->N, cfg->precision, A, d.tiles, st);
    if (e != hipSuccess) return fail_hip(e, "step kernel");
  }
  e = launch_clock_end(clk, t, dt, status, 1, nsteps & 1, st);
  if (e != hipSuccess) return fail_hip(e, "clock kernel");
  if (nsteps & 1) {
    e = launch_copy(copy, u, elems, st);
    if (e != hipSuccess) return fail_hip(e, "copy kernel");
  }
  return ADERDG_OK;
}

int aderdg_sweep_count(aderdg_handle* h, int32_t k, int64_t* sweeps_out) {
  if (!h || !sweeps_out) return fail(ADERDG_E_INVAL, "null argument");
  if (k < 0 || k >= h->nprob) return fail(ADERDG_E_INVAL, "problem index out of range");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "stream synchronize");
  Slot slots[kSlots];
  e = hipMemcpy(slots, h->clocks[k].sweeps, sizeof(slots), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "sweep count read");
  int64_t total = 0;
  for (int i = 0; i < kSlots; ++i) total += (int64_t)slots[i].v;
  *sweeps_out = total;
  return ADERDG_OK;
}

int aderdg_contraction_count(aderdg_handle* h, int32_t k, int64_t* count_out) {
  if (!h || !count_out) return fail(ADERDG_E_INVAL, "null argument");
  if (k < 0 || k >= h->nprob) return fail(ADERDG_E_INVAL, "problem index out of range");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "stream synchronize");
  Slot slots[kSlots];
  e = hipMemcpy(slots, h->clocks[k].contractions, sizeof(slots), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "contraction count read");
  int64_t total = 0;
  for (int i = 0; i < kSlots; ++i) total += (int64_t)slots[i].v;
  *count_out = total;
  return ADERDG_OK;
}

int aderdg_conserved_totals(aderdg_handle* h, int32_t k, const double* u, double* totals_out) {
  g_last_error.clear();
  if (!h || !u || !totals_out) return fail(ADERDG_E_INVAL, "null argument");
  if (k < 0 || k >= h->nprob) return fail(ADERDG_E_INVAL, "problem index out of range");
  const aderdg_config& c = h->cfgs[k];
  const bool is_dg = c.scheme == ADERDG_SCHEME_DG;
  const double dx = (c.x1 - c.x0) / (double)c.ncells;
  hipError_t e = launch_totals(u, c.ncells, is_dg ? c.N : 0, is_dg ? c.N + 1 : 1, h->pdes[k].nvars, dx,
                               h->partials, totals_out, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "totals kernels");
}

int aderdg_operators(int32_t N, double* out, int64_t cap) {
  OpTables t;
  if (!out || !build_op_tables(N, t) || N < 0) return fail(ADERDG_E_INVAL, "bad degree or buffer");
  const int n = N + 1;
  const int64_t need = 2 * n + 3 * n * n + 2 * n + 2 * (int64_t)t.Ns * n;
  if (cap < need) return fail(ADERDG_E_INVAL, "buffer too small");
  int64_t o = 0;
  for (int i = 0; i < n; ++i) out[o++] = t.xi[i];
  for (int i = 0; i < n; ++i) out[o++] = t.w[i];
  for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) out[o++] = t.ktil[i][j];
  for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) out[o++] = t.kappa[i][j];
  for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) out[o++] = t.Dtil[i][j];
  for (int i = 0; i < n; ++i) out[o++] = t.psi0[i];
  for (int i = 0; i < n; ++i) out[o++] = t.psi1[i];
  for (int s = 0; s < t.Ns; ++s) for (int k = 0; k < n; ++k) out[o++] = t.P[s][k];
  for (int k = 0; k < n; ++k) for (int s = 0; s < t.Ns; ++s) out[o++] = t.R[k][s];
  return (int)o;
}

const char* aderdg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------ 2-D ----
// A 2-D handle owns the per-cell scratch the two kernels of a step exchange
// through (face traces; u + volume terms) and a device clock.  The corrector
// reads only that scratch, so it updates the caller's state in place.

struct aderdg2d_handle {
  hipStream_t stream = nullptr;
  aderdg2d_config cfg{};
  int64_t cells = 0;
  double* part = nullptr;
  void* tr = nullptr;
  double* w = nullptr;      // ADER-WENO: nodal WENO values of the averages
  Clock2D* clk = nullptr;
};

namespace {

void release2d(aderdg2d_handle* h) {
  if (h->part) hipFree(h->part);
  if (h->tr) hipFree(h->tr);
  if (h->w) hipFree(h->w);
  if (h->clk) hipFree(h->clk);
  delete h;
}

Args2D args2d(const aderdg2d_handle* h) {
  const aderdg2d_config& c = h->cfg;
  Args2D A{};
  A.cx = c.cells_x;
  A.cy = c.cells_y;
  A.dx = (c.x1 - c.x0) / (double)c.cells_x;
  A.dy = (c.y1 - c.y0) / (double)c.cells_y;
  A.cfl = c.cfl;
  A.fixed_dt = c.fixed_dt;
  A.tol = c.picard_tol;
  A.gamma = c.gamma;
  A.max_iter = c.picard_max_iter;
  A.clk = h->clk;
  A.part = h->part;
  A.tr = h->tr;
  A.scheme = c.scheme;
  return A;
}

}  // namespace

extern "C" {

int aderdg2d_init(const aderdg2d_config* cfg, void* hip_stream, aderdg2d_handle** out) {
  g_last_error.clear();
  if (!cfg || !out) return fail(ADERDG_E_INVAL, "null argument");
  aderdg2d_config c = *cfg;
  if (c.N < 1 || c.N > 9) return fail(ADERDG_E_INVAL, "N must be in 1..9");
  if (c.precision != ADERDG_FP64 && c.precision != ADERDG_FP32_PREDICTOR)
    return fail(ADERDG_E_INVAL, "unknown precision");
  if (c.scheme != ADERDG_SCHEME_DG && c.scheme != ADERDG_SCHEME_FV) return fail(ADERDG_E_INVAL, "unknown scheme");
  if (c.scheme == ADERDG_SCHEME_FV && (c.N > 3 || c.precision != ADERDG_FP64))
    return fail(ADERDG_E_INVAL, "2-D ADER-WENO: N (the WENO degree) must be 1..3, precision FP64");
  if (c.cells_x < 1 || c.cells_y < 1 || c.cells_x > INT32_MAX / c.cells_y)
    return fail(ADERDG_E_INVAL, "cells_x, cells_y must be >= 1 with a product below 2^31");
  if (!(c.x1 > c.x0) || !(c.y1 > c.y0) || !std::isfinite(c.x1 - c.x0) || !std::isfinite(c.y1 - c.y0))
    return fail(ADERDG_E_INVAL, "empty or non-finite domain");
  if (!(c.gamma > 1.0) || !std::isfinite(c.gamma)) return fail(ADERDG_E_INVAL, "gamma must be > 1");
  if (!(c.cfl > 0.0 && c.cfl <= 1.0)) return fail(ADERDG_E_INVAL, "cfl must be in (0, 1]");
  if (!(c.fixed_dt >= 0.0) || !std::isfinite(c.fixed_dt)) return fail(ADERDG_E_INVAL, "fixed_dt must be >= 0");
  if (!std::isfinite(c.picard_tol)) return fail(ADERDG_E_INVAL, "picard_tol must be finite");
  if (c.picard_tol <= 0.0) c.picard_tol = c.precision == ADERDG_FP64 ? 1e-14 : 1e-6;
  if (c.picard_max_iter <= 0) c.picard_max_iter = 64;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  int rc = ensure_tables(device);
  if (rc) return rc;
  aderdg2d_handle* h = new aderdg2d_handle();
  h->stream = (hipStream_t)hip_stream;
  h->cfg = c;
  h->cells = c.cells_x * c.cells_y;
  const int64_t L = (int64_t)(c.N + 1) * (c.N + 1);
  const bool fv = c.scheme == ADERDG_SCHEME_FV;
  // DG: u + volume terms; ADER-WENO: the nodal WENO values (the predictor's initial data)
  e = hipMalloc(fv ? (void**)&h->w : (void**)&h->part, sizeof(double) * h->cells * L * 4);
  const size_t tr_elem = c.precision == ADERDG_FP64 ? sizeof(double) : sizeof(float);
  if (e == hipSuccess) e = hipMalloc(&h->tr, tr_elem * h->cells * 4 * L * 4);
  if (e != hipSuccess) { release2d(h); return fail(ADERDG_E_NOMEM, "scratch allocation"); }
  e = hipMalloc((void**)&h->clk, sizeof(Clock2D));
  if (e != hipSuccess) { release2d(h); return fail(ADERDG_E_NOMEM, "clock allocation"); }
  e = hipMemset(h->clk, 0, sizeof(Clock2D));
  if (e != hipSuccess) { release2d(h); return fail_hip(e, "clock init"); }
  *out = h;
  return ADERDG_OK;
}

int aderdg2d_predict(aderdg2d_handle* h, const double* u, double t, double dt, void* q_out,
                     int32_t* iters_out) {
  g_last_error.clear();
  if (!h || !u || !q_out) return fail(ADERDG_E_INVAL, "null argument");
  if (h->cfg.scheme != ADERDG_SCHEME_DG) return fail(ADERDG_E_INVAL, "predictor-only calls serve the DG scheme");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return fail(ADERDG_E_INVAL, "dt must be > 0 and finite");
  Args2D A = args2d(h);
  A.mode = k2dPredict;
  A.t = t;
  A.dt = dt;
  A.u = const_cast<double*>(u);
  A.q_out = q_out;
  A.iters = iters_out;
  const int cpb = cells_per_block_2d(h->cfg.N, h->cfg.precision);
  hipError_t e = launch_pred2d(h->cfg.N, h->cfg.precision, A, (h->cells + cpb - 1) / cpb, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "predictor launch");
}

int aderdg2d_step(aderdg2d_handle* h, double* u, double* t, const double* t_end, double* dt,
                  int32_t* status, int32_t nsteps) {
  g_last_error.clear();
  if (!h || !u || !t || !t_end || !dt || !status) return fail(ADERDG_E_INVAL, "null argument");
  if (nsteps < 0) return fail(ADERDG_E_INVAL, "nsteps must be >= 0");
  Args2D A = args2d(h);
  A.mode = k2dStep;
  A.u = u;
  A.t_end = t_end;
  const int N = h->cfg.N;
  const int cpb = cells_per_block_2d(N, h->cfg.precision);
  const int cpb2 = cells_per_block_corr2d(N);
  const int64_t blocks = (h->cells + cpb - 1) / cpb, blocks2 = (h->cells + cpb2 - 1) / cpb2;
  hipError_t e = launch_clock2d_begin(h->clk, t, h->stream);
  if (h->cfg.scheme == ADERDG_SCHEME_FV) {
    // ADER-WENO: WENO reconstruction of the averages -> predictor from the
    // nodal WENO values -> update of the averages from the face traces
    if (e == hipSuccess && h->cfg.fixed_dt <= 0.0) e = launch_fv2d_lambda(A, h->stream);
    Args2D P = A;
    P.u = h->w;
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
      A.step = P.step = s;
      e = launch_weno2d(N, A, h->w, h->stream);
      if (e == hipSuccess) e = launch_pred2d(N, h->cfg.precision, P, blocks, h->stream);
      if (e == hipSuccess) e = launch_fv2d_corr(N, A, h->stream);
    }
    if (e == hipSuccess) e = launch_clock2d_end(h->clk, t, dt, status, nsteps & 1, h->stream);
    return e == hipSuccess ? ADERDG_OK : fail_hip(e, "2-D ADER-WENO step launch");
  }
  if (e == hipSuccess && h->cfg.fixed_dt <= 0.0) e = launch_lambda2d(N, A, blocks2, h->stream);
  for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
    A.step = s;
    e = launch_pred2d(N, h->cfg.precision, A, blocks, h->stream);
    if (e == hipSuccess) e = launch_corr2d(N, h->cfg.precision, A, blocks2, h->stream);
  }
  if (e == hipSuccess) e = launch_clock2d_end(h->clk, t, dt, status, nsteps & 1, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "2-D step launch");
}

int aderdg2d_sweep_count(aderdg2d_handle* h, int64_t* sweeps_out) {
  g_last_error.clear();
  if (!h || !sweeps_out) return fail(ADERDG_E_INVAL, "null argument");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "stream synchronisation");
  Slot slots[kSlots];
  e = hipMemcpy(slots, h->clk->sweeps, sizeof(slots), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "sweep count read");
  int64_t total = 0;
  for (int i = 0; i < kSlots; ++i) total += (int64_t)slots[i].v;
  *sweeps_out = total;
  return ADERDG_OK;
}

int aderdg2d_free(aderdg2d_handle* h) {
  if (!h) return ADERDG_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  release2d(h);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "stream synchronisation");
}

}  // extern "C"

// ------------------------------------------------------------------ 3-D ----
struct aderdg3d_handle {
  hipStream_t stream = nullptr;
  aderdg3d_config cfg{};
  int64_t cells = 0;
  double* part = nullptr;
  double* w = nullptr;      // ADER-WENO: nodal WENO values of the averages
  void* tr = nullptr;
  void* qs = nullptr;       // predictor tiles of every cell where they exceed LDS
  Clock3D* clk = nullptr;
};

namespace {

void release3d(aderdg3d_handle* h) {
  if (h->qs) hipFree(h->qs);
  if (h->part) hipFree(h->part);
  if (h->w) hipFree(h->w);
  if (h->tr) hipFree(h->tr);
  if (h->clk) hipFree(h->clk);
  delete h;
}

Args3D args3d(const aderdg3d_handle* h) {
  const aderdg3d_config& c = h->cfg;
  Args3D A{};
  A.c[0] = c.cells_x;
  A.c[1] = c.cells_y;
  A.c[2] = c.cells_z;
  A.h[0] = (c.x1 - c.x0) / (double)c.cells_x;
  A.h[1] = (c.y1 - c.y0) / (double)c.cells_y;
  A.h[2] = (c.z1 - c.z0) / (double)c.cells_z;
  A.cfl = c.cfl;
  A.fixed_dt = c.fixed_dt;
  A.tol = c.picard_tol;
  A.gamma = c.gamma;
  A.max_iter = c.picard_max_iter;
  A.clk = h->clk;
  A.part = h->part;
  A.tr = h->tr;
  A.qs = h->qs;
  A.scheme = c.scheme;
  return A;
}

}  // namespace

extern "C" {

int aderdg3d_init(const aderdg3d_config* cfg, void* hip_stream, aderdg3d_handle** out) {
  g_last_error.clear();
  if (!cfg || !out) return fail(ADERDG_E_INVAL, "null argument");
  aderdg3d_config c = *cfg;
  if (c.precision != ADERDG_FP64 && c.precision != ADERDG_FP32_PREDICTOR)
    return fail(ADERDG_E_INVAL, "unknown precision");
  if (c.scheme != ADERDG_SCHEME_DG && c.scheme != ADERDG_SCHEME_FV) return fail(ADERDG_E_INVAL, "unknown scheme");
  if (c.scheme == ADERDG_SCHEME_FV && (c.N < 1 || c.N > 3 || c.precision != ADERDG_FP64))
    return fail(ADERDG_E_INVAL, "3-D ADER-WENO: N (the WENO degree) must be 1..3, precision FP64");
  if (c.N < 1 || !supported_3d(c.N, c.precision))
    return fail(ADERDG_E_INVAL, "N must be in 1..9");
  if (c.cells_x < 1 || c.cells_y < 1 || c.cells_z < 1 || c.cells_x > INT32_MAX / c.cells_y ||
      c.cells_x * c.cells_y > INT32_MAX / c.cells_z)
    return fail(ADERDG_E_INVAL, "cells_x, cells_y, cells_z must be >= 1 with a product below 2^31");
  const double ext[3] = {c.x1 - c.x0, c.y1 - c.y0, c.z1 - c.z0};
  for (double e : ext)
    if (!(e > 0.0) || !std::isfinite(e)) return fail(ADERDG_E_INVAL, "empty or non-finite domain");
  if (!(c.gamma > 1.0) || !std::isfinite(c.gamma)) return fail(ADERDG_E_INVAL, "gamma must be > 1");
  if (!(c.cfl > 0.0 && c.cfl <= 1.0)) return fail(ADERDG_E_INVAL, "cfl must be in (0, 1]");
  if (!(c.fixed_dt >= 0.0) || !std::isfinite(c.fixed_dt)) return fail(ADERDG_E_INVAL, "fixed_dt must be >= 0");
  if (!std::isfinite(c.picard_tol)) return fail(ADERDG_E_INVAL, "picard_tol must be finite");
  if (c.picard_tol <= 0.0) c.picard_tol = c.precision == ADERDG_FP64 ? 1e-14 : 1e-6;
  if (c.picard_max_iter <= 0) c.picard_max_iter = 64;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  int rc = ensure_tables(device);
  if (rc) return rc;
  aderdg3d_handle* h = new aderdg3d_handle();
  h->stream = (hipStream_t)hip_stream;
  h->cfg = c;
  h->cells = c.cells_x * c.cells_y * c.cells_z;
  const int64_t L = (int64_t)(c.N + 1) * (c.N + 1) * (c.N + 1);
  // DG: u + volume terms; ADER-WENO: the nodal WENO values (the predictor's initial data)
  e = hipMalloc(c.scheme == ADERDG_SCHEME_FV ? (void**)&h->w : (void**)&h->part, sizeof(double) * h->cells * L * 5);
  const size_t tr_elem = c.precision == ADERDG_FP64 ? sizeof(double) : sizeof(float);
  if (e == hipSuccess) e = hipMalloc(&h->tr, tr_elem * h->cells * 6 * L * 5);
  const int64_t tile_bytes = pred3d_tile_bytes_per_cell(c.N, c.precision);
  if (e == hipSuccess && tile_bytes > 0) e = hipMalloc(&h->qs, (size_t)tile_bytes * h->cells);
  if (e != hipSuccess) { release3d(h); return fail(ADERDG_E_NOMEM, "scratch allocation"); }
  e = hipMalloc((void**)&h->clk, sizeof(Clock3D));
  if (e != hipSuccess) { release3d(h); return fail(ADERDG_E_NOMEM, "clock allocation"); }
  e = hipMemset(h->clk, 0, sizeof(Clock3D));
  if (e != hipSuccess) { release3d(h); return fail_hip(e, "clock init"); }
  *out = h;
  return ADERDG_OK;
}

int aderdg3d_predict(aderdg3d_handle* h, const double* u, double t, double dt, void* q_out,
                     int32_t* iters_out) {
  g_last_error.clear();
  if (!h || !u || !q_out) return fail(ADERDG_E_INVAL, "null argument");
  if (h->cfg.scheme != ADERDG_SCHEME_DG) return fail(ADERDG_E_INVAL, "predictor-only calls serve the DG scheme");
  if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(t)) return fail(ADERDG_E_INVAL, "dt must be > 0 and finite");
  Args3D A = args3d(h);
  A.mode = k3dPredict;
  A.t = t;
  A.dt = dt;
  A.u = const_cast<double*>(u);
  A.q_out = q_out;
  A.iters = iters_out;
  const int cpb = cells_per_block_3d(h->cfg.N, h->cfg.precision);
  hipError_t e = launch_pred3d(h->cfg.N, h->cfg.precision, A, (h->cells + cpb - 1) / cpb, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "predictor launch");
}

int aderdg3d_step(aderdg3d_handle* h, double* u, double* t, const double* t_end, double* dt,
                  int32_t* status, int32_t nsteps) {
  g_last_error.clear();
  if (!h || !u || !t || !t_end || !dt || !status) return fail(ADERDG_E_INVAL, "null argument");
  if (nsteps < 0) return fail(ADERDG_E_INVAL, "nsteps must be >= 0");
  Args3D A = args3d(h);
  A.mode = k3dStep;
  A.u = u;
  A.t_end = t_end;
  const int N = h->cfg.N;
  const int cpb = cells_per_block_3d(N, h->cfg.precision), cpb2 = cells_per_block_corr3d(N);
  const int64_t blocks = (h->cells + cpb - 1) / cpb, blocks2 = (h->cells + cpb2 - 1) / cpb2;
  hipError_t e = launch_clock3d_begin(h->clk, t, h->stream);
  if (h->cfg.scheme == ADERDG_SCHEME_FV) {
    // ADER-WENO: WENO reconstruction of the averages -> predictor from the
    // nodal WENO values -> update of the averages from the face traces
    if (e == hipSuccess && h->cfg.fixed_dt <= 0.0) e = launch_fv3d_lambda(A, h->stream);
    Args3D P = A;
    P.u = h->w;
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
      A.step = P.step = s;
      e = launch_weno3d(N, A, h->w, h->stream);
      if (e == hipSuccess) e = launch_pred3d(N, h->cfg.precision, P, blocks, h->stream);
      if (e == hipSuccess) e = launch_fv3d_corr(N, A, h->stream);
    }
    if (e == hipSuccess) e = launch_clock3d_end(h->clk, t, dt, status, nsteps & 1, h->stream);
    return e == hipSuccess ? ADERDG_OK : fail_hip(e, "3-D ADER-WENO step launch");
  }
  if (e == hipSuccess && h->cfg.fixed_dt <= 0.0) e = launch_lambda3d(N, A, blocks2, h->stream);
  for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
    A.step = s;
    e = launch_pred3d(N, h->cfg.precision, A, blocks, h->stream);
    if (e == hipSuccess) e = launch_corr3d(N, h->cfg.precision, A, blocks2, h->stream);
  }
  if (e == hipSuccess) e = launch_clock3d_end(h->clk, t, dt, status, nsteps & 1, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "3-D step launch");
}

int aderdg3d_sweep_count(aderdg3d_handle* h, int64_t* sweeps_out) {
  g_last_error.clear();
  if (!h || !sweeps_out) return fail(ADERDG_E_INVAL, "null argument");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "stream synchronisation");
  Slot slots[kSlots];
  e = hipMemcpy(slots, h->clk->sweeps, sizeof(slots), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "sweep count read");
  int64_t total = 0;
  for (int i = 0; i < kSlots; ++i) total += (int64_t)slots[i].v;
  *sweeps_out = total;
  return ADERDG_OK;
}

int aderdg3d_free(aderdg3d_handle* h) {
  if (!h) return ADERDG_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  release3d(h);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "stream synchronisation");
}

}  // extern "C"

// ------------------------------------------------------------ limited 1-D ----
// A limited handle owns the step's scratch: candidate volume terms, face
// traces and fluxes, the troubled-cell list, subgrid results and a clock.

struct aderdg_lim_handle {
  hipStream_t stream = nullptr;
  aderdg_lim_config cfg{};
  void* scratch = nullptr;
  LimArgs args{};
};

namespace {

void release_lim(aderdg_lim_handle* h) {
  if (h->scratch) hipFree(h->scratch);
  if (h->args.clk) hipFree(h->args.clk);
  delete h;
}

}  // namespace

extern "C" {

int aderdg_lim_init(const aderdg_lim_config* cfg, void* hip_stream, aderdg_lim_handle** out) {
  g_last_error.clear();
  if (!cfg || !out) return fail(ADERDG_E_INVAL, "null argument");
  aderdg_lim_config c = *cfg;
  if (c.N < 1 || c.N > 9) return fail(ADERDG_E_INVAL, "N must be in 1..9");
  if (c.bc != ADERDG_LIM_PERIODIC && c.bc != ADERDG_LIM_TRANSMISSIVE)
    return fail(ADERDG_E_INVAL, "bc must be ADERDG_LIM_PERIODIC or ADERDG_LIM_TRANSMISSIVE");
  if (c.ncells < 3 || c.ncells > (int64_t)INT32_MAX / (2 * c.N + 1))
    return fail(ADERDG_E_INVAL, "ncells must be >= 3 with ncells * (2N+1) below 2^31");
  if (!(c.x1 > c.x0) || !std::isfinite(c.x1 - c.x0)) return fail(ADERDG_E_INVAL, "empty or non-finite domain");
  if (!(c.gamma > 1.0) || !std::isfinite(c.gamma)) return fail(ADERDG_E_INVAL, "gamma must be > 1");
  if (!(c.cfl > 0.0 && c.cfl <= 1.0)) return fail(ADERDG_E_INVAL, "cfl must be in (0, 1]");
  if (c.dims < 1 || c.dims > 3) return fail(ADERDG_E_INVAL, "dims must be 1, 2 or 3");
  if (c.weno_degree == 0) c.weno_degree = 1;
  if (c.weno_degree != 1 && c.weno_degree != 2) return fail(ADERDG_E_INVAL, "weno_degree must be 1 or 2");
  if (c.reserved != 0) return fail(ADERDG_E_INVAL, "reserved must be 0");
  if (!std::isfinite(c.picard_tol)) return fail(ADERDG_E_INVAL, "picard_tol must be finite");
  if (c.picard_tol <= 0.0) c.picard_tol = 1e-14;
  if (c.picard_max_iter <= 0) c.picard_max_iter = 64;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  int rc = ensure_tables(device);
  if (rc) return rc;
  aderdg_lim_handle* h = new aderdg_lim_handle();
  h->stream = (hipStream_t)hip_stream;
  h->cfg = c;
  const int64_t C = c.ncells, n = c.N + 1, Ns = 2 * c.N + 1, M = 3;
  // doubles: vol, trL, trR, G, vext, vfv, gs; then the int32 list
  const int64_t nd = C * n * M + 2 * (C + 2) * n * M + (C + 1) * M + C * 2 * M + C * Ns * M + C * 2 * M;
  // troubled list: kSlots sub-lists, each sized for the cells of its candidate workgroups
  e = hipMalloc(&h->scratch, sizeof(double) * nd + sizeof(int32_t) * (C + (int64_t)(kSlots + 1) * 256));
  if (e != hipSuccess) { release_lim(h); return fail(ADERDG_E_NOMEM, "scratch allocation"); }
  e = hipMalloc((void**)&h->args.clk, sizeof(LimClock));
  if (e != hipSuccess) { release_lim(h); return fail(ADERDG_E_NOMEM, "clock allocation"); }
  e = hipMemset(h->args.clk, 0, sizeof(LimClock));
  if (e != hipSuccess) { release_lim(h); return fail_hip(e, "clock init"); }
  LimArgs& A = h->args;
  A.C = C;
  A.N = c.N;
  A.bc = c.bc;
  A.x0 = c.x0;
  A.dx = (c.x1 - c.x0) / (double)C;
  A.cfl_d = c.cfl / (double)c.dims;
  A.tol = c.picard_tol;
  A.max_iter = c.picard_max_iter;
  A.weno = c.weno_degree;
  A.pp = PdeParams{c.gamma, 0.0, 0.0, 0.0};
  double* d = (double*)h->scratch;
  A.vol = d;  d += C * n * M;
  A.trL = d;  d += (C + 2) * n * M;
  A.trR = d;  d += (C + 2) * n * M;
  A.G = d;    d += (C + 1) * M;
  A.vext = d; d += C * 2 * M;
  A.vfv = d;  d += C * Ns * M;
  A.gs = d;   d += C * 2 * M;
  A.list = (int32_t*)d;
  *out = h;
  return ADERDG_OK;
}

int aderdg_lim_project(aderdg_lim_handle* h, const double* u, double* v) {
  g_last_error.clear();
  if (!h || !u || !v) return fail(ADERDG_E_INVAL, "null argument");
  hipError_t e = launch_lim_project(h->cfg.N, u, v, h->cfg.ncells, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "projection launch");
}

int aderdg_lim_step(aderdg_lim_handle* h, double* u, double* v, int32_t* troubled, double* t,
                    const double* t_end, double* dt, int32_t* status, int32_t nsteps) {
  g_last_error.clear();
  if (!h || !u || !v || !troubled || !t || !t_end || !dt || !status) return fail(ADERDG_E_INVAL, "null argument");
  if (nsteps < 0) return fail(ADERDG_E_INVAL, "nsteps must be >= 0");
  LimArgs A = h->args;
  A.u = u;
  A.v = v;
  A.troubled = troubled;
  A.t_end = t_end;
  hipError_t e = launch_lim_begin(A.clk, t, h->stream);
  if (e == hipSuccess) e = launch_lim_lambda(A, 0, h->stream);
  for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
    A.step = s;
    e = launch_lim_step(A, h->stream);
  }
  if (e == hipSuccess) e = launch_lim_end(A.clk, t, dt, status, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "limited step launch");
}

int aderdg_lim_counters(aderdg_lim_handle* h, int64_t* out4) {
  g_last_error.clear();
  if (!h || !out4) return fail(ADERDG_E_INVAL, "null argument");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "stream synchronisation");
  LimClock c;
  e = hipMemcpy(&c, h->args.clk, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "counter read");
  out4[0] = (int64_t)c.total_troubled;
  out4[1] = (int64_t)c.total_fallback;
  out4[2] = (int64_t)c.total_steps;
  int64_t sw = 0;
  for (int i = 0; i < kSlots; ++i) sw += (int64_t)c.sweeps[i].v;
  out4[3] = sw;
  return ADERDG_OK;
}

int aderdg_lim_free(aderdg_lim_handle* h) {
  if (!h) return ADERDG_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  release_lim(h);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "stream synchronisation");
}

}  // extern "C"

// --------------------------------------------------- limited 2-D step ----
struct aderdg2d_lim_handle {
  hipStream_t stream = nullptr;
  aderdg2d_lim_config cfg{};
  void* scratch = nullptr;
  Clock2D* clk = nullptr;
  Lim2Args args{};
};

namespace {

void release_lim2d(aderdg2d_lim_handle* h) {
  if (h->scratch) hipFree(h->scratch);
  if (h->clk) hipFree(h->clk);
  delete h;
}

}  // namespace

extern "C" {

int aderdg2d_lim_init(const aderdg2d_lim_config* cfg, void* hip_stream, aderdg2d_lim_handle** out) {
  g_last_error.clear();
  if (!cfg || !out) return fail(ADERDG_E_INVAL, "null argument");
  aderdg2d_lim_config c = *cfg;
  if (c.N < 1 || c.N > 9) return fail(ADERDG_E_INVAL, "N must be in 1..9");
  if (c.bc != ADERDG_LIM_PERIODIC && c.bc != ADERDG_LIM_TRANSMISSIVE)
    return fail(ADERDG_E_INVAL, "bc must be ADERDG_LIM_PERIODIC or ADERDG_LIM_TRANSMISSIVE");
  if (c.cells_x < 3 || c.cells_y < 3 || c.cells_x > (1 << 16) || c.cells_y > (1 << 16))
    return fail(ADERDG_E_INVAL, "cells_x and cells_y must be in 3..65536");
  if ((c.cells_x + 2) * (c.cells_y + 2) > ((int64_t)1 << 24))
    return fail(ADERDG_E_INVAL, "at most 2^24 cells with the ghost ring");
  if (!(c.x1 > c.x0) || !(c.y1 > c.y0) || !std::isfinite(c.x1 - c.x0) || !std::isfinite(c.y1 - c.y0))
    return fail(ADERDG_E_INVAL, "empty or non-finite domain");
  if (!(c.gamma > 1.0) || !std::isfinite(c.gamma)) return fail(ADERDG_E_INVAL, "gamma must be > 1");
  if (!(c.cfl > 0.0 && c.cfl <= 1.0)) return fail(ADERDG_E_INVAL, "cfl must be in (0, 1]");
  if (c.reserved != 0) return fail(ADERDG_E_INVAL, "reserved must be 0");
  if (!std::isfinite(c.picard_tol)) return fail(ADERDG_E_INVAL, "picard_tol must be finite");
  if (c.picard_tol <= 0.0) c.picard_tol = 1e-14;
  if (c.picard_max_iter <= 0) c.picard_max_iter = 64;
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  int rc = ensure_tables(device);
  if (rc) return rc;
  aderdg2d_lim_handle* h = new aderdg2d_lim_handle();
  h->stream = (hipStream_t)hip_stream;
  h->cfg = c;
  const int64_t cx = c.cells_x, cy = c.cells_y, P = (cx + 2) * (cy + 2);
  const int64_t n = c.N + 1, L = n * n, Ns = 2 * c.N + 1, M = 4;
  // doubles: up, part, tr (4 faces x L per padded cell), gface, vfv, sflux, uout, vout; then 3 counters
  const int64_t nd = P * L * M * 2 + P * 4 * L * M + P * 2 * n * M + cx * cy * Ns * Ns * M + cx * cy * 4 * Ns * M +
                     cx * cy * L * M + cx * cy * Ns * Ns * M;
  e = hipMalloc(&h->scratch, sizeof(double) * nd + 4 * sizeof(unsigned long long));
  if (e != hipSuccess) { release_lim2d(h); return fail(ADERDG_E_NOMEM, "scratch allocation"); }
  e = hipMalloc((void**)&h->clk, sizeof(Clock2D));
  if (e != hipSuccess) { release_lim2d(h); return fail(ADERDG_E_NOMEM, "clock allocation"); }
  e = hipMemset(h->clk, 0, sizeof(Clock2D));
  if (e == hipSuccess) e = hipMemset(h->scratch, 0, sizeof(double) * nd + 4 * sizeof(unsigned long long));
  if (e != hipSuccess) { release_lim2d(h); return fail_hip(e, "scratch init"); }
  Lim2Args& A = h->args;
  A.cx = cx;
  A.cy = cy;
  A.N = c.N;
  A.bc = c.bc == ADERDG_LIM_PERIODIC ? kLim2Periodic : kLim2Transmissive;
  double* d = (double*)h->scratch;
  A.up = d;       d += P * L * M;
  double* part = d; d += P * L * M;
  double* tr = d;   d += P * 4 * L * M;
  double* gface = d; d += P * 2 * n * M;
  A.vfv = d;      d += cx * cy * Ns * Ns * M;
  A.sflux = d;    d += cx * cy * 4 * Ns * M;
  A.uout = d;     d += cx * cy * L * M;
  A.vout = d;     d += cx * cy * Ns * Ns * M;
  A.cnt = (unsigned long long*)d;
  A.npass = 3;
  Args2D& G = A.dg;
  G.cx = cx + 2;
  G.cy = cy + 2;
  G.dx = (c.x1 - c.x0) / (double)cx;
  G.dy = (c.y1 - c.y0) / (double)cy;
  G.cfl = c.cfl;
  G.tol = c.picard_tol;
  G.gamma = c.gamma;
  G.max_iter = c.picard_max_iter;
  G.mode = k2dStep;
  G.scheme = 0;
  G.clk = h->clk;
  G.u = A.up;
  G.part = part;
  G.tr = tr;
  G.gface = gface;
  G.candidate = 1;
  *out = h;
  return ADERDG_OK;
}

int aderdg2d_lim_project(aderdg2d_lim_handle* h, const double* u, double* v) {
  g_last_error.clear();
  if (!h || !u || !v) return fail(ADERDG_E_INVAL, "null argument");
  Lim2Args A = h->args;
  A.u = const_cast<double*>(u);
  A.v = v;
  hipError_t e = launch_lim2d_project(A, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "projection launch");
}

int aderdg2d_lim_step(aderdg2d_lim_handle* h, double* u, double* v, int32_t* troubled, double* t,
                      const double* t_end, double* dt, int32_t* status, int32_t nsteps) {
  g_last_error.clear();
  if (!h || !u || !v || !troubled || !t || !t_end || !dt || !status) return fail(ADERDG_E_INVAL, "null argument");
  if (nsteps < 0) return fail(ADERDG_E_INVAL, "nsteps must be >= 0");
  Lim2Args A = h->args;
  A.u = u;
  A.v = v;
  A.troubled = troubled;
  A.dg.t_end = t_end;
  const int N = h->cfg.N;
  const int64_t P = A.dg.cx * A.dg.cy;
  const int64_t cpb = cells_per_block_2d(N, ADERDG_FP64), cpc = cells_per_block_corr2d(N);
  hipError_t e = launch_clock2d_begin(A.dg.clk, t, h->stream);
  if (e == hipSuccess) e = launch_lim2d_copy(A, 1, h->stream);
  if (e == hipSuccess) e = launch_lim2d_ghosts(A, h->stream);
  if (e == hipSuccess) e = launch_lambda2d(N, A.dg, (P + cpc - 1) / cpc, h->stream);
  for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
    A.dg.step = s;
    if (s > 0) e = launch_lim2d_ghosts(A, h->stream);
    if (e == hipSuccess) e = launch_pred2d(N, ADERDG_FP64, A.dg, (P + cpb - 1) / cpb, h->stream);
    if (e == hipSuccess) e = launch_corr2d(N, ADERDG_FP64, A.dg, (P + cpc - 1) / cpc, h->stream);
    if (e == hipSuccess) e = launch_lim2d_after_candidate(A, h->stream);
  }
  if (e == hipSuccess) e = launch_lim2d_copy(A, 0, h->stream);
  if (e == hipSuccess) e = launch_clock2d_end(A.dg.clk, t, dt, status, nsteps & 1, h->stream);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "limited 2-D step launch");
}

int aderdg2d_lim_counters(aderdg2d_lim_handle* h, int64_t* out4) {
  g_last_error.clear();
  if (!h || !out4) return fail(ADERDG_E_INVAL, "null argument");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(e, "stream synchronisation");
  unsigned long long cnt[3];
  e = hipMemcpy(cnt, h->args.cnt, sizeof(cnt), hipMemcpyDeviceToHost);
  Clock2D clk;
  if (e == hipSuccess) e = hipMemcpy(&clk, h->clk, sizeof(clk), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "counter read");
  out4[0] = (int64_t)cnt[0];
  out4[1] = (int64_t)cnt[1];
  out4[2] = 0;
  int64_t sw = 0;
  for (int i = 0; i < kSlots; ++i) sw += (int64_t)clk.sweeps[i].v;
  out4[3] = sw;
  return ADERDG_OK;
}

int aderdg2d_lim_free(aderdg2d_lim_handle* h) {
  if (!h) return ADERDG_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  release_lim2d(h);
  return e == hipSuccess ? ADERDG_OK : fail_hip(e, "stream synchronisation");
}

}  // extern "C"
