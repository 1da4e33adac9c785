// api.hip -- C ABI of libdfmesh (include/df.h): run handles, arena layout,
// the recursive sub-cycling scheduler and the host side of the reductions.
//
// Scheduling (Velasco Romero & Masset 2018, Sects. 3.1 and 3.3): one coarse
// step computes the time step on the device (Courant and diffusion limits of
// every level, eq. 55 with two sub-cycles per level), then runs Cycle(0):
//   Cycle(l): [Cycle(l+1) twice, finer level first] ; level step on l ;
//             CommUp l -> l+1 ; CommMean l+1 -> l
// Every launch goes to the caller's stream; nothing in df_step waits on the
// device, so a sequence of steps can be captured into a HIP graph.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "df.h"
#include "dfk.h"

using dfk::Geo;
using dfk::LevBufs;
using dfk::MAXLEV;
using dfk::NQ;
using dfk::Phys;
using dfk::Scal;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_check(hipError_t e, const char *where) {
  if (e == hipSuccess) return DF_OK;
  return fail(DF_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

int launch_check(const char *where) { return hip_check(hipGetLastError(), where); }

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

}  // namespace

int df_fail_internal(int code, const char *msg) { return fail(code, msg); }

struct df_run {
  df_mesh_desc desc{};
  int nl = 0;
  Geo geo[MAXLEV]{};
  Phys phys{};
  LevBufs buf[MAXLEV]{};
  int cur[MAXLEV]{};
  size_t vol[MAXLEV]{};
  size_t acc_n[MAXLEV]{};
  size_t npart[MAXLEV]{};
  // finer levels: cells beyond the active range along each dimension that
  // CommUp into the next finer level reads after a step (0 for the finest)
  int mobs[MAXLEV][3]{};
  size_t need = 0;
  char *base = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  Scal *scal = nullptr;
  double *flog = nullptr;
  size_t esz = 8;      // bytes per stored value (8 FP64, 4 FP32)
  int chunk = 16;      // column segment of the streaming passes
  bool bound = false;
  bool ready = false;
  bool sig_valid = false;  // the signal-speed partials are those of the current state
  bool fuse_xy = true;     // fuse the x and y passes where transport_xy applies
  bool fuse_kc = true;     // fuse the first kick and the compression of level 0 (viscosity off)
  bool fuse_zf = true;     // fuse the z pass with the rebuild, the kick and the end-of-step partials (single level)
  bool slot_mode = false;  // single level: the kicks take the step length from the signal-speed slots
  int subcycle = 0;        // 0: two sub-steps per level; 1: criterion of App. A
  double visc = 0.0;       // artificial-viscosity coefficient (kept across df_set_perturber)
  int xi[MAXLEV];          // sub-steps of level l+1 per step of level l (last coarse step)
  double up[MAXLEV + 1];   // staging of the host-chosen step lengths and time
  double eps = 0.0;
  bool quad = false;   // the domain is the quadrant y, z > 0 (Sect. 3.4)
  double mult = 1.0;   // copies of the domain in the whole gas (4 on the quadrant)
  // nested runs: df_step replays a HIP graph of two coarse steps (which bring
  // every buffer back to its role), one per pattern of the levels' current
  // sets, captured on a private stream; any call that changes a launch's
  // arguments or form marks them stale
  bool use_graphs = true;
  bool graphs_stale = false;
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  unsigned gpat[2] = {0, 0};
  // optional per-kernel-kind timing: event pairs around launches
  bool timing = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
};

namespace {

// ----------------------------------------------------------- arena layout
struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

// floor(i / 2)
int fdiv2_i(int i) { return (i >= 0) ? i / 2 : -((1 - i) / 2); }

void carve(df_run *R, char *base) {
  Carver c{base};
  R->scal = c.take<Scal>(1);
  R->flog = c.take<double>(4 * (size_t)dfk::FLOG);
  const size_t e = R->esz;
  for (int l = 0; l < R->nl; ++l) {
    LevBufs &B = R->buf[l];
    const size_t v = R->vol[l] * e;
    for (int s = 0; s < 2; ++s)
      for (int m = 0; m < NQ; ++m) B.q[s][m] = c.take<char>(v);
    for (int d = 0; d < 3; ++d) B.v[d] = c.take<char>(v);
    // the kicked faces of a fused kick and compression (level 0; the finer
    // levels in FP32, where the fused launch is the faster)
    const bool kcl = l == 0 || R->esz == 4;
    for (int d = 0; d < 3; ++d) B.vk[d] = kcl ? (void *)c.take<char>(v) : nullptr;
    B.etmp = c.take<char>(v);
    B.acc = R->acc_n[l] ? (void *)c.take<char>(R->acc_n[l] * e) : nullptr;
    const Geo &G = R->geo[l];
    B.hw = c.take<double>((size_t)G.n[0] * G.n[1] * G.n[2]);
    B.part = c.take<double>(4 * R->npart[l]);
  }
  R->need = c.off;
}

// ------------------------------------------------------- heat-release weights
// Normalised Gaussian weights of standard deviation sigma = eps over the
// active cells of a level, truncated at r_min + 8 sigma, r_min the distance of
// the eight cells around the perturber's vertex; sigma = 0 gives those eight
// cells 1/8 each (the split of Sect. 3.4).  Stored on the smallest centred box
// of active cells that holds every non-zero weight.
// On the quadrant the box starts at the mirror planes and the weights are
// normalised over the cells and their mirror images (mult copies): the
// domain's cells take a quarter of the release, each its full-box share.
void heat_table(const Geo &G, double sigma, double mult, std::vector<double> &w, int edge[3]) {
  double dx = G.dx;
  auto cen = [&](int d, int i) { return ((double)i - G.org[d] + 0.5) * dx; };
  double r2min = 3.0 * (0.5 * dx) * (0.5 * dx);
  double rcut = std::sqrt(r2min) + 8.0 * sigma;
  int half = (sigma == 0.0) ? 1 : (int)std::ceil(rcut / dx) + 1;
  for (int d = 0; d < 3; ++d) {
    const int want = G.anch[d] ? half : 2 * half;
    edge[d] = want < G.n[d] ? want : G.n[d];
  }
  w.assign((size_t)edge[0] * edge[1] * edge[2], 0.0);
  double sum = 0.0;
  auto first = [&](int d) { return G.anch[d] ? 0 : G.n[d] / 2 - edge[d] / 2; };
  for (int c = 0; c < edge[2]; ++c)
    for (int b = 0; b < edge[1]; ++b)
      for (int a = 0; a < edge[0]; ++a) {
        int i = first(0) + a, j = first(1) + b, k = first(2) + c;
        double x = cen(0, i), y = cen(1, j), z = cen(2, k);
        double r2 = x * x + y * y + z * z;
        double g = 0.0;
        if (sigma == 0.0) g = (r2 <= r2min * (1.0 + 1e-12)) ? 1.0 : 0.0;
        else if (std::sqrt(r2) <= rcut) g = std::exp(-(r2 - r2min) / (2.0 * sigma * sigma));
        w[((size_t)c * edge[1] + b) * edge[0] + a] = g;
        sum += g;
      }
  for (double &x : w) x /= sum * mult;
}

// ---------------------------------------------------------------- timing
// Kernel kinds timed by df_timing_read (the order of the DF_K_* list in df.h).
enum { K_KICK = 0, K_COMPRESS, K_DIFFUSE, K_PASSX, K_PASSY, K_PASSZ, K_REBUILD, K_COMMUP, K_COMMMEAN,
       K_DT, K_FORCE, K_ZERO, K_VISC, K_PASSXY, K_KICKCOMP, K_ZFINISH, K_NKINDS };
static_assert(K_NKINDS == DF_K_NKINDS, "timing kinds follow the DF_K_* list");

struct TScope {
  df_run *R;
  bool on;
  TScope(df_run *r, int kind) : R(r), on(r->timing && r->ev_used + 1 < r->ev.size()) {
    // a record that fails leaves its event unrecorded, which df_timing_read
    // reports when it takes the pair's elapsed time
    if (on) {
      R->ev_kind[R->ev_used / 2] = kind;
      (void)hipEventRecord(R->ev[R->ev_used], R->stream);
    }
  }
  ~TScope() {
    if (on) {
      (void)hipEventRecord(R->ev[R->ev_used + 1], R->stream);
      R->ev_used += 2;
    }
  }
};

// ------------------------------------------------------------- scheduler
// A finer level's step computes, in each stage, only the entries that later
// stages, later sub-steps before the next ghost fill (rem of them) and CommUp
// into the next finer level read: with the step's output needed to a margin m
// beyond the active range, the rebuild and kick needs the z pass's cells to
// m + 1, the z pass the y pass's to m + 1 (m + 3 along z), the y pass the x
// pass's to m + 1 (m + 3 along y and z), the x pass the diffused energy and the
// kicked faces to m + 3, the diffusion the compressed energy to m + 4, the
// compression (and the viscosity) the kicked faces to m + 4, and the first kick
// the state's cells to m + 5 (one more with viscosity): a step reaches 5 (6)
// cells.  Every stage keeps its own bounds (the ghost shell) as well, so the
// entries computed are those of the whole-shell update within the margins.
void level_step(df_run *R, int l, const double *dtp, double scale, int rem) {
  hipStream_t st = R->stream;
  const Geo &G0 = R->geo[l];
  LevBufs &B = R->buf[l];
  const Phys &P = R->phys;
  int c = R->cur[l];
  const int vs = P.visc > 0.0 ? 1 : 0;
  int mo[3];
  for (int d = 0; d < 3; ++d) mo[d] = R->mobs[l][d] + rem * (5 + vs);
  auto stage = [&](int a, int b, int cc) {
    Geo g = G0;
    if (!g.bc) {
      g.mg[0] = mo[0] + a;
      g.mg[1] = mo[1] + b;
      g.mg[2] = mo[2] + cc;
    }
    return g;
  };
  const Geo Gk = stage(4 + vs, 4 + vs, 4 + vs), Gc = stage(4, 4, 4), Gd = stage(3, 3, 3);
  const Geo Gx = stage(1, 3, 3), Gy = stage(1, 1, 3), Gz = stage(1, 1, 1), Grk = stage(0, 0, 0);
  const Geo &G = G0;
  const Geo *Gf = (l + 1 < R->nl) ? &R->geo[l + 1] : nullptr;
  const void *facc = Gf ? R->buf[l + 1].acc : nullptr;
  // single level: the kick sets this step's length from the last end-of-step
  // pass's signal speeds, and the compression logs that pass's force
  Scal *slots = R->slot_mode ? R->scal : nullptr;
  // the first kick and the compression may run as one launch (level 0, and
  // the finer levels in FP32: in FP64 their fused launch, which kicks the
  // high y and z faces of each cell again, made a run of 4 levels of 128^3
  // 0.5-2 % slower than the two launches); the transport passes then read
  // the kicked velocities from vk, and the energy goes q[c][1] -> etmp
  // (compression) -> q[c][1] (diffusion)
  const bool kc = R->fuse_kc && B.vk[0] && !(P.visc > 0.0);
  LevBufs Bt = B;  // buffers the transport passes read
  if (kc) {
    {
      TScope t(R, K_KICKCOMP);
      if (G.bc) dfk::kick_compress(st, G, P, B, c, dtp, 0.5 * scale, scale, slots, R->flog);
      else dfk::kick_compress_fine(st, Gk, Gc, P, B, c, dtp, 0.5 * scale, scale);
    }
    LevBufs Bd = B;
    Bd.q[c][1] = B.etmp;
    Bd.etmp = B.q[c][1];
    { TScope t(R, K_DIFFUSE); dfk::diffuse_heat(st, G.bc ? G : Gd, P, Bd, c, dtp, scale, true, true, slots); }
    for (int d = 0; d < 3; ++d) Bt.v[d] = B.vk[d];
  } else {
    { TScope t(R, K_KICK); dfk::kick(st, Gk, P, B, c, dtp, 0.5 * scale, slots); }
    if (P.visc > 0.0) { TScope t(R, K_VISC); dfk::viscosity(st, Gc, P, B, c, dtp, scale); }
    { TScope t(R, K_COMPRESS); dfk::compress(st, Gc, P, B, c, dtp, scale, slots, R->flog); }
    { TScope t(R, K_DIFFUSE); dfk::diffuse_heat(st, Gd, P, B, c, dtp, scale, true, true); }
  }
  // the x pass reads the new energy from the diffusion output; every buffer
  // keeps its role, so the launches of two consecutive steps repeat exactly
  LevBufs Bx = Bt;
  if (!kc) Bx.q[c][1] = B.etmp;
  // level 0: the x and y passes in one launch, q[c] -> q[1-c] (under a finer
  // level with flux matching on its frontier)
  const bool fused = R->fuse_xy && dfk::transport_xy_fits(G);
  // a finer level: its x and y passes in one launch too, unless the
  // quadrant's images must be set between them (a middle level)
  const bool fused_fine = R->fuse_xy && !G.bc && !(R->quad && Gf);
  if (fused) {
    TScope t(R, K_PASSXY);
    dfk::transport_xy(st, G, P, Bx, c, dtp, scale, R->chunk, Gf, facc);
  } else if (fused_fine) {
    TScope t(R, K_PASSXY);
    dfk::transport_xy_fine(st, Gy, P, Bx, c, dtp, scale, Gf, facc, R->chunk);
  } else {
    // quadrant: a middle level takes the finer level's frontier transfers,
    // whose images lie beyond the planes: the transported set's images are
    // set again after every pass
    const bool mq = Gf && G.level > 0;
    { TScope t(R, K_PASSX); dfk::transport_pass(st, 0, Gx, P, Bx, c, dtp, scale, Gf, facc, R->chunk); }
    if (mq) dfk::mirror_q(st, G, P, B, 1 - c);
    { TScope t(R, K_PASSY); dfk::transport_pass(st, 1, Gy, P, Bt, 1 - c, dtp, scale, Gf, facc, R->chunk); }
    if (mq) dfk::mirror_q(st, G, P, B, c);
  }
  // the z pass and the rebuild take the set the y pass wrote (q[c] after
  // separate passes, q[1-c] after the fused ones)
  const int cy = (fused || fused_fine) ? 1 - c : c;
  // a single-level step ends here: the same launch forms the force and the
  // next step's signal-speed partials; on level 0 without a finer level the z
  // pass joins them (only the new density, energy and face velocities are
  // written)
  Scal *post = R->nl == 1 ? R->scal : nullptr;
  bool zf = false;
  if (R->fuse_zf && post && dfk::transport_z_finish_fits(G)) {
    TScope t(R, K_ZFINISH);
    zf = dfk::transport_z_finish(st, G, P, B, Bt.v, cy, dtp, scale, 0.5 * scale, post, R->chunk);
  }
  if (!zf) {
    { TScope t(R, K_PASSZ); dfk::transport_pass(st, 2, Gz, P, Bt, cy, dtp, scale, Gf, facc, R->chunk); }
    if (Gf && G.level > 0) dfk::mirror_q(st, G, P, B, 1 - cy);
    { TScope t(R, K_REBUILD); dfk::rebuild_kick(st, Grk, P, B, 1 - cy, dtp, 0.5 * scale, true, post); }
  }
  R->cur[l] = 1 - cy;
}

// one step of level l and, first, the xi[l] sub-steps of the finer levels
// under it; rem: sub-steps of level l that follow this one before its next
// ghost fill
void cycle(df_run *R, int l, int rem = 0) {
  if (l + 1 < R->nl) {
    { TScope t(R, K_ZERO); dfk::zero(R->stream, R->buf[l + 1].acc, R->acc_n[l + 1] * R->esz); }
    for (int sub = 0; sub < R->xi[l]; ++sub) cycle(R, l + 1, R->xi[l] - 1 - sub);
  }
  level_step(R, l, &R->scal->dt[l], 1.0, rem);
  if (l + 1 < R->nl) {
    { TScope t(R, K_COMMUP);
      dfk::commup(R->stream, R->geo[l], R->phys, R->buf[l], R->cur[l], R->geo[l + 1], R->buf[l + 1],
                  R->cur[l + 1]);
      // quadrant: the finer level's entries beyond the planes are its images
      dfk::mirror_state(R->stream, R->geo[l + 1], R->phys, R->buf[l + 1], R->cur[l + 1]); }
    { TScope t(R, K_COMMMEAN);
      dfk::commmean(R->stream, R->geo[l + 1], R->phys, R->buf[l + 1], R->cur[l + 1], R->geo[l], R->buf[l],
                    R->cur[l]);
      // and so are the images of the cells the restriction overwrote
      dfk::mirror_state(R->stream, R->geo[l], R->phys, R->buf[l], R->cur[l]); }
  }
}

void compute_dt(df_run *R, int advance) {
  TScope t(R, K_DT);
  for (int l = 0; l < R->nl; ++l) dfk::signal_speed(R->stream, R->geo[l], R->phys, R->buf[l], R->cur[l], R->scal);
  dfk::dt_final(R->stream, R->geo, R->buf, R->nl, R->phys, R->scal, advance);
}

// force of the current state (eq. 18); slot 2 also appends it to the log
void force_reduce(df_run *R, int slot) {
  TScope t(R, K_FORCE);
  double *parts[MAXLEV];
  int np[MAXLEV];
  for (int l = 0; l < R->nl; ++l) {
    np[l] = slot == 1 ? dfk::totals_partials(R->stream, R->geo[l], R->phys, R->buf[l], R->cur[l])
                      : dfk::force_partials(R->stream, R->geo[l], R->phys, R->buf[l], R->cur[l]);
    parts[l] = R->buf[l].part;
  }
  dfk::force_final(R->stream, parts, np, R->nl, R->scal, slot, R->flog);
}

void sync_levels(df_run *R) {
  for (int l = R->nl - 2; l >= 0; --l) {
    dfk::commmean(R->stream, R->geo[l + 1], R->phys, R->buf[l + 1], R->cur[l + 1], R->geo[l], R->buf[l],
                  R->cur[l]);
    dfk::mirror_state(R->stream, R->geo[l], R->phys, R->buf[l], R->cur[l]);
  }
  for (int l = 0; l + 1 < R->nl; ++l) {
    dfk::commup(R->stream, R->geo[l], R->phys, R->buf[l], R->cur[l], R->geo[l + 1], R->buf[l + 1],
                R->cur[l + 1]);
    dfk::mirror_state(R->stream, R->geo[l + 1], R->phys, R->buf[l + 1], R->cur[l + 1]);
  }
}

void *field_ptr(df_run *R, int l, int f) {
  LevBufs &B = R->buf[l];
  if (f == DF_RHO) return B.q[R->cur[l]][0];
  if (f == DF_E) return B.q[R->cur[l]][1];
  return B.v[f - DF_VX];
}

int check_run(const df_run *R, bool need_ready) {
  if (!R) return fail(DF_EINVAL, "null run handle");
  if (!R->bound) return fail(DF_ESTATE, "run not bound to an arena (df_bind)");
  if (need_ready && !R->ready) return fail(DF_ESTATE, "perturber not set (df_set_perturber)");
  return DF_OK;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

// n coarse steps: device time step, recursive cycle, force into the log
// signal-speed and force partials of the current state (post_partials)
void post_reduce(df_run *R) {
  dfk::zero(R->stream, R->scal->smax, sizeof(R->scal->smax));  // the pass refills the signal-speed slots
  for (int l = 0; l < R->nl; ++l) dfk::post_partials(R->stream, R->geo[l], R->phys, R->buf[l], R->cur[l], R->scal);
  R->sig_valid = true;
}

// Sub-cycling criterion of App. A on the host: for per-level limits dtl and
// costs of one level step taken as its active cells, the word xi in {1,2}^(nl-1)
// of largest coarse step min_l dtl[l] prod_{m<l} xi[m] (eq. 55) per cost
// sum_l C_l prod_{m<l} xi[m] (eq. 56).  Words are tried from all-2 down (bit m
// set: xi[m] = 2) and a later word must do strictly better.  Returns the
// coarse step.
double schedule_criterion(const df_run *R, const double *dtl, int *xi) {
  const int nl = R->nl;
  double best_ratio = -1.0, best_dt = 0.0;
  for (long w = (1L << (nl - 1)) - 1; w >= 0; --w) {
    double dt = INFINITY, cost = 0.0, mult = 1.0;
    for (int l = 0; l < nl; ++l) {
      dt = fmin(dt, dtl[l] * mult);
      cost += (double)R->geo[l].n[0] * R->geo[l].n[1] * R->geo[l].n[2] * mult;
      if (l + 1 < nl) mult *= ((w >> l) & 1) ? 2.0 : 1.0;
    }
    const double ratio = dt / cost;
    if (ratio > best_ratio) {
      best_ratio = ratio;
      best_dt = dt;
      for (int m = 0; m + 1 < nl; ++m) xi[m] = ((w >> m) & 1) ? 2 : 1;
    }
  }
  return best_dt;
}

static_assert(offsetof(Scal, t) == MAXLEV * sizeof(double), "the step lengths and the time are uploaded together");

// one coarse step under the criterion: read the per-level limits back, choose
// the schedule, upload the step lengths and the new time, advance, log the force
int criterion_step(df_run *R) {
  if (!R->sig_valid) post_reduce(R);
  dfk::step_final(R->stream, R->geo, R->buf, R->nl, R->phys, R->scal, R->flog, 0, 2);
  Scal h;
  int rc = hip_check(hipMemcpyAsync(&h, R->scal, sizeof(Scal), hipMemcpyDeviceToHost, R->stream), "limits copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(R->stream), "limits copy");
  if (rc) return rc;
  const double dt0 = schedule_criterion(R, h.dtl, R->xi);
  for (int l = 0; l < MAXLEV; ++l) R->up[l] = 0.0;
  R->up[0] = dt0;
  for (int l = 1; l < R->nl; ++l) R->up[l] = R->xi[l - 1] == 2 ? 0.5 * R->up[l - 1] : R->up[l - 1];
  R->up[MAXLEV] = h.t + dt0;  // dt[] and t are adjacent in Scal
  rc = hip_check(hipMemcpyAsync(R->scal->dt, R->up, sizeof(R->up), hipMemcpyHostToDevice, R->stream),
                 "step upload");
  if (rc) return rc;
  cycle(R, 0);
  post_reduce(R);
  dfk::step_final(R->stream, R->geo, R->buf, R->nl, R->phys, R->scal, R->flog, 1, 0);
  return launch_check("df_step");
}

// n coarse steps, each: time step from the signal speeds of the state,
// cycle, force of the new state logged.  One pass after each step gives both
// the force and the next step's signal speeds, and one block kernel between
// two steps logs the force and sets the next time step.
void enqueue_steps(df_run *R, int n) {
  if (n <= 0) return;
  if (R->nl == 1 && R->geo[0].bc && R->geo[0].n[0] % 2 == 0) {
    // single level: no launch between two steps.  Each first kick takes the
    // step length from the slots of the end-of-step pass before it (the
    // rebuild kick, or the signal pass of a changed state), each compression
    // logs the force of the state the step started from, and one kernel logs
    // the last step's force.
    if (!R->sig_valid) {
      TScope t(R, K_DT);
      post_reduce(R);
    }
    R->slot_mode = true;
    for (int s = 0; s < n; ++s) cycle(R, 0);
    R->slot_mode = false;
    {
      TScope t(R, K_FORCE);
      dfk::log_pending(R->stream, R->geo[0], R->buf[0], R->scal, R->flog);
    }
    R->sig_valid = true;
    return;
  }
  if (!R->sig_valid) {
    TScope t(R, K_DT);
    post_reduce(R);
  }
  {
    TScope t(R, K_DT);
    dfk::step_final(R->stream, R->geo, R->buf, R->nl, R->phys, R->scal, R->flog, 0, 1);
  }
  for (int s = 0; s < n; ++s) {
    cycle(R, 0);
    TScope t(R, K_FORCE);
    if (R->nl > 1) post_reduce(R);  // single level: formed by the last kick
    dfk::step_final(R->stream, R->geo, R->buf, R->nl, R->phys, R->scal, R->flog, 1, s + 1 < n);
  }
  R->sig_valid = true;
}

unsigned cur_pattern(const df_run *R) {
  unsigned p = 0;
  for (int l = 0; l < R->nl; ++l) p |= (unsigned)R->cur[l] << l;
  return p;
}

// destroy the step graphs (after the stream has run every replay)
int drop_graphs(df_run *R) {
  int rc = DF_OK;
  if (R->gexec[0] || R->gexec[1]) rc = hip_check(hipStreamSynchronize(R->stream), "graph release");
  for (int s = 0; s < 2; ++s) {
    if (R->gexec[s]) (void)hipGraphExecDestroy(R->gexec[s]);
    R->gexec[s] = nullptr;
  }
  R->graphs_stale = false;
  return rc;
}

// k replays of two coarse steps each: the arithmetic of enqueue_steps(R, 2k)
// (the step length of each replay's first step is taken from the same
// partials by the replay's opening reduction), so the results are bitwise
// those of the eager steps
int graph_steps(df_run *R, int k) {
  int rc = DF_OK;
  if (R->graphs_stale) rc = drop_graphs(R);
  if (rc) return rc;
  if (!R->sig_valid) post_reduce(R);  // eagerly: the graph starts from valid partials
  const unsigned pat = cur_pattern(R);
  int s = -1;
  for (int q = 0; q < 2; ++q)
    if (R->gexec[q] && R->gpat[q] == pat) s = q;
  if (s < 0) {
    s = R->gexec[0] ? 1 : 0;
    if (R->gexec[s]) {
      rc = hip_check(hipStreamSynchronize(R->stream), "graph release");
      if (rc) return rc;
      (void)hipGraphExecDestroy(R->gexec[s]);
      R->gexec[s] = nullptr;
    }
    if (!R->gstream) {
      rc = hip_check(hipStreamCreateWithFlags(&R->gstream, hipStreamNonBlocking), "graph stream");
      if (rc) return rc;
    }
    rc = hip_check(hipStreamBeginCapture(R->gstream, hipStreamCaptureModeRelaxed), "graph capture");
    if (rc) return rc;
    // the capture records the launches without running them: the levels'
    // buffer roles it advances are put back if it fails
    int cur0[MAXLEV];
    std::copy(R->cur, R->cur + R->nl, cur0);
    hipStream_t user = R->stream;
    R->stream = R->gstream;
    enqueue_steps(R, 2);
    R->stream = user;
    hipGraph_t g = nullptr;
    rc = hip_check(hipStreamEndCapture(R->gstream, &g), "graph capture end");
    if (!rc) {
      rc = hip_check(hipGraphInstantiate(&R->gexec[s], g, nullptr, nullptr, 0), "graph instantiate");
      if (rc) R->gexec[s] = nullptr;
    }
    if (g) (void)hipGraphDestroy(g);
    if (!rc && cur_pattern(R) != pat) {
      (void)hipGraphExecDestroy(R->gexec[s]);
      R->gexec[s] = nullptr;
      rc = fail(DF_ESTATE, "two coarse steps did not restore the buffer roles");
    }
    if (rc) {
      std::copy(cur0, cur0 + R->nl, R->cur);
      return rc;
    }
    R->gpat[s] = pat;
  }
  for (int i = 0; i < k && !rc; ++i) rc = hip_check(hipGraphLaunch(R->gexec[s], R->stream), "graph launch");
  return rc;
}

}  // namespace

// ================================================================== ABI

extern "C" {

const char *df_strerror(int code) {
  switch (code) {
    case DF_OK: return "ok";
    case DF_EINVAL: return "invalid argument";
    case DF_ESTATE: return "call out of order";
    case DF_ENOMEM: return "arena too small";
    case DF_EDEVICE: return "HIP runtime error";
    case DF_ENUMERIC: return "non-positive or non-finite density or energy";
    case DF_EBUSY: return "no free slot or HBM budget";
    default: return "unknown error";
  }
}

const char *df_last_error(void) { return g_last_error.c_str(); }

int df_init_mesh(const df_mesh_desc *d, df_run **out) {
  if (!d || !out) return fail(DF_EINVAL, "null argument");
  *out = nullptr;
  if (d->nlevels < 1 || d->nlevels > MAXLEV) return fail(DF_EINVAL, "nlevels must be 1..12");
  const int n[3] = {d->nx, d->ny, d->nz};
  for (int k = 0; k < 3; ++k) {
    if (n[k] < 2 || (n[k] % 2) != 0 || n[k] > 4096) return fail(DF_EINVAL, "cell counts must be even, 2..4096");
    if (d->nlevels > 1 && (n[k] % 4 != 0 || n[k] < 16))
      return fail(DF_EINVAL, "nested runs need cell counts that are multiples of 4 and >= 16");
  }
  if (d->quadrant != 0 && d->quadrant != 1) return fail(DF_EINVAL, "quadrant must be 0 or 1");
  // cells of the finer levels (0: those of level 0)
  const bool own1 = d->nx1 != 0 || d->ny1 != 0 || d->nz1 != 0;
  const int n1[3] = {own1 ? d->nx1 : d->nx, own1 ? d->ny1 : d->ny, own1 ? d->nz1 : d->nz};
  for (int k = 0; k < 3 && own1; ++k)
    if (n1[k] % 4 != 0 || n1[k] < 16 || n1[k] / 2 > n[k] || n1[k] > 4096)
      return fail(DF_EINVAL, "finer-level cell counts must be multiples of 4, >= 16 and at most twice level 0's");
  if (!(d->dx0 > 0.0) || !std::isfinite(d->dx0)) return fail(DF_EINVAL, "dx0 must be positive");
  if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) return fail(DF_EINVAL, "gamma must exceed 1");
  if (!(d->cfl > 0.0) || d->cfl > 1.0) return fail(DF_EINVAL, "cfl must be in (0, 1]");
  if (d->precision != DF_FP64 && d->precision != DF_FP32) return fail(DF_EINVAL, "unknown precision");
  int gf = d->ghost_fine == 0 ? 10 : d->ghost_fine;
  if (d->nlevels > 1 && (gf < 10 || gf > 16)) return fail(DF_EINVAL, "ghost_fine must be 10..16");
  if (!std::isfinite(d->noise_amp) || std::fabs(d->noise_amp) >= 0.5) return fail(DF_EINVAL, "noise_amp out of range");
  if (d->tile_chunk != 0 && (d->tile_chunk < 2 || d->tile_chunk > 256)) return fail(DF_EINVAL, "tile_chunk must be 2..256");

  df_run *R = new df_run();
  R->desc = *d;
  R->nl = d->nlevels;
  R->esz = d->precision == DF_FP32 ? 4 : 8;
  // the finer levels' one-column walks (FP64, 4 waves per SIMD) hide their
  // latency with more, shorter segments: on 4 levels of 128^3, 8 cells run the
  // coarse step 5 % faster than 32, which suits level 0's fused passes
  R->chunk = d->tile_chunk ? d->tile_chunk : (d->precision == DF_FP32 ? 16 : (d->nlevels > 1 ? 8 : 32));
  R->quad = d->quadrant == 1;
  R->mult = R->quad ? 4.0 : 1.0;
  for (int m = 0; m < MAXLEV; ++m) R->xi[m] = 2;
  R->phys.fp32 = d->precision == DF_FP32;
  for (int l = 0; l < R->nl; ++l) {
    Geo &G = R->geo[l];
    for (int k = 0; k < 3; ++k) G.n[k] = l == 0 ? n[k] : n1[k];
    G.g = (l == 0) ? 0 : gf;
    for (int k = 0; k < 3; ++k) G.s[k] = (l == 0) ? G.n[k] + 1 : G.n[k] + 2 * G.g;
    // x = 0 of each row on a 128-byte boundary (16 doubles)
    const int px = (G.g + 15) / 16 * 16;
    G.sy = (px + G.s[0] - G.g + 15) / 16 * 16;
    G.sz = G.sy * G.s[1];
    G.off = px + G.g * G.sy + G.g * G.sz;
    G.dx = std::ldexp(d->dx0, -l);
    G.level = l;
    // the quadrant's level 0 takes the boundary list of Sect. 3.4
    G.bc = (l == 0) ? (R->quad ? 2 : 1) : 0;
    G.has_fine = (l + 1 < R->nl);
    // the finer level's cells cover the central n1/2 cells of this one (on
    // the quadrant: from the mirror planes along y and z)
    for (int k = 0; k < 3; ++k) {
      G.anch[k] = R->quad && k > 0;
      G.org[k] = G.anch[k] ? 0.0 : 0.5 * (double)G.n[k];
      G.cn[k] = G.has_fine ? n1[k] / 2 : 0;
      G.co[k] = G.has_fine ? (G.anch[k] ? 0 : (G.n[k] - G.cn[k]) / 2) : 0;
      G.mg[k] = 1 << 20;  // no margin: the whole stored box
    }
    R->vol[l] = (size_t)G.sz * G.s[2];
    if (R->vol[l] >= ((size_t)1 << 31)) {
      delete R;
      return fail(DF_EINVAL, "a level holds 2^31 entries or more per field");
    }
    size_t face_max = (size_t)G.n[0] * G.n[1];
    if ((size_t)G.n[0] * G.n[2] > face_max) face_max = (size_t)G.n[0] * G.n[2];
    if ((size_t)G.n[1] * G.n[2] > face_max) face_max = (size_t)G.n[1] * G.n[2];
    // frontier accumulators of a fine level: [dir][side][quantity][face]
    R->acc_n[l] = (l > 0) ? (size_t)3 * 2 * NQ * face_max : 0;
    R->npart[l] = dfk::part_count(G);
  }
  // CommUp from a finer level l into l + 1 reads the coarse hosts of the
  // stored fine entries and one neighbour on each side (two above, for the
  // faces): the cells of l it reaches beyond its active range, plus one
  for (int l = 1; l + 1 < R->nl; ++l) {
    const Geo &Gc = R->geo[l], &Gf = R->geo[l + 1];
    for (int k = 0; k < 3; ++k) {
      const int hmin = Gc.co[k] + (Gf.anch[k] ? 0 : fdiv2_i(-Gf.g));
      const int hmax = Gc.co[k] + fdiv2_i(Gf.s[k] - Gf.g - 1);
      const int lo = 1 - hmin, hi = hmax + 2 - (Gc.n[k] - 1);
      R->mobs[l][k] = std::max(0, std::max(lo, hi)) + 1;
    }
  }
  carve(R, nullptr);
  *out = R;
  return DF_OK;
}

int df_required_bytes(const df_run *R, size_t *bytes) {
  if (!R || !bytes) return fail(DF_EINVAL, "null argument");
  *bytes = R->need;
  return DF_OK;
}

int df_bind(df_run *R, void *dev_ptr, size_t bytes, void *stream) {
  if (!R || !dev_ptr) return fail(DF_EINVAL, "null argument");
  if (((uintptr_t)dev_ptr) % ALIGN) return fail(DF_EINVAL, "arena must be 256-byte aligned");
  if (bytes < R->need) return fail(DF_ENOMEM, "arena smaller than df_required_bytes()");
  R->base = (char *)dev_ptr;
  R->bytes = bytes;
  R->stream = (hipStream_t)stream;
  carve(R, R->base);
  R->sig_valid = false;
  int rc = hip_check(hipMemsetAsync(R->base, 0, R->need, R->stream), "df_bind clear");
  if (rc) return rc;
  R->bound = true;
  R->ready = false;
  R->graphs_stale = true;
  return DF_OK;
}

int df_set_perturber(df_run *R, double GM, double eps, double L, double mach, double chi) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (!finite_nonneg(GM) || !finite_nonneg(eps) || !finite_nonneg(L) || !finite_nonneg(mach) ||
      !finite_nonneg(chi))
    return fail(DF_EINVAL, "GM, eps, L, mach and chi must be finite and >= 0");
  const df_mesh_desc &d = R->desc;
  Phys &P = R->phys;
  P.gamma = d.gamma;
  P.gm1 = d.gamma - 1.0;
  P.GM = GM;
  P.eps2 = eps * eps;
  P.L = L;
  P.rho0 = 1.0;
  double cs = 1.0;
  P.V = mach * cs;
  P.chi = chi;
  P.e0 = P.rho0 * cs * cs / (d.gamma * (d.gamma - 1.0));
  P.cfl = d.cfl;
  P.fp32 = d.precision == DF_FP32;
  P.visc = R->visc;
  R->eps = eps;
  hipStream_t st = R->stream;
  // heat tables
  for (int l = 0; l < R->nl; ++l) {
    std::vector<double> w;
    int edge[3] = {0, 0, 0};
    heat_table(R->geo[l], eps, R->mult, w, edge);
    for (int d = 0; d < 3; ++d) R->buf[l].hw_n[d] = edge[d];
    rc = hip_check(hipMemcpyAsync(R->buf[l].hw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, st),
                   "heat table upload");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(st), "heat table upload");
    if (rc) return rc;
  }
  // initial state: both transported sets and the diffusion buffer hold the
  // uniform background so that no entry of any array is ever uninitialised
  for (int l = 0; l < R->nl; ++l) {
    LevBufs &B = R->buf[l];
    R->cur[l] = 1;
    dfk::init_state(st, R->geo[l], P, B, 1, d.seed, 0.0);
    std::swap(B.etmp, B.q[1][1]);
    dfk::init_state(st, R->geo[l], P, B, 1, d.seed, 0.0);
    std::swap(B.etmp, B.q[1][1]);
    R->cur[l] = 0;
    dfk::init_state(st, R->geo[l], P, B, 0, d.seed, d.noise_amp);
    if (B.acc) dfk::zero(st, B.acc, R->acc_n[l] * R->esz);
    for (int k = 0; k < 3; ++k)
      if (B.vk[k]) dfk::zero(st, B.vk[k], R->vol[l] * R->esz);
  }
  Scal zero{};
  for (int q = 0; q < 3; ++q) zero.fmul[q] = (q > 0 && R->quad) ? 0.0 : R->mult;
  zero.tmul = R->mult;
  rc = hip_check(hipMemcpyAsync(R->scal, &zero, sizeof(Scal), hipMemcpyHostToDevice, st), "scalars");
  if (rc) return rc;
  sync_levels(R);
  post_reduce(R);
  rc = launch_check("df_set_perturber");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(st), "df_set_perturber");
  if (rc) return rc;
  R->ready = true;
  R->graphs_stale = true;
  return DF_OK;
}

int df_step(df_run *R, int32_t n) {
  int rc = check_run(R, true);
  if (rc) return rc;
  if (n < 0) return fail(DF_EINVAL, "negative step count");
  if (R->subcycle == 1 && R->nl > 1) {
    for (int s = 0; s < n; ++s) {
      rc = criterion_step(R);
      if (rc) return rc;
    }
    return DF_OK;
  }
  // nested runs replay graphs of two coarse steps (one per-step launch
  // sequence has a few hundred short kernels); timing runs stay eager
  if (R->nl > 1 && R->use_graphs && !R->timing && n >= 2) {
    rc = graph_steps(R, n / 2);
    if (rc) return rc;
    n %= 2;
  }
  enqueue_steps(R, n);
  return launch_check("df_step");
}

int df_set_step_graphs(df_run *R, int32_t on) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (on != 0 && on != 1) return fail(DF_EINVAL, "step graphs must be 0 or 1");
  R->use_graphs = on == 1;
  R->graphs_stale = true;
  return DF_OK;
}

int df_set_subcycling(df_run *R, int32_t mode) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (mode != 0 && mode != 1) return fail(DF_EINVAL, "sub-cycling mode must be 0 or 1");
  R->subcycle = mode;
  for (int m = 0; m < MAXLEV; ++m) R->xi[m] = 2;
  R->graphs_stale = true;
  return DF_OK;
}

int df_set_viscosity(df_run *R, double c2) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (!std::isfinite(c2) || c2 < 0.0) return fail(DF_EINVAL, "viscosity coefficient must be finite and >= 0");
  R->visc = c2;
  R->phys.visc = c2;
  R->graphs_stale = true;
  return DF_OK;
}

int df_set_transport_fusion(df_run *R, int32_t on) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (on != 0 && on != 1) return fail(DF_EINVAL, "transport fusion must be 0 or 1");
  R->fuse_xy = on == 1;
  R->graphs_stale = true;
  return DF_OK;
}

int df_set_kick_fusion(df_run *R, int32_t on) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (on != 0 && on != 1) return fail(DF_EINVAL, "kick fusion must be 0 or 1");
  R->fuse_kc = on == 1;
  R->graphs_stale = true;
  return DF_OK;
}

int df_set_finish_fusion(df_run *R, int32_t on) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (on != 0 && on != 1) return fail(DF_EINVAL, "finish fusion must be 0 or 1");
  R->fuse_zf = on == 1;
  R->graphs_stale = true;
  return DF_OK;
}

int df_set_boundaries(df_run *R, int32_t mode) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (mode != 0 && mode != 1) return fail(DF_EINVAL, "boundary mode must be 0 or 1");
  if (R->quad && mode != 1) return fail(DF_EINVAL, "the quadrant takes the boundary list of Sect. 3.4 (mode 1)");
  R->geo[0].bc = mode == 1 ? 2 : 1;
  R->sig_valid = false;
  R->graphs_stale = true;
  return DF_OK;
}

int df_get_schedule(df_run *R, int32_t *xi, int32_t n) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (!xi || n < R->nl - 1) return fail(DF_EINVAL, "schedule output needs nlevels-1 entries");
  for (int m = 0; m + 1 < R->nl; ++m) xi[m] = R->xi[m];
  return DF_OK;
}

static int reduce3(df_run *R, int slot, double out[4]) {
  force_reduce(R, slot);
  int rc = launch_check("reduction");
  if (rc) return rc;
  Scal h;
  rc = hip_check(hipMemcpyAsync(&h, R->scal, sizeof(Scal), hipMemcpyDeviceToHost, R->stream), "reduction copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(R->stream), "reduction sync");
  if (rc) return rc;
  const double *src = slot == 0 ? h.force : h.totals;
  for (int q = 0; q < 3; ++q) out[q] = src[q];
  if (slot == 0) out[3] = h.t;
  if (h.health) return fail(DF_ENUMERIC, "non-positive or non-finite density or energy");
  return DF_OK;
}

int df_force(df_run *R, double out[4]) {
  int rc = check_run(R, true);
  if (rc) return rc;
  if (!out) return fail(DF_EINVAL, "null output");
  return reduce3(R, 0, out);
}

int df_totals(df_run *R, double out[3]) {
  int rc = check_run(R, true);
  if (rc) return rc;
  if (!out) return fail(DF_EINVAL, "null output");
  double tmp[4];
  rc = reduce3(R, 1, tmp);
  for (int q = 0; q < 3; ++q) out[q] = tmp[q];
  return rc;
}

// background of a field (values are stored as departures from it)
static double field_back(const df_run *R, int f) {
  if (f == DF_RHO) return R->phys.rho0;
  if (f == DF_E) return R->phys.e0;
  if (f == DF_VX) return -R->phys.V;
  return 0.0;
}

static int field_io(df_run *R, int l, int f, double *hout, const double *hin) {
  int rc = check_run(R, true);
  if (rc) return rc;
  if (l < 0 || l >= R->nl || f < DF_RHO || f > DF_VZ) return fail(DF_EINVAL, "bad level or field");
  const Geo &G = R->geo[l];
  const size_t nv = R->vol[l];
  std::vector<char> raw(nv * R->esz);
  void *dev = field_ptr(R, l, f);
  rc = hip_check(hipMemcpyAsync(raw.data(), dev, raw.size(), hipMemcpyDeviceToHost, R->stream), "field copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(R->stream), "field copy");
  if (rc) return rc;
  const bool f32 = R->esz == 4;
  float *rf = reinterpret_cast<float *>(raw.data());
  double *rd = reinterpret_cast<double *>(raw.data());
  const double back = field_back(R, f);
  int e[3] = {G.n[0], G.n[1], G.n[2]};
  if (f >= DF_VX) e[f - DF_VX] += 1;
  size_t a = 0;
  for (int k = 0; k < e[2]; ++k)
    for (int j = 0; j < e[1]; ++j)
      for (int i = 0; i < e[0]; ++i) {
        const size_t c = (size_t)(G.off + i + (long)j * G.sy + (long)k * G.sz);
        if (hout) {
          hout[a++] = back + (f32 ? (double)rf[c] : rd[c]);
        } else {
          const double dv = hin[a++] - back;
          if (f32) rf[c] = (float)dv;
          else rd[c] = dv;
        }
      }
  if (hin) {
    R->sig_valid = false;
    rc = hip_check(hipMemcpyAsync(dev, raw.data(), raw.size(), hipMemcpyHostToDevice, R->stream), "field copy");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(R->stream), "field copy");
  }
  return rc;
}

int df_get_field(df_run *R, int32_t level, int32_t field, double *host) {
  if (!host) return fail(DF_EINVAL, "null output");
  return field_io(R, level, field, host, nullptr);
}

int df_set_field(df_run *R, int32_t level, int32_t field, const double *host) {
  if (!host) return fail(DF_EINVAL, "null input");
  return field_io(R, level, field, nullptr, host);
}

int df_sync_levels(df_run *R) {
  int rc = check_run(R, true);
  if (rc) return rc;
  sync_levels(R);
  R->sig_valid = false;
  rc = launch_check("df_sync_levels");
  if (rc) return rc;
  return hip_check(hipStreamSynchronize(R->stream), "df_sync_levels");
}

int df_get_dt(df_run *R, double *dt) {
  int rc = check_run(R, true);
  if (rc) return rc;
  if (!dt) return fail(DF_EINVAL, "null output");
  compute_dt(R, 0);
  rc = launch_check("df_get_dt");
  if (rc) return rc;
  Scal h;
  rc = hip_check(hipMemcpyAsync(&h, R->scal, sizeof(Scal), hipMemcpyDeviceToHost, R->stream), "dt copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(R->stream), "dt copy");
  *dt = h.dt[0];
  if (R->subcycle == 1 && R->nl > 1) {
    int xi[MAXLEV];
    *dt = schedule_criterion(R, h.dtl, xi);
  }
  return rc;
}

int df_debug_stage(df_run *R, int32_t stage, double dt) {
  int rc = check_run(R, true);
  if (rc) return rc;
  if (R->nl != 1) return fail(DF_EINVAL, "stage harness needs a single-level run");
  if (!std::isfinite(dt)) return fail(DF_EINVAL, "dt must be finite");
  hipStream_t st = R->stream;
  rc = hip_check(hipMemcpyAsync(&R->scal->dbg_dt, &dt, sizeof(double), hipMemcpyHostToDevice, st), "dt upload");
  if (rc) return rc;
  const double *dtp = &R->scal->dbg_dt;
  R->sig_valid = false;
  const Geo &G = R->geo[0];
  LevBufs &B = R->buf[0];
  const Phys &P = R->phys;
  int c = R->cur[0];
  switch (stage) {
    case 1: dfk::kick(st, G, P, B, c, dtp, 1.0); break;
    case 2: dfk::compress(st, G, P, B, c, dtp, 1.0); break;
    case 3: dfk::diffuse_heat(st, G, P, B, c, dtp, 1.0, true, false); std::swap(B.etmp, B.q[c][1]); break;
    case 4: dfk::diffuse_heat(st, G, P, B, c, dtp, 1.0, false, true); std::swap(B.etmp, B.q[c][1]); break;
    case 5:
      dfk::transport_pass(st, 0, G, P, B, c, dtp, 1.0, nullptr, nullptr, R->chunk);
      dfk::transport_pass(st, 1, G, P, B, 1 - c, dtp, 1.0, nullptr, nullptr, R->chunk);
      dfk::transport_pass(st, 2, G, P, B, c, dtp, 1.0, nullptr, nullptr, R->chunk);
      dfk::rebuild_kick(st, G, P, B, 1 - c, dtp, 0.0, false);
      R->cur[0] = 1 - c;
      break;
    case 6:
      dfk::compress(st, G, P, B, c, dtp, 1.0);
      dfk::diffuse_heat(st, G, P, B, c, dtp, 1.0, true, true);
      std::swap(B.etmp, B.q[c][1]);
      break;
    case 7: level_step(R, 0, dtp, 1.0, 0); break;
    case 8: dfk::viscosity(st, G, P, B, c, dtp, 1.0); break;
    default: return fail(DF_EINVAL, "unknown stage");
  }
  rc = launch_check("df_debug_stage");
  if (rc) return rc;
  return hip_check(hipStreamSynchronize(st), "df_debug_stage");
}

int df_force_log(df_run *R, double *out, int32_t cap, int32_t *count) {
  int rc = check_run(R, true);
  if (rc) return rc;
  if (!out || !count || cap < 0) return fail(DF_EINVAL, "bad output");
  Scal h;
  rc = hip_check(hipMemcpyAsync(&h, R->scal, sizeof(Scal), hipMemcpyDeviceToHost, R->stream), "log copy");
  if (rc) return rc;
  std::vector<double> ring(4 * (size_t)dfk::FLOG);
  rc = hip_check(hipMemcpyAsync(ring.data(), R->flog, ring.size() * sizeof(double), hipMemcpyDeviceToHost, R->stream),
                 "log copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(R->stream), "log copy");
  if (rc) return rc;
  unsigned int n = h.nlog;
  unsigned int avail = n < (unsigned)dfk::FLOG ? n : (unsigned)dfk::FLOG;
  unsigned int take = avail < (unsigned)cap ? avail : (unsigned)cap;
  for (unsigned int e = 0; e < take; ++e) {
    unsigned int idx = (n - take + e) % dfk::FLOG;
    for (int q = 0; q < 4; ++q) out[4 * e + q] = ring[4 * (size_t)idx + q];
  }
  *count = (int32_t)take;
  return DF_OK;
}

int df_timing_enable(df_run *R, int32_t max_launches) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (max_launches < 0 || max_launches > (1 << 20)) return fail(DF_EINVAL, "max_launches out of range");
  rc = hip_check(hipStreamSynchronize(R->stream), "timing");
  if (rc) return rc;
  for (hipEvent_t e : R->ev) (void)hipEventDestroy(e);  // idle after the synchronisation
  R->ev.clear();
  R->ev_kind.clear();
  R->ev_used = 0;
  R->timing = max_launches > 0;
  if (!R->timing) return DF_OK;
  R->ev.resize(2 * (size_t)max_launches);
  R->ev_kind.resize((size_t)max_launches);
  for (auto &e : R->ev) {
    rc = hip_check(hipEventCreate(&e), "event create");
    if (rc) return rc;
  }
  return DF_OK;
}

int df_timing_read(df_run *R, double *ms, int32_t *count, int32_t nkinds) {
  int rc = check_run(R, false);
  if (rc) return rc;
  if (!ms || !count || nkinds < 1) return fail(DF_EINVAL, "bad output");
  for (int k = 0; k < nkinds; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  rc = hip_check(hipStreamSynchronize(R->stream), "timing");
  if (rc) return rc;
  for (size_t p = 0; p + 1 < R->ev_used; p += 2) {
    float t = 0.0f;
    rc = hip_check(hipEventElapsedTime(&t, R->ev[p], R->ev[p + 1]), "event time");
    if (rc) return rc;
    int kind = R->ev_kind[p / 2];
    if (kind < nkinds) {
      ms[kind] += t;
      count[kind] += 1;
    }
  }
  R->ev_used = 0;
  return DF_OK;
}

int df_stream_copy(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src) return fail(DF_EINVAL, "null pointer");
  if (((uintptr_t)dst | (uintptr_t)src | bytes) % 16) return fail(DF_EINVAL, "copy needs 16-byte alignment");
  const char *d = (const char *)dst, *s = (const char *)src;
  if (d < s + bytes && s < d + bytes) return fail(DF_EINVAL, "overlapping copy ranges");
  if (bytes / 16 / 1024 >= (1u << 31)) return fail(DF_EINVAL, "copy larger than 32 TiB");
  dfk::stream_copy((hipStream_t)stream, dst, src, bytes / 16);
  return launch_check("df_stream_copy");
}

int df_destroy(df_run *R) {
  if (!R) return fail(DF_EINVAL, "null run handle");
  if (R->gexec[0] || R->gexec[1]) (void)drop_graphs(R);
  if (R->gstream) (void)hipStreamDestroy(R->gstream);
  for (hipEvent_t e : R->ev) (void)hipEventDestroy(e);  // released once any pending record completes
  delete R;
  return DF_OK;
}

}  // extern "C"

// ====================================================================== engine
//
// Continuous batching of independent runs on one GPU.  The engine owns nothing
// but host metadata: the caller passes one device arena (its HBM budget) and a
// stream.  Each admitted job is a run carved from a free range of the arena
// (first fit, 256-byte aligned) and initialised on the engine's admission
// stream.  One engine step advances every active job by two coarse steps: the
// launches of all jobs are captured once into a HIP graph, spread over the
// worker streams (forked from and joined back to the caller's stream inside
// the capture, so the kernels of different jobs overlap on the device), and
// the graph is replayed on the caller's stream.  Two steps bring every buffer
// of every job back to its role, so the same graph replays until the set of
// jobs changes (an admission, a completion or a release), when it is captured
// again.  A job's arithmetic does not depend on the other jobs, on its stream
// or on the graph, so its results are bitwise those of the same job run alone.

namespace {

constexpr int ENGINE_MAX_SLOTS = 1024;
constexpr int ENGINE_STEPS_PER_REPLAY = 2;

struct EngineJob {
  bool used = false;
  df_run *run = nullptr;
  size_t off = 0, len = 0;
  int32_t remaining = 0;  // coarse steps still to run
  bool active = false;    // in the graph
  bool done = false;      // all steps enqueued
  bool reported = false;  // returned by poll
  int worker = 0;
};

struct Pending {
  hipEvent_t ev;
  std::vector<int> slots;
};

}  // namespace

struct df_engine {
  char *base = nullptr;
  size_t bytes = 0;
  hipStream_t main = nullptr, admin = nullptr;
  hipStream_t cap = nullptr;  // capture origin (the caller's stream may be the null stream)
  std::vector<hipStream_t> workers;
  std::vector<EngineJob> jobs;
  std::vector<std::pair<size_t, size_t>> freel;  // (offset, length), sorted, coalesced
  hipGraphExec_t exec = nullptr;
  int exec_tab = -1;  // the job table of the current graph's batched launches
  // replaced graphs whose launches may still run on the device: each is
  // destroyed (and its job table freed for reuse) once the event recorded
  // after its last launch has completed
  struct Retired {
    hipGraphExec_t exec;
    hipEvent_t ev;
    int tab;
  };
  std::vector<Retired> retired;
  // device job tables of the batched launches (allocated outside the arena,
  // reused once their graph is retired)
  struct Tab {
    void *dev = nullptr;
    size_t cap = 0;
    bool busy = false;
  };
  std::vector<Tab> tabs;
  long batched = 0;  // jobs in the batched launches of the current graph
  bool dirty = true;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  std::vector<Pending> pending;
  std::vector<int> finished;  // completed and not yet polled
  std::vector<hipEvent_t> ev_pool;
  long replays = 0, captures = 0;
};

namespace {

bool arena_take(df_engine *E, size_t need, size_t &off) {
  need = align_up(need);
  for (size_t i = 0; i < E->freel.size(); ++i) {
    auto &fr = E->freel[i];
    if (fr.second >= need) {
      off = fr.first;
      fr.first += need;
      fr.second -= need;
      if (fr.second == 0) E->freel.erase(E->freel.begin() + (long)i);
      return true;
    }
  }
  return false;
}

void arena_give(df_engine *E, size_t off, size_t len) {
  len = align_up(len);
  auto &F = E->freel;
  size_t i = 0;
  while (i < F.size() && F[i].first < off) ++i;
  F.insert(F.begin() + (long)i, {off, len});
  // coalesce neighbours
  if (i + 1 < F.size() && F[i].first + F[i].second == F[i + 1].first) {
    F[i].second += F[i + 1].second;
    F.erase(F.begin() + (long)i + 1);
  }
  if (i > 0 && F[i - 1].first + F[i - 1].second == F[i].first) {
    F[i - 1].second += F[i].second;
    F.erase(F.begin() + (long)i);
  }
}

hipEvent_t engine_event(df_engine *E) {
  if (!E->ev_pool.empty()) {
    hipEvent_t e = E->ev_pool.back();
    E->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event create")) return nullptr;
  return e;
}

// destroy the retired graphs that the device has finished with (all of them
// when wait is set)
void engine_reap(df_engine *E, bool wait) {
  size_t k = 0;
  for (auto &r : E->retired) {
    hipError_t q = wait ? hipEventSynchronize(r.ev) : hipEventQuery(r.ev);
    if (q != hipSuccess) {
      E->retired[k++] = r;
      continue;
    }
    (void)hipGraphExecDestroy(r.exec);  // its last launch has completed
    E->ev_pool.push_back(r.ev);
    if (r.tab >= 0) E->tabs[r.tab].busy = false;
  }
  E->retired.resize(k);
}

int engine_capture(df_engine *E) {
  if (E->exec) {
    // launches of the old graph may be in flight on the caller's stream
    hipEvent_t ev = engine_event(E);
    if (!ev) return DF_EDEVICE;
    int rc = hip_check(hipEventRecord(ev, E->main), "event record");
    if (rc) return rc;
    E->retired.push_back({E->exec, ev, E->exec_tab});
    E->exec = nullptr;
    E->exec_tab = -1;
  }
  engine_reap(E, false);
  std::vector<int> act;
  for (int s = 0; s < (int)E->jobs.size(); ++s)
    if (E->jobs[s].used && E->jobs[s].active) act.push_back(s);
  E->dirty = false;
  E->batched = 0;
  if (act.empty()) return DF_OK;
  // A dry run of every job's two steps with a recorder: the jobs whose every
  // launch is a batched stage, in the same sequence of stages, advance together,
  // one launch per stage; the others keep launches of their own.
  std::vector<dfk::Recorder> rec(act.size());
  std::vector<char> bat(act.size(), 0);
  std::vector<int> seq;  // stage sequence (kind classes) of the batched jobs
  auto cls = [](int kind) {
    return kind <= dfk::JK_KC_F2 ? 0 : kind <= dfk::JK_DF_F2 ? 1 : kind <= dfk::JK_XY_F2F ? 2 : kind <= dfk::JK_ZF_F ? 3 : 4;
  };
  // every job's buffer roles and signal state before the capture: a capture
  // that fails leaves the jobs where they were
  std::vector<std::vector<int>> cur_save(act.size());
  std::vector<char> sig_save(act.size());
  for (size_t q = 0; q < act.size(); ++q) {
    df_run *R = E->jobs[act[q]].run;
    cur_save[q].assign(R->cur, R->cur + R->nl);
    sig_save[q] = R->sig_valid;
  }
  auto restore = [&](int code) {
    for (size_t q = 0; q < act.size(); ++q) {
      df_run *R = E->jobs[act[q]].run;
      std::copy(cur_save[q].begin(), cur_save[q].end(), R->cur);
      R->sig_valid = sig_save[q];
    }
    E->batched = 0;
    E->dirty = true;
    return code;
  };
  for (size_t q = 0; q < act.size(); ++q) {
    df_run *R = E->jobs[act[q]].run;
    const bool timing = R->timing;
    R->timing = false;
    dfk::set_recorder(&rec[q]);
    enqueue_steps(R, ENGINE_STEPS_PER_REPLAY);
    dfk::set_recorder(nullptr);
    R->timing = timing;
    bool ok = !rec[q].failed && !rec[q].recs.empty();
    if (ok) {
      std::vector<int> c;
      for (const auto &r : rec[q].recs) c.push_back(cls(r.kind));
      if (seq.empty()) seq = c;
      ok = c == seq;
    }
    if (ok) {
      bat[q] = 1;
      E->batched++;
    } else {
      // launched by the job itself below
      std::copy(cur_save[q].begin(), cur_save[q].end(), R->cur);
      R->sig_valid = sig_save[q];
    }
  }
  // the job tables: per stage of the sequence and per kind, the entries of
  // the jobs (256-byte aligned) and their block offsets
  struct Group {
    int kind, n;
    size_t off_e, off_s;
    unsigned nblocks;
  };
  std::vector<Group> groups;
  std::vector<unsigned char> host;
  auto grow = [&](size_t bytes) {
    const size_t off = align_up(host.size());
    host.resize(off + bytes);
    return off;
  };
  for (size_t p = 0; p < seq.size() && E->batched; ++p) {
    for (int kind = 0; kind < dfk::JK_N; ++kind) {
      std::vector<size_t> qs;
      for (size_t q = 0; q < act.size(); ++q)
        if (bat[q] && rec[q].recs[p].kind == kind) qs.push_back(q);
      if (qs.empty()) continue;
      const size_t esz = dfk::job_entry_size(kind);
      Group g{kind, (int)qs.size(), grow(esz * qs.size()), 0, 0};
      std::vector<unsigned> start(qs.size() + 1, 0);
      for (size_t u = 0; u < qs.size(); ++u) {
        const dfk::JobRec &r = rec[qs[u]].recs[p];
        std::memcpy(host.data() + g.off_e + u * esz, r.bytes.data(), esz);
        // one block per job for the force log; else the job's blocks, padded
        // to a multiple of 8 (XCD placement)
        const unsigned nb = kind == dfk::JK_LOG ? 1u : (r.nblk + 7u) / 8u * 8u;
        start[u + 1] = start[u] + nb;
      }
      g.nblocks = start.back();
      g.off_s = grow(start.size() * sizeof(unsigned));
      std::memcpy(host.data() + g.off_s, start.data(), start.size() * sizeof(unsigned));
      groups.push_back(g);
    }
  }
  int tab = -1;
  int rc = DF_OK;
  if (!groups.empty()) {
    for (size_t u = 0; u < E->tabs.size() && tab < 0; ++u)
      if (!E->tabs[u].busy && E->tabs[u].cap >= host.size()) tab = (int)u;
    if (tab < 0) {
      df_engine::Tab t;
      t.cap = (host.size() + (1u << 20) - 1) / (1u << 20) * (1u << 20);
      rc = hip_check(hipMalloc(&t.dev, t.cap), "job table");
      if (rc) return restore(rc);
      E->tabs.push_back(t);
      tab = (int)E->tabs.size() - 1;
    }
    rc = hip_check(hipMemcpyAsync(E->tabs[tab].dev, host.data(), host.size(), hipMemcpyHostToDevice, E->admin),
                   "job table upload");
    if (!rc) rc = hip_check(hipStreamSynchronize(E->admin), "job table upload");
    if (rc) return restore(rc);
  }
  rc = hip_check(hipStreamBeginCapture(E->cap, hipStreamCaptureModeRelaxed), "graph capture");
  if (rc) return restore(rc);
  // a failed fork or join leaves the capture unusable: end it and report
  auto abandon = [&](int code) {
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(E->cap, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    return restore(code);
  };
  rc = hip_check(hipEventRecord(E->fork, E->cap), "graph fork");
  for (size_t w = 0; !rc && w < E->workers.size(); ++w)
    rc = hip_check(hipStreamWaitEvent(E->workers[w], E->fork, 0), "graph fork");
  if (rc) return abandon(rc);
  size_t nw = 0;
  for (size_t q = 0; q < act.size(); ++q) {
    if (bat[q]) continue;
    EngineJob &J = E->jobs[act[q]];
    J.worker = (int)(nw++ % E->workers.size());
    df_run *R = J.run;
    R->stream = E->workers[J.worker];
    const bool timing = R->timing;
    R->timing = false;
    enqueue_steps(R, ENGINE_STEPS_PER_REPLAY);
    R->timing = timing;
  }
  // the batched jobs, one launch per stage, on the capture stream
  for (const Group &g : groups) {
    const char *base = static_cast<const char *>(E->tabs[tab].dev);
    dfk::launch_jobs(E->cap, g.kind, base + g.off_e, reinterpret_cast<const unsigned *>(base + g.off_s), g.n,
                     g.nblocks);
  }
  for (size_t w = 0; !rc && w < E->workers.size(); ++w) {
    rc = hip_check(hipEventRecord(E->join[w], E->workers[w]), "graph join");
    if (!rc) rc = hip_check(hipStreamWaitEvent(E->cap, E->join[w], 0), "graph join");
  }
  if (rc) return abandon(rc);
  hipGraph_t g = nullptr;
  rc = hip_check(hipStreamEndCapture(E->cap, &g), "graph capture end");
  if (rc) return restore(rc);
  rc = hip_check(hipGraphInstantiate(&E->exec, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);  // the instantiated graph does not need it
  if (rc) {
    E->exec = nullptr;
    return restore(rc);
  }
  if (tab >= 0) E->tabs[tab].busy = true;
  E->exec_tab = tab;
  E->captures++;
  return rc;
}

int check_engine(const df_engine *E) { return E ? DF_OK : fail(DF_EINVAL, "null engine"); }

// finished jobs whose last replay has completed on the device
void engine_collect(df_engine *E, bool wait) {
  size_t k = 0;
  for (; k < E->pending.size(); ++k) {
    Pending &p = E->pending[k];
    hipError_t q = wait ? hipEventSynchronize(p.ev) : hipEventQuery(p.ev);
    if (q != hipSuccess) break;
    for (int s : p.slots) E->finished.push_back(s);
    E->ev_pool.push_back(p.ev);
  }
  E->pending.erase(E->pending.begin(), E->pending.begin() + (long)k);
  engine_reap(E, wait);
}

}  // namespace

extern "C" {

int df_engine_create(void *dev_arena, size_t bytes, void *stream, int32_t nstreams, df_engine **out) {
  if (!dev_arena || !out) return fail(DF_EINVAL, "null argument");
  if (((uintptr_t)dev_arena) % ALIGN) return fail(DF_EINVAL, "arena must be 256-byte aligned");
  if (nstreams < 1 || nstreams > 4) return fail(DF_EINVAL, "nstreams must be 1..4");
  df_engine *E = new df_engine();
  E->base = (char *)dev_arena;
  E->bytes = bytes / ALIGN * ALIGN;
  E->main = (hipStream_t)stream;
  E->jobs.resize(ENGINE_MAX_SLOTS);
  E->freel.push_back({0, E->bytes});
  int rc = hip_check(hipStreamCreate(&E->admin), "stream create");
  if (!rc) rc = hip_check(hipStreamCreate(&E->cap), "stream create");
  for (int w = 0; w < nstreams && !rc; ++w) {
    hipStream_t s = nullptr;
    rc = hip_check(hipStreamCreate(&s), "stream create");
    E->workers.push_back(s);
    hipEvent_t j = nullptr;
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&j, hipEventDisableTiming), "event create");
    E->join.push_back(j);
  }
  if (!rc) rc = hip_check(hipEventCreateWithFlags(&E->fork, hipEventDisableTiming), "event create");
  if (rc) {
    df_engine_destroy(E);
    return rc;
  }
  *out = E;
  return DF_OK;
}

int df_engine_job_bytes(const df_mesh_desc *desc, size_t *bytes) {
  if (!bytes) return fail(DF_EINVAL, "null output");
  df_run *R = nullptr;
  int rc = df_init_mesh(desc, &R);
  if (rc) return rc;
  *bytes = align_up(R->need);
  delete R;
  return DF_OK;
}

int df_engine_admit(df_engine *E, const df_mesh_desc *desc, const double perturber[5], int32_t nsteps,
                    int32_t *slot) {
  int rc = check_engine(E);
  if (rc) return rc;
  if (!desc || !perturber || !slot || nsteps < 1) return fail(DF_EINVAL, "bad admission arguments");
  int s = -1;
  for (int k = 0; k < (int)E->jobs.size(); ++k)
    if (!E->jobs[k].used) {
      s = k;
      break;
    }
  if (s < 0) return fail(DF_EBUSY, "no free job slot");
  df_run *R = nullptr;
  rc = df_init_mesh(desc, &R);
  if (rc) return rc;
  size_t off = 0;
  if (!arena_take(E, R->need, off)) {
    delete R;
    return fail(DF_EBUSY, "HBM budget exhausted");
  }
  rc = df_bind(R, E->base + off, align_up(R->need), E->admin);
  if (!rc)
    rc = df_set_perturber(R, perturber[0], perturber[1], perturber[2], perturber[3], perturber[4]);
  if (rc) {
    arena_give(E, off, R->need);
    delete R;
    return rc;
  }
  EngineJob &J = E->jobs[s];
  J = EngineJob();
  J.used = true;
  J.run = R;
  J.off = off;
  J.len = R->need;
  J.remaining = (nsteps + ENGINE_STEPS_PER_REPLAY - 1) / ENGINE_STEPS_PER_REPLAY * ENGINE_STEPS_PER_REPLAY;
  J.active = true;
  E->dirty = true;
  *slot = s;
  return DF_OK;
}

int df_engine_step(df_engine *E, int32_t n) {
  int rc = check_engine(E);
  if (rc) return rc;
  if (n < 0) return fail(DF_EINVAL, "negative step count");
  for (int r = 0; r < n; ++r) {
    if (E->dirty) {
      rc = engine_capture(E);
      if (rc) return rc;
    }
    if (!E->exec) return DF_OK;  // nothing active
    rc = hip_check(hipGraphLaunch(E->exec, E->main), "graph launch");
    if (rc) return rc;
    E->replays++;
    Pending p;
    for (int s = 0; s < (int)E->jobs.size(); ++s) {
      EngineJob &J = E->jobs[s];
      if (!J.used || !J.active) continue;
      J.remaining -= ENGINE_STEPS_PER_REPLAY;
      if (J.remaining <= 0) {
        J.active = false;
        J.done = true;
        p.slots.push_back(s);
        E->dirty = true;
      }
    }
    if (!p.slots.empty()) {
      p.ev = engine_event(E);
      if (!p.ev) return DF_EDEVICE;
      const int rc = hip_check(hipEventRecord(p.ev, E->main), "event record");
      if (rc) return rc;
      E->pending.push_back(p);
    }
  }
  return DF_OK;
}

int df_engine_poll(df_engine *E, int32_t *done, int32_t cap, int32_t *ndone) {
  int rc = check_engine(E);
  if (rc) return rc;
  if (!ndone || (cap > 0 && !done)) return fail(DF_EINVAL, "bad output");
  engine_collect(E, false);
  int32_t k = 0;
  size_t used = 0;
  for (; used < E->finished.size() && k < cap; ++used) {
    int s = E->finished[used];
    E->jobs[s].reported = true;
    done[k++] = s;
  }
  E->finished.erase(E->finished.begin(), E->finished.begin() + (long)used);
  *ndone = k;
  return DF_OK;
}

int df_engine_active(df_engine *E, int32_t *nactive, size_t *free_bytes) {
  int rc = check_engine(E);
  if (rc) return rc;
  int32_t a = 0;
  for (auto &J : E->jobs) a += (J.used && J.active) ? 1 : 0;
  size_t fb = 0;
  for (auto &fr : E->freel) fb = fr.second > fb ? fr.second : fb;
  if (nactive) *nactive = a;
  if (free_bytes) *free_bytes = fb;
  return DF_OK;
}

static int engine_job(df_engine *E, int32_t slot, EngineJob **J) {
  int rc = check_engine(E);
  if (rc) return rc;
  if (slot < 0 || slot >= (int)E->jobs.size() || !E->jobs[slot].used) return fail(DF_EINVAL, "bad slot");
  *J = &E->jobs[slot];
  return DF_OK;
}

// results of a job: a job returned by poll has completed on the device; any
// other job waits for the engine's work enqueued so far.  Reads then go to the
// admission stream.
static int engine_quiesce(df_engine *E, EngineJob *J) {
  if (!(J->done && J->reported)) {
    int rc = hip_check(hipStreamSynchronize(E->main), "engine sync");
    if (rc) return rc;
    engine_collect(E, true);
  }
  J->run->stream = E->admin;
  if (J->active) E->dirty = true;  // its stream changed: capture again
  return DF_OK;
}

int df_engine_force(df_engine *E, int32_t slot, double out[4]) {
  EngineJob *J = nullptr;
  int rc = engine_job(E, slot, &J);
  if (rc) return rc;
  rc = engine_quiesce(E, J);
  if (rc) return rc;
  return df_force(J->run, out);
}

int df_engine_get_field(df_engine *E, int32_t slot, int32_t level, int32_t field, double *host) {
  EngineJob *J = nullptr;
  int rc = engine_job(E, slot, &J);
  if (rc) return rc;
  rc = engine_quiesce(E, J);
  if (rc) return rc;
  return df_get_field(J->run, level, field, host);
}

int df_engine_release(df_engine *E, int32_t slot) {
  EngineJob *J = nullptr;
  int rc = engine_job(E, slot, &J);
  if (rc) return rc;
  rc = engine_quiesce(E, J);
  if (rc) return rc;
  // a job released before a poll reported it must not be reported later: by
  // then its slot may hold a newly admitted job
  for (auto &p : E->pending) p.slots.erase(std::remove(p.slots.begin(), p.slots.end(), slot), p.slots.end());
  E->finished.erase(std::remove(E->finished.begin(), E->finished.end(), slot), E->finished.end());
  if (J->active) E->dirty = true;  // the graph holds its launches
  arena_give(E, J->off, J->len);
  delete J->run;
  *J = EngineJob();
  return DF_OK;
}

int df_engine_stats(df_engine *E, int64_t out[3]) {
  int rc = check_engine(E);
  if (rc) return rc;
  if (!out) return fail(DF_EINVAL, "null output");
  out[0] = E->replays;
  out[1] = E->captures;
  out[2] = E->batched;
  return DF_OK;
}

int df_engine_destroy(df_engine *E) {
  if (!E) return fail(DF_EINVAL, "null engine");
  // a failed synchronisation is reported; the teardown below goes on (its
  // destroy calls have nothing further to report)
  const int rc = E->main ? hip_check(hipStreamSynchronize(E->main), "engine destroy") : DF_OK;
  engine_reap(E, true);
  if (E->exec) (void)hipGraphExecDestroy(E->exec);
  for (auto &t : E->tabs)
    if (t.dev) (void)hipFree(t.dev);
  for (auto &J : E->jobs)
    if (J.used) delete J.run;
  for (auto &p : E->pending) (void)hipEventDestroy(p.ev);
  for (hipEvent_t e : E->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : E->join)
    if (e) (void)hipEventDestroy(e);
  if (E->fork) (void)hipEventDestroy(E->fork);
  for (hipStream_t w : E->workers)
    if (w) (void)hipStreamDestroy(w);
  if (E->admin) (void)hipStreamDestroy(E->admin);
  if (E->cap) (void)hipStreamDestroy(E->cap);
  delete E;
  return rc;
}

}  // extern "C"
