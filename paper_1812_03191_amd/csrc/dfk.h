// dfk.h -- internal interface between the C-ABI runtime (api.hip) and the
// gfx950 kernels (dfk.hip) of libdfmesh.  Not installed; not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace dfk {

constexpr int NQ = 8;       // transported set: rho, e, P-x, P+x, P-y, P+y, P-z, P+z
constexpr int NSTATE = 5;   // rho, e, vx, vy, vz
constexpr int MAXLEV = 12;
constexpr int NSLOT = 512;  // signal-speed slots of a single-level run

// Array geometry of one level.  Every field of a level is one 3-D array,
// x fastest; entry (i,j,k), i in [-g, s[0]-g), is at off + i + j*sy + k*sz.
// A face field stores at (i,j,k) the face on the low side of cell (i,j,k)
// along its own axis.  Rows are padded so that x = 0 of every row sits on a
// 128-byte boundary.  Level 0 stores no ghosts (g = 0, s = n + 1: its
// boundary conditions are applied on read); finer levels store a ghost shell
// of width g (s = n + 2g).
struct Geo {
  int n[3];
  int g;
  int s[3];      // stored extent along each dimension
  long sy, sz;
  long off;
  double dx;
  int level;
  int bc;        // level 0 reads its outer boundary conditions: 1 inflow at x_max and outflow elsewhere,
                 // 2 the boundary list of Sect. 3.4 (background at both flow ends, mirror walls); 0 finer levels
  int has_fine;  // a finer level covers a central box of this level
  int co[3];     // that box: first covered cell and number of covered cells (the
  int cn[3];     // finer level's cell count / 2), centred on the perturber's vertex
  int mg[3];     // finer levels: a launch computes entries at most mg[d] cells beyond the active range
                 // along d (faces up to face n + mg[d]), set per stage by the scheduler; large: no limit
  int anch[3];   // quadrant: the dimension starts at the perturber's mirror plane
  double org[3]; // index of the perturber's vertex along each dimension (n/2, or 0 when anchored)
};

// Gas and perturber parameters (code units).  The fields are stored as
// departures from the uniform background (rho0, e0, wind (-V, 0, 0)).
struct Phys {
  double gamma, gm1;   // adiabatic index, gamma - 1
  double GM, eps2;     // perturber mass and squared Plummer length
  double L;            // luminosity
  double V;            // wind speed (gas enters through x_max at -V)
  double chi, rho0, e0;
  double cfl;
  int fp32;            // storage type: float (1) or double (0)
  double visc;         // artificial-viscosity coefficient C2 (0: off)
};

// Device-resident scalars of a run (one small array in the arena).
struct Scal {
  double dt[MAXLEV];         // step length of each level for the current coarse step
  double t;                  // time
  double dbg_dt;             // step length used by the stage harness
  double force[3];
  double totals[3];
  int health;                // bit 0: a non-positive or non-finite rho or e seen
  unsigned int nlog;         // force-log entries written so far
  double dtl[MAXLEV];        // per-level step limits cfl min(dx/smax, dx^2/6chi) of the last time step
  // single-level runs: the largest signal speed of the last end-of-step pass,
  // as the bits of a non-negative double, in NSLOT slots (block h takes slot
  // h mod NSLOT, so a slot is only met by blocks of one XCD, h mod 8)
  unsigned long long smax[NSLOT];
  double tlog;               // time of the state whose force partials await the log
  int pending;               // 1: the end-of-step force partials are not logged yet
  // the whole gas from the domain's sums: 1 for the full box; on the quadrant
  // 4 (the domain and its three mirror images) for Fx and the totals, 0 for
  // the force components normal to the mirror planes
  double fmul[3];
  double tmul;
};

constexpr int FLOG = 4096;   // force-log ring: (Fx, Fy, Fz, t) per coarse step

// Buffers of one level, in the run's storage type (double or float).
struct LevBufs {
  void *q[2][NQ];     // ping-pong transported sets; q[cur][0], q[cur][1] are rho, e
  void *v[3];         // face velocities
  void *vk[3];        // level 0: face velocities after the first kick of a fused kick and compression
  void *etmp;         // diffusion output (the compressed energy after a fused kick and compression)
  void *acc;          // frontier transfers of this (fine) level: [dir][side][q][t2][t1]
  double *hw;         // heat weights on a box of hw_n[0] x hw_n[1] x hw_n[2] cells
                      // centred on the perturber vertex (x fastest)
  int hw_n[3];        // box extent (0: no heat table)
  double *part;       // reduction partials: three planes of one value per block, then the signal speeds
};

// ---- launchers (all asynchronous on `st`) ---------------------------------
void init_state(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, uint64_t seed,
                double amp);
// with slots (single-level runs on level 0): the step length from the signal
// speeds the last end-of-step pass left in slots->smax, written to slots->dt[0]
// and added to slots->t by the kick itself
void kick(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
          double fac, Scal *slots = nullptr);
// face velocities from the transported momenta of q[src], then an optional
// kick; with post (level 0 with a kick) the same launch also forms the force
// and signal-speed partials of post_partials for the new state
void rebuild_kick(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src,
                  const double *dtp, double fac, bool do_kick, Scal *post = nullptr);
// with log (single-level runs on level 0): the first block also clears
// log->smax for this step's end-of-step pass and logs a pending force (the
// partials in B.part, at log->tlog) into flog
void compress(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
              double fac, Scal *log = nullptr, double *flog = nullptr);
// artificial viscosity over fac dt: e in place; the face velocities through
// the three momentum arrays of q[1-cur] as scratch (they are free before the
// x pass writes them)
void viscosity(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
               double fac);
// writes etmp; the caller swaps etmp and q[cur][1]; with clear (level 0) the
// first block also clears clear->smax (after a fused kick and compression)
void diffuse_heat(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur,
                  const double *dtp, double fac, bool do_diff, bool do_heat, Scal *clear = nullptr);
// level 0 without artificial viscosity: the first kick (fac kfac, as kick) and
// the compression (fac cfac, as compress) in one launch.  Reads B.v and
// q[cur]; writes the kicked face velocities to B.vk and the compressed energy
// to B.etmp (q[cur][1] keeps the energy before the step).  With slots: the
// step length from the slots and the pending force logged, as kick and
// compress with log do; the slots are left for diffuse_heat to clear.
void kick_compress(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
                   double kfac, double cfac, Scal *slots, double *flog);
// the same on a finer level: the kick (fac kfac, face ranges within Gk's
// margins) reads B.v and writes B.vk, the compression (fac cfac, cells within
// Gc's margins) writes B.etmp
void kick_compress_fine(hipStream_t st, const Geo &Gk, const Geo &Gc, const Phys &P, LevBufs &B, int cur,
                        const double *dtp, double kfac, double cfac);
// one transport pass q[src] -> q[1-src]; dir 0 builds the momenta from the
// face velocities; a fine level adds its frontier transfers into B.acc; a
// level with a finer one (Gf, fine_acc) takes that level's sums on the frontier
// chunk: cells per column segment of the streaming y and z passes
void transport_pass(hipStream_t st, int dir, const Geo &G, const Phys &P, LevBufs &B, int src,
                    const double *dtp, double fac, const Geo *Gf, const void *fine_acc, int chunk);
// fused x and y passes q[src] -> q[1-src] of level 0 (bc 1, at most 128
// cells along x, an even count above 64); under a finer level Gf, the
// transfers through its frontier faces are its sums from fine_acc; false,
// launching nothing, when the level does not qualify
bool transport_xy(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src, const double *dtp,
                  double fac, int chunk, const Geo *Gf, const void *fine_acc);
bool transport_xy_fits(const Geo &G);
// fused x and y passes q[src] -> q[1-src] of a finer level (no boundary
// conditions): G carries the y pass's margins; the entries written and the
// frontier transfers taken and accumulated are those of the separate x and y
// passes (x with G's x margin and y, z margins two cells wider)
void transport_xy_fine(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src, const double *dtp,
                       double fac, const Geo *Gf, const void *fine_acc, int chunk);
// the z pass q[src] -> q[1-src] (face velocities vin[2]) fused with the
// velocity rebuild, the kick (fac kfac) into B.v and the end-of-step partials
// of post_partials (as rebuild_kick with post S) on level 0 without a finer
// level (bc 1, at most 128 cells along x, an even row count); only the new
// density and energy of q[1-src] are written.  false, launching nothing, when
// the level does not qualify, S is null or vin[2] is B.v[2] (the walk reads
// the face velocities the finish writes)
bool transport_z_finish(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, void *const *vin, int src,
                        const double *dtp, double fac, double kfac, Scal *S, int chunk);
bool transport_z_finish_fits(const Geo &G);
void zero(hipStream_t st, void *p, size_t bytes);
void commup(hipStream_t st, const Geo &Gc, const Phys &P, LevBufs &Bc, int curc, const Geo &Gf,
            LevBufs &Bf, int curf);
void commmean(hipStream_t st, const Geo &Gf, const Phys &P, LevBufs &Bf, int curf, const Geo &Gc,
              LevBufs &Bc, int curc);
// quadrant, finer levels: the entries beyond the mirror planes as the images
// of the level's own (rho, e of q[cur] and the face velocities; or the
// transported set q[set], the momenta normal to a plane swapped and reversed);
// nothing on level 0 or off the quadrant
void mirror_state(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur);
void mirror_q(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int set);
// per-block maxima of the signal speed of one level into the signal region of
// B.part; health flag
void signal_speed(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, Scal *S);
// dt of every level from the per-block maxima; t += dt0 if advance
void dt_final(hipStream_t st, const Geo *G, const LevBufs *B, int nl, const Phys &P, Scal *S,
              int advance);
// force (3 FP64 sums) of one level into B.part, then the fixed-order final sum
int force_partials(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur);
// force partials (as force_partials) and the signal-speed partials of the
// next time step (as signal_speed) of the current state, in one pass
void post_partials(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, Scal *S);
// one block: with do_force the force of the partials of post_partials over
// all levels, appended to the log; then with do_dt = 1 the time step from
// their signal speeds (two sub-steps per level), advancing the time, with
// do_dt = 2 only each level's own step limit into S->dtl
void step_final(hipStream_t st, const Geo *G, LevBufs *B, int nl, const Phys &P, Scal *S, double *flog,
                int do_force, int do_dt);
// slot 0: S->force; slot 1: S->totals; slot 2: S->force and the force log
void force_final(hipStream_t st, double *const *parts, const int *nparts, int nl, Scal *S,
                 int slot, double *flog);
int totals_partials(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur);
size_t part_count(const Geo &G);
// plain copy of n 16-byte words (measurement reference)
void stream_copy(hipStream_t st, void *dst, const void *src, size_t n16);
// logs a pending force of a single-level run (as compress with log does)
void log_pending(hipStream_t st, const Geo &G, LevBufs &B, Scal *S, double *flog);

// Batched stages (the engine): while a recorder is set on the calling thread,
// the launchers of the single-level fused step (the fused kick and
// compression, the diffusion with heat release, the fused x + y pass, the
// fused z pass and step end, the force log) record their launch arguments
// instead of launching; any other launch marks the recording failed and is
// not made.  launch_jobs then makes one launch for one stage of several runs
// from a device table of their records.
enum JobKind {
  JK_KC_D1, JK_KC_D2, JK_KC_F1, JK_KC_F2,      // kick + compression: FP64/FP32, boundary mode 1/2
  JK_DF_D1, JK_DF_D2, JK_DF_F1, JK_DF_F2,      // diffusion + heat release
  JK_XY_D1P, JK_XY_D1F, JK_XY_D2P, JK_XY_D2F,  // fused x + y: cells per lane 1/2, rows partial/full
  JK_XY_F1P, JK_XY_F1F, JK_XY_F2P, JK_XY_F2F,
  JK_ZF_D, JK_ZF_F,                            // fused z pass and step end
  JK_LOG,                                      // force log after the last step
  JK_N
};
struct JobRec {
  int kind;
  unsigned nblk;                     // blocks of the run's own launch
  std::vector<unsigned char> bytes;  // the launch's table entry (job_entry_size(kind) bytes)
};
struct Recorder {
  std::vector<JobRec> recs;
  bool failed = false;
};
void set_recorder(Recorder *r);
size_t job_entry_size(int kind);
// one launch of stage `kind` for n runs: `entries` a device array of their
// records' bytes, `start` n + 1 device block offsets (multiples of 8),
// nblocks = start[n]
void launch_jobs(hipStream_t st, int kind, const void *entries, const unsigned *start, int n, unsigned nblocks);

}  // namespace dfk
