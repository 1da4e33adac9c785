/*
 * df.h -- C ABI of libdfmesh, an MI355X (gfx950) library that advances a
 * uniform gas streaming past a massive, optionally luminous point perturber on
 * nested, x2-refined Cartesian meshes and reduces the gravitational force the
 * gas exerts on the perturber.  The method is that of Velasco Romero & Masset
 * (2018), "Numerical study of dynamical friction with thermal effects -- I",
 * Sects. 2.1 and 3: the governing equations (eqs. 1-3), the split source /
 * transport step S(dt/2) T(dt) S(dt/2) (eq. 15), thermal diffusion (eqs.
 * 19-22), heat release at the perturber's vertex, nested meshes with CommUp /
 * CommMean / CommFlux and recursive sub-cycling (Sects. 3.1-3.3), and the force
 * monitor (eq. 18).
 *
 * Conventions (code units G = rho0 = c_s = 1 unless set otherwise):
 *  - the perturber sits at the origin, which is the central vertex of every
 *    level; level l+1 has half the cell size of level l and covers its central
 *    half in each dimension (or, with finer levels of half level 0's cells,
 *    level 1 covers the central quarter of level 0);
 *  - the gas enters through the x_max face with velocity (-mach c_s, 0, 0);
 *    every other outer face of level 0 is a zero-gradient outflow boundary;
 *  - fields: DF_RHO density, DF_E internal energy per unit volume, and the
 *    face-centred velocities DF_VX, DF_VY, DF_VZ (v_x on the faces normal to
 *    x, ...);
 *  - the force is reported as (Fx, Fy, Fz); Fx is the component along the
 *    perturber's motion through the gas (+x): drag < 0, thrust > 0.
 *
 * Memory and streams: the caller owns a device arena (for instance a uint8
 * tensor) and a HIP stream; the library carves every buffer out of the arena
 * and launches every kernel on that stream.  Both must outlive the run.  The
 * library owns the opaque handles and their host metadata.  Host buffers
 * passed in or out belong to the caller.  A handle is not thread-safe: use it
 * from one host thread at a time.
 *
 * Errors: every function returns DF_OK (0) or a negative DF_E* code;
 * df_strerror() names a code and df_last_error() returns the text of the last
 * error raised on the calling thread (with the HIP message for DF_EDEVICE).
 */
#ifndef DF_H
#define DF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DF_OK 0
#define DF_EINVAL (-1)   /* bad size, level, field or parameter               */
#define DF_ESTATE (-2)   /* call out of order (step before bind/perturber ...) */
#define DF_ENOMEM (-3)   /* arena smaller than df_required_bytes()            */
#define DF_EDEVICE (-4)  /* HIP runtime error                                 */
#define DF_ENUMERIC (-5) /* density or energy non-positive or not finite      */
#define DF_EBUSY (-6)    /* engine: no free slot or HBM budget exhausted      */

enum { DF_FP64 = 0, DF_FP32 = 1 };
enum { DF_RHO = 0, DF_E = 1, DF_VX = 2, DF_VY = 3, DF_VZ = 4 };

typedef struct df_run df_run;

/* Mesh description (Sect. 3.4).
 *  nx, ny, nz : active cells of level 0 (and of every level unless nx1 is
 *               set), each even (the perturber is a vertex), each a multiple
 *               of 4 and >= 16 when nlevels > 1;
 *  nlevels    : 1..12;
 *  dx0        : cell size of level 0 (> 0);
 *  gamma      : adiabatic index (> 1); cfl: Courant factor in (0, 1];
 *  precision  : DF_FP64 (FP64 storage and arithmetic) or DF_FP32 (FP32
 *               storage of the departure from the uniform background, FP32
 *               stencils, FP64 force and totals);
 *  ghost_fine : ghost width of levels >= 1 (0 selects 10, the least width that
 *               carries two sub-cycles without a refill, Sect. 3.2.1);
 *  seed, noise_amp : every active density is multiplied by 1 + noise_amp (2U-1),
 *               U uniform in [0,1) from a counter-based SplitMix64 stream;
 *  tile_chunk : cells per column segment of the streaming y and z transport
 *               passes (0 selects 16 for FP32 storage, and for FP64 32 on one
 *               level and 8 on nested meshes; 2..256),
 *               a launch-shape parameter that does not change results;
 *  nx1, ny1, nz1 : cells of every level >= 1 (0: those of level 0), each a
 *               multiple of 4, >= 16 and at most twice level 0's count.  Level
 *               l+1 covers the central n_{l+1}/2 cells of level l along each
 *               dimension: the central half when all levels have the same
 *               cells, the central quarter of level 0 when the finer levels
 *               have half its cells (the hierarchy of Sects. 4.1.3, 4.2.2);
 *  quadrant   : 1: the domain is the paper's quadrant (Sect. 3.4) -- with the
 *               flow along x here, y > 0 and z > 0, the perturber's vertex on
 *               the low y and z faces, which are its mirror planes; every
 *               level starts at the planes (nx, ny, nz count the quadrant's
 *               cells); level 0 takes the boundary list of Sect. 3.4 (its
 *               mode 1, the only one df_set_boundaries then accepts), the
 *               entries of the finer levels beyond the planes are their own
 *               mirror images; the force and totals are those of the whole
 *               gas (the domain and its three images: Fy = Fz = 0). */
typedef struct {
  int32_t nx, ny, nz;
  int32_t nlevels;
  double dx0;
  double gamma;
  double cfl;
  int32_t precision;
  int32_t ghost_fine;
  uint64_t seed;
  double noise_amp;
  int32_t tile_chunk;
  int32_t nx1, ny1, nz1;
  int32_t quadrant;
} df_mesh_desc;

/* Validate a mesh description and create a run handle (host memory only; no
 * HIP call).  *out receives the handle.  DF_EINVAL on a bad description. */
int df_init_mesh(const df_mesh_desc *desc, df_run **out);

/* Device bytes the run needs for its arena (256-byte aligned). */
int df_required_bytes(const df_run *run, size_t *bytes);

/* Attach a caller-owned device arena of `bytes` bytes at `dev_ptr` (device
 * pointer, 256-byte aligned) and the HIP stream `stream` (hipStream_t, may be
 * NULL for the null stream).  The arena is cleared.  DF_ENOMEM if too small. */
int df_bind(df_run *run, void *dev_ptr, size_t bytes, void *stream);

/* Set the perturber and the gas (Sect. 2, eq. 16): GM >= 0, Plummer softening
 * eps >= 0 (also the standard deviation of the Gaussian heat-release weights;
 * eps = 0 splits the heat equally over the 8 cells around the perturber),
 * luminosity L >= 0, mach = V / c_s >= 0, thermal diffusivity chi >= 0.
 * Resets t = 0 and writes the initial state (uniform wind plus density noise,
 * levels made consistent by restriction then prolongation).  Synchronises the
 * stream.  Requires df_bind(). */
int df_set_perturber(df_run *run, double GM, double eps, double L, double mach, double chi);

/* Advance n >= 0 coarse steps (Sect. 3.1, time step scheduling; Sect. 3.3,
 * the staging list of sub-cycles and communications): each step takes its
 * length from the Courant and diffusion limits of every level, then runs the
 * recursive sub-cycled update -- the finer level's two steps first, then the
 * level's own step S(dt/2) T(dt) S(dt/2) of eq. 15 with the thermal sources
 * in between, then CommUp and CommMean (Sect. 3.2) -- and logs the force of
 * eq. 18.  Enqueues kernels on the bound stream and returns without
 * synchronising; DF_ESTATE before df_bind and df_set_perturber, DF_EINVAL
 * for n < 0.  Errors raised by the device surface at the next synchronising
 * call. */
int df_step(df_run *run, int32_t n);

/* Force on the perturber (eq. 18, FP64): out[0..2] = Fx, Fy, Fz, out[3] = t.
 * Synchronises the stream; DF_ENUMERIC if the health check of the last steps
 * found a non-positive or non-finite density or energy. */
int df_force(df_run *run, double out[4]);

/* The force log: df_step appends (Fx, Fy, Fz, t) after every coarse step to a
 * device ring of 4096 entries (the force time series monitored in Sect. 3.4).
 * Copies the last min(steps, 4096, cap) entries, oldest first, to out (4
 * doubles each) and their number to *count.  Synchronises. */
int df_force_log(df_run *run, double *out, int32_t cap, int32_t *count);

/* Composite totals over uncovered active cells (FP64): out[0] mass,
 * out[1] internal energy, out[2] kinetic energy (face velocities averaged to
 * the cell centres) -- the conserved quantities whose transfers the levels
 * match at their frontiers (Sect. 3.2.3), each coarse cell covered by a
 * finer level left out.  Synchronises; DF_ENUMERIC as df_force. */
int df_totals(df_run *run, double out[3]);

/* Copy a field of one level to / from host memory (FP64 values, x fastest):
 * the density and internal energy of eqs. 1 and 3, centred in the cells, and
 * the velocity components of eq. 2, staggered on the cell faces normal to
 * them (the centred and staggered quantities of Sect. 3.2.1).  Centred
 * fields: nx*ny*nz entries.  Face fields: one more entry along their own axis
 * (DF_VX: (nx+1)*ny*nz, x fastest).  The host buffer belongs to the caller.
 * Synchronises; DF_EINVAL for a bad level or field or a null buffer.  After
 * df_set_field, call df_sync_levels() before stepping a nested run. */
int df_get_field(df_run *run, int32_t level, int32_t field, double *host);
int df_set_field(df_run *run, int32_t level, int32_t field, const double *host);

/* Restrict every level onto its parent (finest first), then refill the ghost
 * entries of every finer level from its parent (CommMean then CommUp). */
int df_sync_levels(df_run *run);

/* The coarse time step the next df_step would take (synchronises). */
int df_get_dt(df_run *run, double *dt);

/* Sub-cycling of the nested levels (App. A, eqs. 55-56).  mode 0 (default):
 * every level takes two steps per step of the next coarser one (xi = 2).
 * mode 1: at the start of each coarse step the per-level step limits
 * dt_l = cfl min(dx_l / max(c_s + |v|), dx_l^2 / (6 chi)) are read back and the
 * word xi in {1,2}^(nlevels-1) of largest coarse step min_l dt_l prod_{m<l}
 * xi_m per cost sum_l C_l prod_{m<l} xi_m is taken, C_l being the active cell
 * count of level l; words are tried from all-2 down (xi_m = 2 where bit m of
 * the word is set) and a later word must do strictly better.  In mode 1
 * df_step synchronises once per coarse step (the engine's jobs always use
 * mode 0).  DF_EINVAL for other modes. */
int df_set_subcycling(df_run *run, int32_t mode);

/* Artificial viscosity: the SubStep2 that the staging list of Sect. 3.3 names
 * without giving it, taken as the von Neumann-Richtmyer viscosity of ZEUS
 * (Stone & Norman 1992): per dimension d and cell, dv = v_d(high face) -
 * v_d(low face), q_d = c2 rho dv^2 in compression (dv < 0), else 0; the face
 * velocities lose dt (q_d(c) - q_d(c-1)) / (dx rho_face) and the energy
 * dt sum_d q_d dv / dx, applied after the first kick of each level step.  c2 = 0
 * (the default) switches it off; DF_EINVAL for negative or non-finite c2. */
int df_set_viscosity(df_run *run, double c2);

/* Launch shape of the transport step (the x, y, z passes of T in eq. 15,
 * Sect. 3.2.3 and 3.3): on (1, default) the x and y passes of level 0 run
 * as one launch when level 0 uses the default boundaries and has at most 128
 * cells along x (an even count above 64; under a finer level, with the flux
 * matching on its frontier inside the launch), and those of every finer level
 * (in the quadrant, of a finer level with no finer one): each row's x pass is
 * taken in registers and fed to the y pass, so the x pass's results never
 * reach device memory.  off (0): every pass is a launch of its own.  The
 * results agree to rounding either way (the same operations in the same order;
 * the compiler may pair a product and a sum into one fused multiply-add
 * differently); DF_EINVAL for other values. */
int df_set_transport_fusion(df_run *run, int32_t on);

/* Launch shape of the first two sub-steps of a level step (the velocity
 * source S(dt/2) of eq. 15 and the compressional heating of Sect. 3.3, as
 * SubStep1 and SubStep3): on (1, default) one launch on level 0, and on the
 * finer levels of an FP32 run, when the artificial viscosity is off, whose
 * threads kick their cells' faces and then compress their cells from the
 * kicked velocities of all six faces (the faces of neighbouring cells are
 * taken from the neighbouring threads or kicked again with the same
 * arithmetic, not stored);
 * the kicked velocities and the compressed energy go to buffers of their own,
 * so that every thread reads the state before the step.  off (0): two
 * launches.  The results agree to rounding either way; DF_EINVAL for other
 * values. */
int df_set_kick_fusion(df_run *run, int32_t on);

/* Launch shape of the end of a single-level step (the z pass of T, the
 * velocity rebuild after it and the second velocity source S(dt/2) of eq. 15,
 * with the force of eq. 18 and the next step's signal speeds): on (1,
 * default) one launch when the level has at most 128 cells along x, an even
 * count of rows and the default boundaries, and the first kick is fused with
 * the compression (df_set_kick_fusion, so that the z pass reads that kick's
 * own copy of the face velocities) -- the z pass's results go from
 * the waves that compute them to the waves that rebuild and kick the face
 * velocities through LDS, one plane at a time, so the eight transported
 * fields never reach device memory; off (0): the z pass and the rebuild and
 * kick are launches of their own.  The results agree to rounding either way;
 * DF_EINVAL for other values. */
int df_set_finish_fusion(df_run *run, int32_t on);

/* Launch form of df_step on nested runs (the recursion of Sects. 3.1 and 3.3:
 * a few hundred short launches per coarse step): on (1, default) the launches
 * of two coarse steps are captured once into a HIP graph on a private stream
 * and df_step replays it on the bound stream (n / 2 replays; an odd last step
 * and runs with kernel timing enabled are launched directly); a graph is kept
 * per pattern of the levels' current buffer sets and captured again after any
 * call that changes the launches (perturber, boundaries, viscosity, launch
 * switches, sub-cycling, bind).  off (0): every launch is made directly.  The
 * results are bitwise the same either way; DF_EINVAL for other values.
 * Single-level runs are always launched directly. */
int df_set_step_graphs(df_run *run, int32_t on);

/* Outer boundary conditions of level 0 (Sect. 3.4).  mode 0 (default): the
 * gas enters through x_max with the unperturbed state (rho0, -V, 0, 0, e0) and
 * every other boundary is zero-gradient outflow.  mode 1: the paper's list,
 * with the flow along x and the full box (of which the paper's quadrant is a
 * quarter by symmetry): ghosts beyond both flow ends hold rho0, -V (normal
 * velocity) and e0, with the tangential velocities mirror-symmetric; the
 * four transverse boundaries are walls across which every field is
 * mirror-symmetric except the normal velocity, which is antisymmetric (zero
 * on the wall).  Takes effect from the next call that advances or reduces;
 * DF_EINVAL for other modes. */
int df_set_boundaries(df_run *run, int32_t mode);

/* xi_l (sub-steps of level l+1 per step of level l) of the last coarse step
 * into xi[0 .. nlevels-2]; n is the capacity of xi (DF_EINVAL if below
 * nlevels-1). */
int df_get_schedule(df_run *run, int32_t *xi, int32_t n);

/* Run one stage of the level update on a single-level run, with step dt:
 *  1 velocity kick over dt, 2 compressional heating, 3 thermal diffusion,
 *  4 heat release, 5 transport, 6 stages 2-4, 7 a whole level step,
 *  8 artificial viscosity (df_set_viscosity).
 * Used by the parity tests.  DF_EINVAL for other stages or nested runs. */
int df_debug_stage(df_run *run, int32_t stage, double dt);

/* Kernel timing for measurement (off by default).  df_timing_enable(run, n)
 * creates 2n HIP events and from then on records an event pair on the bound
 * stream around each of the next n kernel launches of df_step (0 disables and
 * frees them).  df_timing_read(run, ms, count, nkinds) synchronises, adds the
 * elapsed times by kernel kind into ms[kind] and the launch numbers into
 * count[kind] (kinds DF_K_*), and restarts the recording.  DF_K_FORCE is the
 * pass after each step that forms both the force partials and the next step's
 * signal speeds, with the one-block kernel that logs the force and sets the
 * next time step; DF_K_DT is the time step before the first step of a df_step
 * call (with a signal pass if the state was changed by other calls);
 * DF_K_PASSXY the fused x and y transport passes (df_set_transport_fusion),
 * DF_K_KICKCOMP the fused first kick and compression (df_set_kick_fusion),
 * DF_K_ZFINISH the z pass fused with the rebuild and kick
 * (df_set_finish_fusion). */
enum {
  DF_K_KICK = 0, DF_K_COMPRESS, DF_K_DIFFUSE, DF_K_PASSX, DF_K_PASSY, DF_K_PASSZ, DF_K_REBUILD,
  DF_K_COMMUP, DF_K_COMMMEAN, DF_K_DT, DF_K_FORCE, DF_K_ZERO, DF_K_VISC, DF_K_PASSXY, DF_K_KICKCOMP,
  DF_K_ZFINISH, DF_K_NKINDS
};
int df_timing_enable(df_run *run, int32_t max_launches);
int df_timing_read(df_run *run, double *ms, int32_t *count, int32_t nkinds);

/* Release the handle (not the caller's arena or stream). */
int df_destroy(df_run *run);

/* ---------------------------------------------------------------- engine
 * Continuous batching of independent runs (for instance a Mach / luminosity
 * sweep) on one GPU.  The caller owns one device arena, which is the HBM
 * budget, and a stream.  Each admitted job is a run carved from a free range of
 * the arena.  df_engine_step advances every active job by 2 coarse steps per
 * call of its count: the launches of all active jobs are captured into one HIP
 * graph and replayed on the caller's stream; the graph is captured again when
 * the set of jobs changes.  Single-level jobs whose step takes the fused
 * launches (at most 128 cells along x, the default boundaries) advance
 * together: one launch per stage carries the blocks of all of them, each
 * block reading its job's launch arguments from a device table (allocated by
 * the engine outside the arena, a few hundred bytes per job and stage); the
 * other jobs' own launches are spread over nstreams worker streams so that
 * they overlap on the device.  A job's results are bitwise those of the same
 * job run alone.  Jobs run a multiple of 2 coarse steps (nsteps rounded up). */
typedef struct df_engine df_engine;

/* dev_arena: device pointer (256-byte aligned) of `bytes` bytes owned by the
 * caller; stream: hipStream_t of the caller; nstreams: 1..4 worker streams. */
int df_engine_create(void *dev_arena, size_t bytes, void *stream, int32_t nstreams, df_engine **out);

/* Arena bytes one job of this description takes. */
int df_engine_job_bytes(const df_mesh_desc *desc, size_t *bytes);

/* Admit a job: perturber = {GM, eps, L, mach, chi} (as df_set_perturber),
 * nsteps >= 1 coarse steps.  Initialises it (synchronously, on the engine's own
 * stream) and returns its slot.  DF_EBUSY if no arena range or slot is free. */
int df_engine_admit(df_engine *eng, const df_mesh_desc *desc, const double perturber[5], int32_t nsteps,
                    int32_t *slot);

/* n engine steps (2 coarse steps of every active job each); asynchronous. */
int df_engine_step(df_engine *eng, int32_t n);

/* Slots of jobs that ran all their steps and whose work has completed on the
 * device since the last poll (non-blocking): up to cap into done[], count into
 * *ndone. */
int df_engine_poll(df_engine *eng, int32_t *done, int32_t cap, int32_t *ndone);

/* Number of active jobs and the largest free arena range in bytes. */
int df_engine_active(df_engine *eng, int32_t *nactive, size_t *free_bytes);

/* Results of a job (synchronise the engine's work so far): force as df_force,
 * fields as df_get_field. */
int df_engine_force(df_engine *eng, int32_t slot, double out[4]);
int df_engine_get_field(df_engine *eng, int32_t slot, int32_t level, int32_t field, double *host);

/* Free a job's slot and arena range (synchronises). */
int df_engine_release(df_engine *eng, int32_t slot);

/* out[0] graph replays, out[1] graph captures since creation, out[2] jobs
 * advanced by the batched launches of the current graph (one launch per stage
 * for all of them). */
int df_engine_stats(df_engine *eng, int64_t out[3]);

int df_engine_destroy(df_engine *eng);

/* Measurement reference (no part of the method): a plain device copy of
 * `bytes` bytes from src to dst on `stream` (a hipStream_t, or NULL), by a
 * grid-stride kernel with 16-byte loads and stores, asynchronous.  Both
 * pointers must be 16-byte aligned device memory and bytes a multiple of 16
 * (DF_EINVAL otherwise); the ranges must not overlap.  Its rate is the
 * attainable HBM bandwidth the kernels' rooflines are set beside. */
int df_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the force on
 * the perturber of one level's density field, as df_force computes it for a
 * single-level run, with no arena, no handle and no allocation.
 *  rho    : device pointer, nx*ny*nz total densities (FP64, x fastest, no
 *           padding), read only; the perturber sits at the central vertex and
 *           cell (i,j,k) is centred at ((i - nx/2 + 1/2) dx, ...);
 *  nx, ny, nz : even, >= 2, at most DF_FORCE_DENSITY_MAX_CELLS cells;
 *  dx > 0, GM >= 0, eps >= 0 (Plummer length), rho0 the background density;
 *  out    : device pointer to 3 doubles, receives (Fx, Fy, Fz);
 *  stream : hipStream_t (or NULL); asynchronous, launches two kernels.
 * The per-block partials live in a 96 KiB device array of the library, one
 * per GPU, held until the process ends: calls that overlap on one GPU (two
 * streams, or two host threads) race on it and must be serialised.  No step
 * allocates or synchronises, so the call can be captured into a HIP graph.
 * DF_EINVAL for bad sizes or parameters or null pointers, DF_EDEVICE when the
 * array's device address cannot be obtained or a launch fails. */
#define DF_FORCE_DENSITY_MAX_CELLS (1L << 31)
int df_force_density(const double *rho, int32_t nx, int32_t ny, int32_t nz, double dx, double GM, double eps,
                     double rho0, double *out, void *stream);

const char *df_strerror(int code);
const char *df_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DF_H */
