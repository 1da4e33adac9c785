/*
 * dfo.c -- plain FP64 CPU reference ("the oracle") of the per-timestep update
 * of a uniform gas streaming past a massive, optionally luminous point
 * perturber on nested, x2-refined Cartesian meshes, after Velasco Romero &
 * Masset (2018), "Numerical study of dynamical friction with thermal effects
 * -- I", Sect. 3 (numerical implementation) and Sect. 2.1 (eqs. 1-3).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which is
 * loaded by the test-suite, by the smoke check and by the CPU-baseline leg of
 * the benchmark, and by nothing else.  The HIP product library never links,
 * loads or calls it, and the two share no code, headers or tables.
 *
 * Style: every stage is a separate loop nest that reads the values before the
 * stage and writes new ones (Jacobi sweeps, no fusion, no blocking), in the
 * order of the paper's staging list (Sect. 3.3).  FP64 throughout; build with
 * -ffp-contract=off so that no multiply-add is fused behind the reader's back.
 * OpenMP only distributes independent cells over k-planes; every reduction
 * runs serially in a fixed order, so results do not depend on thread count.
 *
 * Where the paper leaves the discrete form to the cited hydro-code papers
 * (ZEUS / FARGO3D substeps, van Leer transport), this file takes the reading
 * listed at each function.  Parity status of each function is stated in its
 * comment ("pinned by" = the independent check in tests/, "parity unpinned"
 * where no check other than this code exists).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define DFO_MAXLEV 16
#define NSTATE 5 /* rho, e, vx, vy, vz */
#define NQ 8     /* transported: rho, e, P-x, P+x, P-y, P+y, P-z, P+z */

enum { S_RHO = 0, S_E = 1, S_VX = 2, S_VY = 3, S_VZ = 4 };

typedef struct {
  int nx, ny, nz;     /* active cells per level (same on every level)      */
  int nlevels;        /* >= 1; level l+1 covers the central half of level l */
  int g0, gf;         /* ghost width on level 0 and on finer levels        */
  double dx0;         /* cell size on level 0                              */
  double gamma, cfl;  /* adiabatic index, Courant factor                   */
  double rho0, cs;    /* background density and adiabatic sound speed     */
  uint64_t seed;      /* density-noise seed                                */
  double noise_amp;   /* relative amplitude of the density noise           */
  double GM, eps, L, mach, chi; /* perturber and gas parameters            */
  int subcycle;       /* 0: two sub-steps per level; 1: App. A criterion    */
  int bcmode;         /* level-0 boundaries: 0 inflow/outflow; 1 Sect. 3.4  */
  double visc;        /* artificial-viscosity coefficient C2 (0: off)       */
  int nx1, ny1, nz1;  /* cells of every level >= 1 (0: those of level 0)    */
  int quadrant;       /* 1: the domain is y > 0, z > 0 (Sect. 3.4's quadrant) */
} dfo_params;

typedef struct {
  int n[3], g, s[3];
  size_t vol;
  double dx;
  double *st[NSTATE];
  double *q[NQ], *qn[NQ], *fl[NQ], *sp[NQ];
  double *tmp;
  double *acc[3][2][NQ]; /* fine-level frontier transfers [dir][side][q]   */
  double *hw;            /* heat-release weight per active cell            */
  double org[3];         /* index of the perturber's vertex along each dimension */
} lev_t;

typedef struct {
  dfo_params p;
  int nl;
  lev_t lev[DFO_MAXLEV];
  double t, dt_last, bflux, e0, V;
  long nsteps;
  int xi[DFO_MAXLEV];    /* sub-steps of level l+1 per step of level l       */
  int anch[3];           /* quadrant: the domain starts at the perturber's mirror plane */
  double mult;           /* copies of the domain in the whole space (mirror images) */
} run_t;

/* ------------------------------------------------------------------ index */
/* The finer level l+1 covers the central n_{l+1}/2 cells of level l in each
 * dimension (every level has the perturber's vertex at its centre): with
 * equal cell counts that is the central half (Sect. 3.4), with the finer
 * levels half as wide as level 0 level 1 covers the central quarter of it
 * (the mesh of Sect. 4.1.3 and 4.2.2).  o: first covered cell, h: count. */
static void cov_box(const run_t *R, int lc, int o[3], int h[3]);
static void mirror_fill(run_t *R, int lvl);

static inline size_t IX(const lev_t *L, int i, int j, int k) {
  return ((size_t)(k + L->g) * (size_t)L->s[1] + (size_t)(j + L->g)) * (size_t)L->s[0] +
         (size_t)(i + L->g);
}
static inline long STR(const lev_t *L, int d) {
  return d == 0 ? 1L : (d == 1 ? (long)L->s[0] : (long)L->s[0] * (long)L->s[1]);
}
/* cell-centre coordinate along dimension d (perturber on the central vertex,
 * or on the low face of an anchored dimension of the quadrant) */
static inline double XC(const lev_t *L, int d, int i) {
  return ((double)i - L->org[d] + 0.5) * L->dx;
}

/* -------------------------------------------------------------- potential */

/* Plummer potential of the perturber, eq. 16 with the minus sign of the point
 * mass potential of Sect. 2.1 (the sign is lost in the typeset eq. 16). */
static double phi_at(const run_t *R, const lev_t *L, int i, int j, int k) {
  double x = XC(L, 0, i), y = XC(L, 1, j), z = XC(L, 2, k);
  return -R->p.GM / sqrt(x * x + y * y + z * z + R->p.eps * R->p.eps);
}

/* ------------------------------------------------------- van Leer limiter */

/* Harmonic (van Leer 1977) limited difference of two one-sided differences. */
static inline double vl(double a, double b) { return (a * b > 0.0) ? 2.0 * a * b / (a + b) : 0.0; }

/* ----------------------------------------------------------- ranges */
/* Level 0 computes its active entries and reads boundary ghosts that are
 * refilled before every stage.  Finer levels have no boundary conditions:
 * after the ghost fill from the coarse level (CommUp) every entry whose
 * stencil lies inside the allocated array is advanced, so that the ghost
 * shell, twice as wide as one cycle's dependency radius, carries valid data
 * through both sub-cycles without a second fill (Sect. 3.2.1). */
typedef struct { int lo[3], hi[3]; } box_t;

/* faces normal to dimension dn whose two neighbour cells exist */
static box_t box_faces(const lev_t *L, int lvl, int dn) {
  box_t b;
  for (int d = 0; d < 3; ++d) {
    if (lvl == 0) { b.lo[d] = 0; b.hi[d] = L->n[d] + (d == dn ? 1 : 0); }
    else { b.lo[d] = -L->g + (d == dn ? 1 : 0); b.hi[d] = L->n[d] + L->g; }
  }
  return b;
}
/* cells whose right faces exist in every dimension */
static box_t box_cells_r(const lev_t *L, int lvl) {
  box_t b;
  for (int d = 0; d < 3; ++d) {
    if (lvl == 0) { b.lo[d] = 0; b.hi[d] = L->n[d]; }
    else { b.lo[d] = -L->g; b.hi[d] = L->n[d] + L->g - 1; }
  }
  return b;
}
/* cells with both neighbours in every dimension */
static box_t box_cells_1(const lev_t *L, int lvl) {
  box_t b;
  for (int d = 0; d < 3; ++d) {
    if (lvl == 0) { b.lo[d] = 0; b.hi[d] = L->n[d]; }
    else { b.lo[d] = -L->g + 1; b.hi[d] = L->n[d] + L->g - 1; }
  }
  return b;
}

/* --------------------------------------------------- boundary conditions */
/* Level-0 boundaries, mode 0 (reading of Sect. 3.4 for a full box with the gas
 * entering through x_max): the upstream ghosts hold the unperturbed inflow
 * state (rho0, -V, 0, 0, e0); every other ghost copies the nearest active
 * cell (centred fields and tangential velocities) or the boundary face
 * (normal velocity), i.e. zero-gradient outflow.
 * Mode 1 (the boundary list of Sect. 3.4, with the flow along x and the full
 * box, of which the paper's quadrant is one quarter by symmetry): at both
 * flow ends the ghosts hold rho0, -V (normal velocity) and e0 and the
 * tangential velocities are mirror-symmetric; at the four transverse walls
 * every field is mirror-symmetric except the normal velocity, which is
 * antisymmetric (zero on the wall). */

/* mirror index of a ghost across the low (idx < 0) or high (idx >= n) side */
static inline int mirror(int idx, int n) { return idx < 0 ? -1 - idx : (idx >= n ? 2 * n - 1 - idx : idx); }

/* centred field; qin = the value held at the flow ends (inflow in mode 0);
 * xdir: mode 1 holds qin at both flow ends (else mirror-symmetric there) */
static void bc_centred_x(const run_t *R, lev_t *L, double *a, double qin, int xdir) {
  int g = L->g, nx = L->n[0], ny = L->n[1], nz = L->n[2];
  int m1 = R->p.bcmode == 1;
  for (int k = -g; k < nz + g; ++k)
    for (int j = -g; j < ny + g; ++j) {
      for (int i = nx; i < nx + g; ++i)
        a[IX(L, i, j, k)] = (m1 && !xdir) ? a[IX(L, mirror(i, nx), j, k)] : qin;
      for (int i = -g; i < 0; ++i)
        a[IX(L, i, j, k)] = m1 ? (xdir ? qin : a[IX(L, mirror(i, nx), j, k)]) : a[IX(L, 0, j, k)];
    }
  for (int k = -g; k < nz + g; ++k)
    for (int i = -g; i < nx + g; ++i) {
      for (int j = -g; j < 0; ++j) a[IX(L, i, j, k)] = a[IX(L, i, m1 ? mirror(j, ny) : 0, k)];
      for (int j = ny; j < ny + g; ++j) a[IX(L, i, j, k)] = a[IX(L, i, m1 ? mirror(j, ny) : ny - 1, k)];
    }
  for (int j = -g; j < ny + g; ++j)
    for (int i = -g; i < nx + g; ++i) {
      for (int k = -g; k < 0; ++k) a[IX(L, i, j, k)] = a[IX(L, i, j, m1 ? mirror(k, nz) : 0)];
      for (int k = nz; k < nz + g; ++k) a[IX(L, i, j, k)] = a[IX(L, i, j, m1 ? mirror(k, nz) : nz - 1)];
    }
}

static void bc_centred(const run_t *R, lev_t *L, double *a, double qin) { bc_centred_x(R, L, a, qin, 1); }

/* velocity normal to faces of dimension dn; active faces are 0..n[dn] */
static void bc_face(const run_t *R, lev_t *L, double *a, int dn) {
  int g = L->g, n[3] = {L->n[0], L->n[1], L->n[2]};
  int i, j, k;
  if (R->p.bcmode == 1) {
    /* x: flow ends */
    for (k = -g; k < n[2] + g; ++k)
      for (j = -g; j < n[1] + g; ++j) {
        if (dn == 0) {
          for (i = n[0]; i < n[0] + g; ++i) a[IX(L, i, j, k)] = -R->V;
          for (i = -g; i < 0; ++i) a[IX(L, i, j, k)] = -R->V;
        } else {
          for (i = n[0]; i < n[0] + g; ++i) a[IX(L, i, j, k)] = a[IX(L, mirror(i, n[0]), j, k)];
          for (i = -g; i < 0; ++i) a[IX(L, i, j, k)] = a[IX(L, mirror(i, n[0]), j, k)];
        }
      }
    /* y, z: walls */
    for (k = -g; k < n[2] + g; ++k)
      for (i = -g; i < n[0] + g; ++i) {
        if (dn == 1) {
          a[IX(L, i, 0, k)] = 0.0;
          a[IX(L, i, n[1], k)] = 0.0;
          for (j = -g; j < 0; ++j) a[IX(L, i, j, k)] = -a[IX(L, i, -j, k)];
          for (j = n[1] + 1; j < n[1] + g; ++j) a[IX(L, i, j, k)] = -a[IX(L, i, 2 * n[1] - j, k)];
        } else {
          for (j = -g; j < 0; ++j) a[IX(L, i, j, k)] = a[IX(L, i, mirror(j, n[1]), k)];
          for (j = n[1]; j < n[1] + g; ++j) a[IX(L, i, j, k)] = a[IX(L, i, mirror(j, n[1]), k)];
        }
      }
    for (j = -g; j < n[1] + g; ++j)
      for (i = -g; i < n[0] + g; ++i) {
        if (dn == 2) {
          a[IX(L, i, j, 0)] = 0.0;
          a[IX(L, i, j, n[2])] = 0.0;
          for (k = -g; k < 0; ++k) a[IX(L, i, j, k)] = -a[IX(L, i, j, -k)];
          for (k = n[2] + 1; k < n[2] + g; ++k) a[IX(L, i, j, k)] = -a[IX(L, i, j, 2 * n[2] - k)];
        } else {
          for (k = -g; k < 0; ++k) a[IX(L, i, j, k)] = a[IX(L, i, j, mirror(k, n[2]))];
          for (k = n[2]; k < n[2] + g; ++k) a[IX(L, i, j, k)] = a[IX(L, i, j, mirror(k, n[2]))];
        }
      }
    return;
  }
  /* x */
  for (k = -g; k < n[2] + g; ++k)
    for (j = -g; j < n[1] + g; ++j) {
      if (dn == 0) {
        for (i = n[0] + 1; i < n[0] + g; ++i) a[IX(L, i, j, k)] = -R->V;
        a[IX(L, n[0], j, k)] = -R->V;
        for (i = -g; i < 0; ++i) a[IX(L, i, j, k)] = a[IX(L, 0, j, k)];
      } else {
        for (i = n[0]; i < n[0] + g; ++i) a[IX(L, i, j, k)] = 0.0;
        for (i = -g; i < 0; ++i) a[IX(L, i, j, k)] = a[IX(L, 0, j, k)];
      }
    }
  /* y */
  for (k = -g; k < n[2] + g; ++k)
    for (i = -g; i < n[0] + g; ++i) {
      int top = (dn == 1) ? n[1] : n[1] - 1;
      for (j = -g; j < 0; ++j) a[IX(L, i, j, k)] = a[IX(L, i, 0, k)];
      for (j = top + 1; j < n[1] + g; ++j) a[IX(L, i, j, k)] = a[IX(L, i, top, k)];
    }
  /* z */
  for (j = -g; j < n[1] + g; ++j)
    for (i = -g; i < n[0] + g; ++i) {
      int top = (dn == 2) ? n[2] : n[2] - 1;
      for (k = -g; k < 0; ++k) a[IX(L, i, j, k)] = a[IX(L, i, j, 0)];
      for (k = top + 1; k < n[2] + g; ++k) a[IX(L, i, j, k)] = a[IX(L, i, j, top)];
    }
}

static void bc_state(run_t *R) {
  lev_t *L = &R->lev[0];
  bc_centred(R, L, L->st[S_RHO], R->p.rho0);
  bc_centred(R, L, L->st[S_E], R->e0);
  for (int d = 0; d < 3; ++d) bc_face(R, L, L->st[S_VX + d], d);
}

/* inflow values of the transported quantities */
static double q_inflow(const run_t *R, int iq) {
  if (iq == 0) return R->p.rho0;
  if (iq == 1) return R->e0;
  if (iq == 2 || iq == 3) return R->p.rho0 * (-R->V);
  return 0.0;
}

/* mode 1: the pair of momenta normal to a wall (P- = rho v(low face), P+ = rho
 * v(high face)): the mirror of a cell has its faces swapped and the normal
 * velocity reversed, so P-(ghost) = -P+(mirror cell) and P+(ghost) = -P-(mirror) */
static void bc_wall_pair(lev_t *L, double *pm, double *pp, int d) {
  int g = L->g, n[3] = {L->n[0], L->n[1], L->n[2]};
  for (int a2 = -g; a2 < n[(d + 2) % 3] + g; ++a2)
    for (int a1 = -g; a1 < n[(d + 1) % 3] + g; ++a1)
      for (int side = 0; side < 2; ++side)
        for (int t = 0; t < g; ++t) {
          int id[3], im[3];
          id[(d + 1) % 3] = im[(d + 1) % 3] = a1;
          id[(d + 2) % 3] = im[(d + 2) % 3] = a2;
          id[d] = side ? n[d] + t : -1 - t;
          im[d] = mirror(id[d], n[d]);
          size_t c = IX(L, id[0], id[1], id[2]), m = IX(L, im[0], im[1], im[2]);
          pm[c] = -pp[m];
          pp[c] = -pm[m];
        }
}

static void bc_q(run_t *R) {
  lev_t *L = &R->lev[0];
  if (R->p.bcmode != 1) {
    for (int iq = 0; iq < NQ; ++iq) bc_centred(R, L, L->q[iq], q_inflow(R, iq));
    return;
  }
  /* rho, e, P-x, P+x: background at the flow ends; every quantity
   * mirror-symmetric at the walls, then the wall-normal momentum pairs
   * replaced by their reversed mirrors.  The tangential momenta at the flow
   * ends are those of the ghost's own state: the background density times the
   * mirror cell's velocity, P = rho0 (P_m / rho_m) (Sect. 3.4 sets the
   * primitive variables in the ghost zones). */
  for (int iq = 0; iq < NQ; ++iq) bc_centred_x(R, L, L->q[iq], q_inflow(R, iq), iq < 4);
  int g = L->g, nx = L->n[0];
  for (int iq = 4; iq < NQ; ++iq)
    for (int k = -g; k < L->n[2] + g; ++k)
      for (int j = -g; j < L->n[1] + g; ++j)
        for (int t = 0; t < g; ++t)
          for (int side = 0; side < 2; ++side) {
            int i = side ? nx + t : -1 - t, im = mirror(i, nx);
            int jm = mirror(j, L->n[1]), km = mirror(k, L->n[2]);
            size_t c = IX(L, i, j, k), m = IX(L, im, jm, km);
            L->q[iq][c] = L->q[0][c] * (L->q[iq][m] / L->q[0][m]);
          }
  bc_wall_pair(L, L->q[4], L->q[5], 1);
  bc_wall_pair(L, L->q[6], L->q[7], 2);
}

/* reset the upstream (inflow) face of level 0 to the injection velocity;
 * mode 1 also holds the wall faces at zero normal velocity */
static void reset_inflow_face(run_t *R) {
  lev_t *L = &R->lev[0];
  for (int k = -L->g; k < L->n[2] + L->g; ++k)
    for (int j = -L->g; j < L->n[1] + L->g; ++j) L->st[S_VX][IX(L, L->n[0], j, k)] = -R->V;
  if (R->p.bcmode == 1) {
    for (int k = -L->g; k < L->n[2] + L->g; ++k)
      for (int i = -L->g; i < L->n[0] + L->g; ++i) {
        L->st[S_VY][IX(L, i, 0, k)] = 0.0;
        L->st[S_VY][IX(L, i, L->n[1], k)] = 0.0;
      }
    for (int j = -L->g; j < L->n[1] + L->g; ++j)
      for (int i = -L->g; i < L->n[0] + L->g; ++i) {
        L->st[S_VZ][IX(L, i, j, 0)] = 0.0;
        L->st[S_VZ][IX(L, i, j, L->n[2])] = 0.0;
      }
  }
}

/* ------------------------------------------------------------------ kick */
/* Source sub-step S(h), the velocity part (SubStep1 of the staging list,
 * Sect. 3.2.3, eq. 15): every face velocity receives
 *   v_f -= h * [ (p_c - p_{c-1}) / (dx * rho_face) + (Phi_c - Phi_{c-1}) / dx ]
 * with p = (gamma-1) e (Sect. 2.1), rho_face the mean of the two adjacent
 * cells and Phi the Plummer potential at cell centres (eq. 16).
 * Pinned by: uniform-flow invariance, linear sound speed, cold-drag sign and
 * GM^2 scaling, mirror symmetry. */
static void kick(run_t *R, int lvl, double h) {
  lev_t *L = &R->lev[lvl];
  const double gm1 = R->p.gamma - 1.0, dx = L->dx;
  const double *rho = L->st[S_RHO], *e = L->st[S_E];
  for (int dn = 0; dn < 3; ++dn) {
    box_t b = box_faces(L, lvl, dn);
    long s = STR(L, dn);
    double *v = L->st[S_VX + dn];
#pragma omp parallel for schedule(static)
    for (int k = b.lo[2]; k < b.hi[2]; ++k)
      for (int j = b.lo[1]; j < b.hi[1]; ++j)
        for (int i = b.lo[0]; i < b.hi[0]; ++i) {
          size_t c = IX(L, i, j, k), m = c - (size_t)s;
          int im = i - (dn == 0), jm = j - (dn == 1), km = k - (dn == 2);
          double rface = 0.5 * (rho[m] + rho[c]);
          double gradp = gm1 * (e[c] - e[m]) / (dx * rface);
          double gradphi = (phi_at(R, L, i, j, k) - phi_at(R, L, im, jm, km)) / dx;
          v[c] = v[c] - h * (gradp + gradphi);
        }
  }
  if (lvl == 0) reset_inflow_face(R);
}

/* ----------------------------------------------------------- compression */
/* Compressional heating -p div(v) (SubStep3 of the staging list), taken in
 * the time-centred implicit form of the ZEUS-type codes the paper builds on:
 * with a = (gamma-1) dt div(v) / 2,  e <- e (1 - a) / (1 + a).
 * Pinned by: linear sound speed sqrt(gamma p0/rho0) (an isothermal update
 * would give sqrt(p0/rho0)), uniform-flow invariance. */
static void compress(run_t *R, int lvl, double dt) {
  lev_t *L = &R->lev[lvl];
  const double gm1 = R->p.gamma - 1.0, dx = L->dx;
  const double *u = L->st[S_VX], *v = L->st[S_VY], *w = L->st[S_VZ];
  double *e = L->st[S_E];
  box_t b = box_cells_r(L, lvl);
  long sx = STR(L, 0), sy = STR(L, 1), sz = STR(L, 2);
#pragma omp parallel for schedule(static)
  for (int k = b.lo[2]; k < b.hi[2]; ++k)
    for (int j = b.lo[1]; j < b.hi[1]; ++j)
      for (int i = b.lo[0]; i < b.hi[0]; ++i) {
        size_t c = IX(L, i, j, k);
        double divv = ((u[c + sx] - u[c]) + (v[c + sy] - v[c]) + (w[c + sz] - w[c])) / dx;
        double a = 0.5 * gm1 * dt * divv;
        e[c] = e[c] * (1.0 - a) / (1.0 + a);
      }
}

/* ------------------------------------------------- artificial viscosity */
/* SubStep2 of the staging list (Sect. 3.3), which the paper names without
 * giving it: the von Neumann-Richtmyer viscosity of ZEUS (Stone & Norman
 * 1992, ApJS 80, 753), opt-in with coefficient C2 = p.visc (0: off, the
 * default).  Per dimension d and cell c, with dv = v_d(high face) - v_d(low
 * face): q_d(c) = C2 rho(c) dv^2 where dv < 0 (compression), else 0.  Each face
 * velocity v_d -= dt (q_d(c) - q_d(c-1)) / (dx rho_face) with rho_face the
 * mean of the two cells, and e(c) -= dt sum_d q_d(c) dv_d(c) / dx, all from
 * the values before the stage.  On level 0 the faces reset by the boundary
 * conditions (the inflow face, walls) keep their values. */
static double visc_q(const lev_t *L, const double *rho, const double *v, size_t c, long s, double c2) {
  double dv = v[c + s] - v[c];
  return dv < 0.0 ? c2 * rho[c] * dv * dv : 0.0;
}

static void viscosity(run_t *R, int lvl, double dt) {
  const double c2 = R->p.visc;
  if (!(c2 > 0.0)) return;
  lev_t *L = &R->lev[lvl];
  const double dx = L->dx, *rho = L->st[S_RHO];
  double *e = L->st[S_E];
  /* energy, from the pre-stage velocities */
  box_t cb = box_cells_r(L, lvl);
#pragma omp parallel for schedule(static)
  for (int k = cb.lo[2]; k < cb.hi[2]; ++k)
    for (int j = cb.lo[1]; j < cb.hi[1]; ++j)
      for (int i = cb.lo[0]; i < cb.hi[0]; ++i) {
        size_t c = IX(L, i, j, k);
        double de = 0.0;
        for (int d = 0; d < 3; ++d) {
          const double *v = L->st[S_VX + d];
          long s = STR(L, d);
          de += visc_q(L, rho, v, c, s, c2) * (v[c + s] - v[c]);
        }
        e[c] -= dt * de / dx;
      }
  /* face velocities, new values into tmp then copied back (Jacobi) */
  for (int d = 0; d < 3; ++d) {
    double *v = L->st[S_VX + d];
    long s = STR(L, d);
    box_t b = box_faces(L, lvl, d);
    if (lvl > 0) { b.lo[d] = -L->g + 1; for (int e2 = 0; e2 < 3; ++e2) b.hi[e2] = L->n[e2] + L->g - 1; }
    memcpy(L->tmp, v, L->vol * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = b.lo[2]; k < b.hi[2]; ++k)
      for (int j = b.lo[1]; j < b.hi[1]; ++j)
        for (int i = b.lo[0]; i < b.hi[0]; ++i) {
          size_t c = IX(L, i, j, k), m = c - (size_t)s;
          double qc = visc_q(L, rho, v, c, s, c2), qm = visc_q(L, rho, v, m, s, c2);
          L->tmp[c] = v[c] - dt * (qc - qm) / (dx * 0.5 * (rho[m] + rho[c]));
        }
    memcpy(v, L->tmp, L->vol * sizeof(double));
  }
  if (lvl == 0) reset_inflow_face(R);
}

/* ------------------------------------------------------------- diffusion */
/* Thermal diffusion, eqs. 19-22: face energy fluxes proportional to chi rho0
 * times the difference of e/rho across the face, times the face area over the
 * cell size, and the cell energy changed by dt times the flux divergence over
 * the cell volume.  The flux is taken down the gradient of e/rho (Fourier's
 * law), the sign under which the linearised energy equation (eq. 28) is
 * dissipative; eqs. 3 and 22 as typeset carry the opposite sign on both the
 * flux and the update, which cancels.  All fluxes use the values before the
 * stage (Jacobi).
 * Pinned by: exact decay of discrete cosine modes, Gaussian closed form with
 * second-order convergence, uniform invariance. */
static double fourier_flux(double chi_rho0, double Tl, double Tr, double dx) {
  double area = dx * dx;
  return -chi_rho0 * (Tr - Tl) * area / dx; /* energy per unit time through the face, +d direction */
}

static void diffuse(run_t *R, int lvl, double dt) {
  if (R->p.chi == 0.0) return;
  lev_t *L = &R->lev[lvl];
  const double dx = L->dx, vol = dx * dx * dx, kr = R->p.chi * R->p.rho0;
  const double *rho = L->st[S_RHO];
  double *e = L->st[S_E], *e0 = L->tmp;
  memcpy(e0, e, L->vol * sizeof(double));
  box_t b = box_cells_1(L, lvl);
#pragma omp parallel for schedule(static)
  for (int k = b.lo[2]; k < b.hi[2]; ++k)
    for (int j = b.lo[1]; j < b.hi[1]; ++j)
      for (int i = b.lo[0]; i < b.hi[0]; ++i) {
        size_t c = IX(L, i, j, k);
        double Tc = e0[c] / rho[c];
        double net = 0.0;
        for (int d = 0; d < 3; ++d) {
          long s = STR(L, d);
          double Tm = e0[c - s] / rho[c - s], Tp = e0[c + s] / rho[c + s];
          double f_left = fourier_flux(kr, Tm, Tc, dx);
          double f_right = fourier_flux(kr, Tc, Tp, dx);
          net += f_right - f_left;
        }
        e[c] = e0[c] - dt * net / vol;
      }
}

/* ------------------------------------------------------------ heat release */
/* Release of L dt into the cells around the perturber (Sect. 3.4): the paper
 * splits it equally over the 8 cells sharing the perturber's vertex.  The
 * weights generalise this to a normalised Gaussian of width sigma = eps over
 * the active cells (truncated at r_min + 8 sigma); sigma = 0 is exactly the
 * 8-cell split.
 * Pinned by: sum of deposited energy = L dt, weights = 1/8 on 8 cells. */
static void heat_weights(run_t *R, int lvl) {
  lev_t *L = &R->lev[lvl];
  size_t na = (size_t)L->n[0] * L->n[1] * L->n[2];
  double sig = R->p.eps;
  double r2min = INFINITY;
  for (int k = 0; k < L->n[2]; ++k)
    for (int j = 0; j < L->n[1]; ++j)
      for (int i = 0; i < L->n[0]; ++i) {
        double x = XC(L, 0, i), y = XC(L, 1, j), z = XC(L, 2, k);
        double r2 = x * x + y * y + z * z;
        if (r2 < r2min) r2min = r2;
      }
  double rcut = sqrt(r2min) + 8.0 * sig;
  double sum = 0.0;
  for (int k = 0; k < L->n[2]; ++k)
    for (int j = 0; j < L->n[1]; ++j)
      for (int i = 0; i < L->n[0]; ++i) {
        double x = XC(L, 0, i), y = XC(L, 1, j), z = XC(L, 2, k);
        double r2 = x * x + y * y + z * z;
        double gw = 0.0;
        if (sig == 0.0) gw = (r2 == r2min) ? 1.0 : 0.0;
        else if (sqrt(r2) <= rcut) gw = exp(-(r2 - r2min) / (2.0 * sig * sig));
        L->hw[((size_t)k * L->n[1] + j) * L->n[0] + i] = gw;
        sum += gw;
      }
  /* quadrant: the cells' mirror images hold the same weights, so the whole
   * set sums to mult times the domain's */
  for (size_t a = 0; a < na; ++a) L->hw[a] /= sum * R->mult;
}

static void heat(run_t *R, int lvl, double dt) {
  if (R->p.L == 0.0) return;
  lev_t *L = &R->lev[lvl];
  double vol = L->dx * L->dx * L->dx;
  double *e = L->st[S_E];
  for (int k = 0; k < L->n[2]; ++k)
    for (int j = 0; j < L->n[1]; ++j)
      for (int i = 0; i < L->n[0]; ++i) {
        double w = L->hw[((size_t)k * L->n[1] + j) * L->n[0] + i];
        if (w != 0.0) e[IX(L, i, j, k)] += R->p.L * dt * w / vol;
      }
  /* quadrant, finer levels: the ghosts beyond a mirror plane are advanced
   * with the level as the mirror images of its cells (mirror_fill), so the
   * images of the heated cells are heated too */
  if (lvl == 0 || !(R->anch[1] || R->anch[2])) return;
  const int g = L->g;
  for (int k = -g; k < L->n[2]; ++k)
    for (int j = -g; j < L->n[1]; ++j) {
      if (j >= 0 && k >= 0) continue;
      if ((j < 0 && !R->anch[1]) || (k < 0 && !R->anch[2])) continue;
      const int jm = j < 0 ? -1 - j : j, km = k < 0 ? -1 - k : k;
      if (jm >= L->n[1] || km >= L->n[2]) continue;
      for (int i = 0; i < L->n[0]; ++i) {
        double w = L->hw[((size_t)km * L->n[1] + jm) * L->n[0] + i];
        if (w != 0.0) e[IX(L, i, j, k)] += R->p.L * dt * w / vol;
      }
    }
}

/* ------------------------------------------------------------- transport */
/* Transport T(dt) (FluxIntegration + Transport of the staging list), reading
 * of the FARGO3D/ZEUS upwind scheme with van Leer's second-order face values:
 *  - transported set: rho, e and, per dimension d, the two cell momenta
 *    P-_d = rho_c v_d(left face), P+_d = rho_c v_d(right face);
 *  - dimensional passes x, y, z; each face f between c- and c+ moves with the
 *    velocity a_f left by the first half kick (the partially updated v^p of
 *    Sect. 3.2.3), the same for all three passes;
 *  - van Leer upwind face value of a cell quantity s, with the limited
 *    difference ds_c = vl(s_{c+1}-s_c, s_c-s_{c-1}) and nu = a_f dt / dx:
 *      a_f > 0 : s_{c-} + ds_{c-} (1 - nu) / 2
 *      else    : s_{c+} - ds_{c+} (1 + nu) / 2
 *  - mass transfer M_f = face(rho) a_f dt dx^2 (area and time integrated);
 *    the other quantities move as face(q/rho) M_f (consistent transport),
 *    q/rho taken with the density before the pass;
 *  - each cell changes by minus the difference of its two face transfers
 *    divided by its volume;
 *  - after the z pass the face velocities are rebuilt as
 *    (P+_{c-} + P-_{c+}) / (rho_{c-} + rho_{c+}).
 * Flux matching (CommFlux, Sect. 3.2.3): a fine level adds its transfers
 * through its outer (frontier) faces into accumulators over its two
 * sub-cycles; the coarse level replaces its own transfers through the same
 * interfaces by the sum of the 4 fine faces and 2 sub-cycles.
 * Pinned by: uniform invariance (bitwise), mass accounting to round-off on a
 * single level, composite mass conservation across levels, linear sound
 * speed, and the conservation of energy and of the three momenta (the sum of
 * the cell momenta the stage builds against the one its rebuilt faces hold)
 * by the transport stage on one level, to round-off.  The choice of the
 * momentum pairing and the matching of momentum and energy transfers across
 * levels are a reading: parity unpinned beyond those checks. */
static void build_momenta(run_t *R, int lvl) {
  lev_t *L = &R->lev[lvl];
  const double *rho = L->st[S_RHO];
  box_t b = box_cells_r(L, lvl);
  memcpy(L->q[0], rho, L->vol * sizeof(double));
  memcpy(L->q[1], L->st[S_E], L->vol * sizeof(double));
  for (int d = 0; d < 3; ++d) {
    const double *v = L->st[S_VX + d];
    long s = STR(L, d);
    double *pm = L->q[2 + 2 * d], *pp = L->q[3 + 2 * d];
#pragma omp parallel for schedule(static)
    for (int k = b.lo[2]; k < b.hi[2]; ++k)
      for (int j = b.lo[1]; j < b.hi[1]; ++j)
        for (int i = b.lo[0]; i < b.hi[0]; ++i) {
          size_t c = IX(L, i, j, k);
          pm[c] = rho[c] * v[c];
          pp[c] = rho[c] * v[c + s];
        }
  }
}

static inline double upwind_face(const double *s, size_t cm, long st, double a, double nu) {
  size_t cp = cm + (size_t)st;
  if (a > 0.0) {
    double ds = vl(s[cp] - s[cm], s[cm] - s[cm - st]);
    return s[cm] + 0.5 * ds * (1.0 - nu);
  } else {
    double ds = vl(s[cp + st] - s[cp], s[cp] - s[cm]);
    return s[cp] - 0.5 * ds * (1.0 + nu);
  }
}

/* transverse dimensions of a face normal to dn, in increasing order */
static void tdims(int dn, int *t1, int *t2) {
  *t1 = (dn == 0) ? 1 : 0;
  *t2 = (dn == 2) ? 1 : 2;
}

static void transport_pass(run_t *R, int lvl, int dn, double dt) {
  lev_t *L = &R->lev[lvl];
  const double dx = L->dx, vol = dx * dx * dx;
  const double *a = L->st[S_VX + dn];
  long s = STR(L, dn);
  int g = L->g;
  /* specific values from the values before the pass */
  for (int iq = 1; iq < NQ; ++iq) {
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < L->vol; ++c) L->sp[iq][c] = L->q[iq][c] / L->q[0][c];
  }
  /* faces */
  box_t fb;
  for (int d = 0; d < 3; ++d) {
    if (lvl == 0) { fb.lo[d] = 0; fb.hi[d] = L->n[d] + (d == dn ? 1 : 0); }
    else if (d == dn) { fb.lo[d] = -g + 2; fb.hi[d] = L->n[d] + g - 1; }
    else { fb.lo[d] = -g; fb.hi[d] = L->n[d] + g; }
  }
  for (int iq = 0; iq < NQ; ++iq) memset(L->fl[iq], 0, L->vol * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = fb.lo[2]; k < fb.hi[2]; ++k)
    for (int j = fb.lo[1]; j < fb.hi[1]; ++j)
      for (int i = fb.lo[0]; i < fb.hi[0]; ++i) {
        size_t f = IX(L, i, j, k), cm = f - (size_t)s;
        double af = a[f], nu = af * dt / dx;
        double M = upwind_face(L->q[0], cm, s, af, nu) * af * dt * dx * dx;
        L->fl[0][f] = M;
        for (int iq = 1; iq < NQ; ++iq) L->fl[iq][f] = upwind_face(L->sp[iq], cm, s, af, nu) * M;
      }
  int t1, t2;
  tdims(dn, &t1, &t2);
  /* fine level: accumulate frontier transfers */
  if (lvl > 0) {
    for (int side = 0; side < 2; ++side) {
      int fi = side ? L->n[dn] : 0;
      for (int b2 = 0; b2 < L->n[t2]; ++b2)
        for (int b1 = 0; b1 < L->n[t1]; ++b1) {
          int id[3];
          id[dn] = fi; id[t1] = b1; id[t2] = b2;
          size_t f = IX(L, id[0], id[1], id[2]);
          size_t aidx = (size_t)b2 * L->n[t1] + b1;
          for (int iq = 0; iq < NQ; ++iq) L->acc[dn][side][iq][aidx] += L->fl[iq][f];
        }
    }
  }
  /* coarse level under a finer one: overwrite transfers on the frontier */
  if (lvl < R->nl - 1) {
    lev_t *F = &R->lev[lvl + 1];
    int o[3], h[3];
    cov_box(R, lvl, o, h);
    for (int side = 0; side < 2; ++side) {
      int fi = side ? o[dn] + h[dn] : o[dn];
      for (int b2 = o[t2]; b2 < o[t2] + h[t2]; ++b2)
        for (int b1 = o[t1]; b1 < o[t1] + h[t1]; ++b1) {
          int id[3];
          id[dn] = fi; id[t1] = b1; id[t2] = b2;
          size_t f = IX(L, id[0], id[1], id[2]);
          int f1 = 2 * (b1 - o[t1]), f2 = 2 * (b2 - o[t2]);
          for (int iq = 0; iq < NQ; ++iq) {
            const double *A = F->acc[dn][side][iq];
            size_t nt = (size_t)F->n[t1];
            double s00 = A[(size_t)f2 * nt + f1], s10 = A[(size_t)f2 * nt + f1 + 1];
            double s01 = A[(size_t)(f2 + 1) * nt + f1], s11 = A[(size_t)(f2 + 1) * nt + f1 + 1];
            L->fl[iq][f] = (s00 + s10) + (s01 + s11);
          }
        }
    }
  }
  /* level 0: net mass through the outer boundary (diagnostic) */
  if (lvl == 0) {
    double net = 0.0;
    for (int b2 = 0; b2 < L->n[t2]; ++b2)
      for (int b1 = 0; b1 < L->n[t1]; ++b1) {
        int id[3];
        id[t1] = b1; id[t2] = b2;
        id[dn] = 0;
        net += L->fl[0][IX(L, id[0], id[1], id[2])];
        id[dn] = L->n[dn];
        net -= L->fl[0][IX(L, id[0], id[1], id[2])];
      }
    R->bflux += net;
  }
  /* cells */
  box_t cb = fb;
  if (lvl == 0) cb.hi[dn] = L->n[dn];
  else { cb.lo[dn] = -g + 2; cb.hi[dn] = L->n[dn] + g - 2; }
  for (int iq = 0; iq < NQ; ++iq) memcpy(L->qn[iq], L->q[iq], L->vol * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = cb.lo[2]; k < cb.hi[2]; ++k)
    for (int j = cb.lo[1]; j < cb.hi[1]; ++j)
      for (int i = cb.lo[0]; i < cb.hi[0]; ++i) {
        size_t c = IX(L, i, j, k);
        for (int iq = 0; iq < NQ; ++iq)
          L->qn[iq][c] = L->q[iq][c] - (L->fl[iq][c + s] - L->fl[iq][c]) / vol;
      }
  for (int iq = 0; iq < NQ; ++iq) { double *t = L->q[iq]; L->q[iq] = L->qn[iq]; L->qn[iq] = t; }
}

static void rebuild_velocities(run_t *R, int lvl) {
  lev_t *L = &R->lev[lvl];
  const double *rho = L->q[0];
  for (int dn = 0; dn < 3; ++dn) {
    box_t b = box_faces(L, lvl, dn);
    long s = STR(L, dn);
    const double *pm = L->q[2 + 2 * dn], *pp = L->q[3 + 2 * dn];
    double *v = L->st[S_VX + dn];
#pragma omp parallel for schedule(static)
    for (int k = b.lo[2]; k < b.hi[2]; ++k)
      for (int j = b.lo[1]; j < b.hi[1]; ++j)
        for (int i = b.lo[0]; i < b.hi[0]; ++i) {
          size_t c = IX(L, i, j, k), m = c - (size_t)s;
          v[c] = (pp[m] + pm[c]) / (rho[m] + rho[c]);
        }
  }
  if (lvl == 0) reset_inflow_face(R);
}

static void mirror_q(run_t *R, int lvl);

static void transport(run_t *R, int lvl, double dt) {
  lev_t *L = &R->lev[lvl];
  build_momenta(R, lvl);
  /* quadrant: a finer level with a finer one of its own takes that level's
   * transfers on its frontier faces, whose mirror images lie in its ghosts */
  const int mq = lvl > 0 && lvl < R->nl - 1 && (R->anch[1] || R->anch[2]);
  for (int dn = 0; dn < 3; ++dn) {
    if (lvl == 0) bc_q(R);
    transport_pass(R, lvl, dn, dt);
    if (mq) mirror_q(R, lvl);
  }
  if (lvl == 0) bc_q(R);
  rebuild_velocities(R, lvl);
  memcpy(L->st[S_RHO], L->q[0], L->vol * sizeof(double));
  memcpy(L->st[S_E], L->q[1], L->vol * sizeof(double));
}

/* ------------------------------------------------------- one level step */
/* The staging of one step of length dt on one level (Sect. 3.3 and eq. 15):
 * S(dt/2) [kick] -> SubStep3(dt) [compression, diffusion, heat release]
 * -> T(dt) [transport with flux matching] -> S(dt/2) [kick]. */
static void hydro_step(run_t *R, int lvl, double dt) {
  int l0 = (lvl == 0);
  if (l0) bc_state(R);
  kick(R, lvl, 0.5 * dt);
  if (l0) bc_state(R);
  viscosity(R, lvl, dt);
  if (l0) bc_state(R);
  compress(R, lvl, dt);
  if (l0) bc_state(R);
  diffuse(R, lvl, dt);
  heat(R, lvl, dt);
  if (l0) bc_state(R);
  transport(R, lvl, dt);
  if (l0) bc_state(R);
  kick(R, lvl, 0.5 * dt);
  if (l0) bc_state(R);
}

/* ------------------------------------------------------- CommUp / CommMean */
/* CommUp (Sect. 3.2.1, Fig. 2): every fine entry outside the fine active set
 * is interpolated from the 27 coarse entries around its host, first along z
 * to the fine position, then along y, then along x, each one-dimensional step
 * using van Leer's limited slope.  Positions: a fine cell centre sits a
 * quarter coarse cell from its host centre; a fine face along its own normal
 * coincides with a coarse face (even index) or sits half-way between two,
 * where it takes their mean (a reading: the paper says only that staggered
 * fields differ by their alignment; the mean keeps the fill mirror-symmetric).
 * Pinned by: restriction of a prolongation returns the coarse data,
 * exactness on uniform data, ghost-width independence. */
static inline int fdiv2(int i) { return (i >= 0) ? i / 2 : -((-i + 1) / 2); }

static void commup_fill(run_t *R, int lc, int all) {
  lev_t *C = &R->lev[lc], *F = &R->lev[lc + 1];
  int o[3], hc[3];
  cov_box(R, lc, o, hc);
  int g = F->g;
  for (int fld = 0; fld < NSTATE; ++fld) {
    int stag = (fld >= S_VX) ? fld - S_VX : -1;
    const double *Q = C->st[fld];
    double *out = F->st[fld];
    long sz = STR(C, 2);
#pragma omp parallel for schedule(static)
    for (int k = -g; k < F->n[2] + g; ++k)
      for (int j = -g; j < F->n[1] + g; ++j)
        for (int i = -g; i < F->n[0] + g; ++i) {
          int id[3] = {i, j, k};
          int active = 1, beyond_plane = 0;
          for (int d = 0; d < 3; ++d) {
            int hi = F->n[d] + (d == stag ? 1 : 0);
            if (id[d] < 0 || id[d] >= hi) active = 0;
            if (id[d] < 0 && R->anch[d]) beyond_plane = 1;
          }
          if (active && !all) continue;
          /* quadrant: entries beyond a mirror plane take the fine level's own
           * mirror images instead (mirror_fill) */
          if (beyond_plane) continue;
          int H[3], odd[3];
          double del[3];
          for (int d = 0; d < 3; ++d) {
            H[d] = o[d] + fdiv2(id[d]);
            odd[d] = id[d] - 2 * fdiv2(id[d]);
            del[d] = odd[d] ? 0.25 : -0.25;
          }
          /* one 1-D step: value at the fine position from three consecutive
           * coarse values m, c, p around the host.  Along a face field's own
           * axis an even fine face is the host coarse face itself and an odd
           * one lies half-way between the host face and the next, where the
           * mean of the two is taken (it needs no limiter). */
#define STEP1D(d, m, c, p)                                                         \
  ((d) == stag ? (odd[d] ? 0.5 * ((c) + (p)) : (c)) : (c) + vl((p) - (c), (c) - (m)) * del[d])
          double qz[3][3], r[3];
          for (int a = -1; a <= 1; ++a)
            for (int bb = -1; bb <= 1; ++bb) {
              size_t c = IX(C, H[0] + a, H[1] + bb, H[2]);
              qz[a + 1][bb + 1] = STEP1D(2, Q[c - sz], Q[c], Q[c + sz]);
            }
          for (int a = 0; a < 3; ++a) r[a] = STEP1D(1, qz[a][0], qz[a][1], qz[a][2]);
          out[IX(F, i, j, k)] = STEP1D(0, r[0], r[1], r[2]);
#undef STEP1D
        }
  }
}

/* Quadrant (Sect. 3.4): the mirror planes y = 0 and z = 0 bound every level.
 * Level 0 reads its wall ghosts as mirror images (bc_state); on a finer level
 * the ghost entries beyond an anchored face are the mirror images of its own
 * entries -- centred fields and tangential velocities even, the normal
 * velocity odd (zero on the plane) -- set after each CommUp (which fills them
 * from the coarse level first, so that the corners beyond a frontier take
 * the mirror of their prolonged values), and after each CommMean into the
 * level (the images of the cells it overwrites are the restricted values
 * too, as in the full box).  Both sub-cycles then advance these
 * ghosts with the level (by the scheme's mirror symmetry they stay the mirror
 * images within the dependency radius of the active cells), as the
 * full box advances the same entries as active cells.
 * Pinned by: a quadrant run equals the quarter y, z > 0 of the full box,
 * bitwise (1 to 3 levels, both hierarchies). */
static void mirror_fill(run_t *R, int lvl) {
  lev_t *L = &R->lev[lvl];
  const int g = L->g;
  for (int d = 1; d < 3; ++d) {
    if (!R->anch[d]) continue;
    for (int fld = 0; fld < NSTATE; ++fld) {
      const int normal = (fld == S_VX + d);
      double *a = L->st[fld];
      const long sd = STR(L, d);
      for (int k = -g; k < L->n[2] + g; ++k)
        for (int j = -g; j < L->n[1] + g; ++j)
          for (int i = -g; i < L->n[0] + g; ++i) {
            const int id[3] = {i, j, k};
            if (id[d] >= 0) continue;
            const size_t c = IX(L, i, j, k);
            const long m = id[d];
            if (normal) a[c] = -a[c - 2 * m * sd];      /* face m < 0 <- face -m */
            else a[c] = a[c + (-1 - 2 * m) * sd];        /* cell m < 0 <- cell -1-m */
          }
    }
  }
}

/* the transported set beyond the mirror planes of a finer level: the mirror
 * images of its cells, the momenta normal to a plane swapped and reversed
 * (P-_d of an image is -P+_d of its cell), after every transport pass of a
 * level that takes a finer level's frontier transfers (their images are not
 * matched otherwise) */
static void mirror_q(run_t *R, int lvl) {
  lev_t *L = &R->lev[lvl];
  const int g = L->g;
  for (int d = 1; d < 3; ++d) {
    if (!R->anch[d]) continue;
    const long sd = STR(L, d);
    for (int iq = 0; iq < NQ; ++iq) {
      const int pair = (iq == 2 + 2 * d) ? iq + 1 : ((iq == 3 + 2 * d) ? iq - 1 : -1);
      double *a = L->q[iq];
      const double *src = pair >= 0 ? L->q[pair] : L->q[iq];
      const double sgn = pair >= 0 ? -1.0 : 1.0;
      for (int k = -g; k < L->n[2] + g; ++k)
        for (int j = -g; j < L->n[1] + g; ++j)
          for (int i = -g; i < L->n[0] + g; ++i) {
            const int id[3] = {i, j, k};
            if (id[d] >= 0) continue;
            const size_t c = IX(L, i, j, k);
            a[c] = sgn * src[c + (-1 - 2 * (long)id[d]) * sd];
          }
    }
  }
}

static void commup(run_t *R, int lc) {
  commup_fill(R, lc, 0);
  if (R->anch[1] || R->anch[2]) mirror_fill(R, lc + 1);
}

/* CommMean / CommDown (Sect. 3.2.2, Figs. 3-4): coarse centred values in the
 * region covered by the fine level are replaced by the mean of their 8 fine
 * cells, coarse face velocities by the mean of the 4 coincident fine faces
 * (including the faces on the frontier).  The whole covered box is
 * overwritten (the paper overwrites 4 layers on the contour; the values this
 * leaves on uncovered cells are the same whenever 4 layers suffice).
 * Pinned by: restriction of a prolongation, composite mass conservation,
 * exactness on uniform data. */
static void commmean(run_t *R, int lc) {
  lev_t *C = &R->lev[lc], *F = &R->lev[lc + 1];
  int o[3], h[3];
  cov_box(R, lc, o, h);
  for (int fld = 0; fld < NSTATE; ++fld) {
    int stag = (fld >= S_VX) ? fld - S_VX : -1;
    const double *Q = F->st[fld];
    double *out = C->st[fld];
    int hk = h[2] + (stag == 2), hj = h[1] + (stag == 1), hi = h[0] + (stag == 0);
#pragma omp parallel for schedule(static)
    for (int K = 0; K < hk; ++K)
      for (int J = 0; J < hj; ++J)
        for (int I = 0; I < hi; ++I) {
          int fi = 2 * I, fj = 2 * J, fk = 2 * K;
          double val;
          if (stag < 0) {
            double c000 = Q[IX(F, fi, fj, fk)], c100 = Q[IX(F, fi + 1, fj, fk)];
            double c010 = Q[IX(F, fi, fj + 1, fk)], c110 = Q[IX(F, fi + 1, fj + 1, fk)];
            double c001 = Q[IX(F, fi, fj, fk + 1)], c101 = Q[IX(F, fi + 1, fj, fk + 1)];
            double c011 = Q[IX(F, fi, fj + 1, fk + 1)], c111 = Q[IX(F, fi + 1, fj + 1, fk + 1)];
            val = (((c000 + c100) + (c010 + c110)) + ((c001 + c101) + (c011 + c111))) * 0.125;
          } else {
            int e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
            int t1, t2;
            tdims(stag, &t1, &t2);
            e1[t1] = 1; e2[t2] = 1;
            double f00 = Q[IX(F, fi, fj, fk)];
            double f10 = Q[IX(F, fi + e1[0], fj + e1[1], fk + e1[2])];
            double f01 = Q[IX(F, fi + e2[0], fj + e2[1], fk + e2[2])];
            double f11 = Q[IX(F, fi + e1[0] + e2[0], fj + e1[1] + e2[1], fk + e1[2] + e2[2])];
            val = ((f00 + f10) + (f01 + f11)) * 0.25;
          }
          out[IX(C, o[0] + I, o[1] + J, o[2] + K)] = val;
        }
  }
  if ((R->anch[1] || R->anch[2]) && lc > 0) mirror_fill(R, lc);
}

/* ---------------------------------------------------------------- cycle */
/* Recursive sub-cycling (Sect. 3.1, 3.3): two steps of dt/2 on level l+1 per
 * step dt on level l, the finer level first; then CommUp and CommMean in the
 * order of the staging list.  The frontier accumulators of level l+1 are
 * cleared before its two sub-cycles. */
static void cycle(run_t *R, int lvl, double dt) {
  if (lvl < R->nl - 1) {
    lev_t *F = &R->lev[lvl + 1];
    for (int d = 0; d < 3; ++d) {
      int t1, t2;
      tdims(d, &t1, &t2);
      size_t na = (size_t)F->n[t1] * F->n[t2];
      for (int side = 0; side < 2; ++side)
        for (int iq = 0; iq < NQ; ++iq) memset(F->acc[d][side][iq], 0, na * sizeof(double));
    }
    /* xi sub-steps of the finer level, each of dt / xi */
    for (int sub = 0; sub < R->xi[lvl]; ++sub) cycle(R, lvl + 1, R->xi[lvl] == 2 ? 0.5 * dt : dt);
  }
  hydro_step(R, lvl, dt);
  if (lvl < R->nl - 1) {
    commup(R, lvl);
    commmean(R, lvl);
  }
}

/* ------------------------------------------------------------- time step */
/* Time-step limit of each level: the Courant limit dx / max(c_s + |v|) over
 * the active cells and their face velocities, c_s = sqrt(gamma (gamma-1) e/rho),
 * and (reading: the paper does not state it) the explicit-diffusion limit
 * dx^2 / (6 chi), times the Courant factor: dtl[l] = cfl * min(...). */
static void level_limits(run_t *R, double *dtl) {
  double gg = R->p.gamma * (R->p.gamma - 1.0);
  for (int l = 0; l < R->nl; ++l) {
    lev_t *L = &R->lev[l];
    const double *rho = L->st[S_RHO], *e = L->st[S_E];
    double smax = 0.0;
    for (int k = 0; k < L->n[2]; ++k)
      for (int j = 0; j < L->n[1]; ++j)
        for (int i = 0; i < L->n[0]; ++i) {
          size_t c = IX(L, i, j, k);
          double cs = sqrt(gg * e[c] / rho[c]);
          for (int d = 0; d < 3; ++d) {
            const double *v = L->st[S_VX + d];
            double a = fabs(v[c]), b = fabs(v[c + STR(L, d)]);
            double sig = cs + (a > b ? a : b);
            if (sig > smax) smax = sig;
          }
        }
    double dt = L->dx / smax;
    if (R->p.chi > 0.0) {
      double dd = L->dx * L->dx / (6.0 * R->p.chi);
      if (dd < dt) dt = dd;
    }
    dtl[l] = R->p.cfl * dt;
  }
}

/* Coarse step of a schedule xi (eq. 55): min over levels of dtl[l] times the
 * product of xi[m] for m < l. */
static double schedule_dt(int nl, const double *dtl, const int *xi) {
  double best = INFINITY, prod = 1.0;
  for (int l = 0; l < nl; ++l) {
    double v = dtl[l] * prod;
    if (v < best) best = v;
    if (l < nl - 1) prod *= (double)xi[l];
  }
  return best;
}

/* Sub-cycling criterion of App. A: among the 2^(n-1) words xi in {1,2}^(n-1)
 * the one of largest coarse step (eq. 55) per cost (eq. 56, the cost of a level
 * step taken as its active cell count); words are tried from all-2 downwards
 * (xi[m] = 2 where bit m of the word is set) and a later word must do strictly
 * better, so ties keep the most sub-cycling.  Without the criterion xi = 2. */
static void choose_schedule(int nl, const double *dtl, const double *cost, int use_criterion, int *xi) {
  for (int m = 0; m < nl - 1; ++m) xi[m] = 2;
  if (!use_criterion || nl < 2) return;
  double best = -1.0;
  int cand[DFO_MAXLEV];
  for (long w = (1L << (nl - 1)) - 1; w >= 0; --w) {
    for (int m = 0; m < nl - 1; ++m) cand[m] = (w >> m) & 1 ? 2 : 1;
    double c = 0.0, prod = 1.0;
    for (int l = 0; l < nl; ++l) {
      c += cost[l] * prod;
      if (l < nl - 1) prod *= (double)cand[l];
    }
    double r = schedule_dt(nl, dtl, cand) / c;
    if (r > best) {
      best = r;
      for (int m = 0; m < nl - 1; ++m) xi[m] = cand[m];
    }
  }
}

/* Coarse step of the current state; sets R->xi. */
static double dt_rule(run_t *R) {
  double dtl[DFO_MAXLEV], cost[DFO_MAXLEV];
  level_limits(R, dtl);
  for (int l = 0; l < R->nl; ++l) cost[l] = (double)R->lev[l].n[0] * R->lev[l].n[1] * R->lev[l].n[2];
  choose_schedule(R->nl, dtl, cost, R->p.subcycle, R->xi);
  return schedule_dt(R->nl, dtl, R->xi);
}

/* ---------------------------------------------------------------- force */
/* Gravitational force of the gas on the perturber, eq. 18 (and eq. 4): sum
 * over cells of G M rho dV r / (r^2 + eps^2)^{3/2}, level by level, skipping
 * coarse cells covered by a finer level.  The uniform background contributes
 * exactly zero by the symmetry of the cell centres about the perturber, so the
 * sum is taken over (rho - rho0) to avoid cancellation.  Neumaier-compensated
 * sums per k-plane, then over planes in order.
 * Pinned by: zero for uniform data, mirror-odd components vanish, cold drag
 * negative and proportional to GM^2 at small GM, Newton's shell theorem (a
 * Gaussian over-density pulls as its mass at its centre: to round-off on one
 * level, at second order in the cell size across a frontier, which fixes the
 * covered cells) and the softened point mass of a single cell. */
typedef struct { double s, c; } nsum_t;
static inline void nadd(nsum_t *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}

static int covered(const run_t *R, int l, int i, int j, int k) {
  if (l >= R->nl - 1) return 0;
  int id[3] = {i, j, k}, o[3], h[3];
  cov_box(R, l, o, h);
  for (int d = 0; d < 3; ++d)
    if (id[d] < o[d] || id[d] >= o[d] + h[d]) return 0;
  return 1;
}

static void force(run_t *R, double out[3]) {
  nsum_t tot[3] = {{0, 0}, {0, 0}, {0, 0}};
  double eps2 = R->p.eps * R->p.eps;
  for (int l = 0; l < R->nl; ++l) {
    lev_t *L = &R->lev[l];
    double vol = L->dx * L->dx * L->dx;
    for (int k = 0; k < L->n[2]; ++k) {
      nsum_t pl[3] = {{0, 0}, {0, 0}, {0, 0}};
      for (int j = 0; j < L->n[1]; ++j)
        for (int i = 0; i < L->n[0]; ++i) {
          if (covered(R, l, i, j, k)) continue;
          double x = XC(L, 0, i), y = XC(L, 1, j), z = XC(L, 2, k);
          double d2 = x * x + y * y + z * z + eps2;
          double w = R->p.GM * (L->st[S_RHO][IX(L, i, j, k)] - R->p.rho0) * vol / (d2 * sqrt(d2));
          nadd(&pl[0], w * x);
          nadd(&pl[1], w * y);
          nadd(&pl[2], w * z);
        }
      for (int d = 0; d < 3; ++d) nadd(&tot[d], pl[d].s + pl[d].c);
    }
  }
  /* quadrant: the force of the whole gas, the domain's mirror images
   * included (they cancel the components normal to the mirror planes) */
  for (int d = 0; d < 3; ++d) out[d] = R->anch[d] ? 0.0 : R->mult * (tot[d].s + tot[d].c);
}

/* composite totals over uncovered active cells: mass, internal energy,
 * kinetic energy (face velocities averaged to centres), net inflow of mass
 * through the level-0 boundary since the start */
static void totals(run_t *R, double out[4]) {
  nsum_t m = {0, 0}, ei = {0, 0}, ek = {0, 0};
  for (int l = 0; l < R->nl; ++l) {
    lev_t *L = &R->lev[l];
    double vol = L->dx * L->dx * L->dx;
    for (int k = 0; k < L->n[2]; ++k)
      for (int j = 0; j < L->n[1]; ++j)
        for (int i = 0; i < L->n[0]; ++i) {
          if (covered(R, l, i, j, k)) continue;
          size_t c = IX(L, i, j, k);
          double r = L->st[S_RHO][c];
          double v2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            double vc = 0.5 * (L->st[S_VX + d][c] + L->st[S_VX + d][c + STR(L, d)]);
            v2 += vc * vc;
          }
          nadd(&m, r * vol);
          nadd(&ei, L->st[S_E][c] * vol);
          nadd(&ek, 0.5 * r * v2 * vol);
        }
  }
  /* quadrant: the whole gas (the domain and its mirror images) */
  out[0] = R->mult * (m.s + m.c);
  out[1] = R->mult * (ei.s + ei.c);
  out[2] = R->mult * (ek.s + ek.c);
  out[3] = R->mult * R->bflux;
}

/* ---------------------------------------------------------- initial state */
/* SplitMix64 (Steele, Lea & Flood 2014, "Fast splittable pseudorandom number
 * generators") used as a counter-based generator: output n of the stream with
 * seed s is the SplitMix64 finaliser applied to s + (n+1) * golden gamma. */
static uint64_t smix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
static double uniform01(uint64_t seed, uint64_t n) {
  uint64_t z = smix(seed + (n + 1ULL) * 0x9e3779b97f4a7c15ULL);
  return (double)(z >> 11) * 0x1.0p-53;
}

static void restrict_prolong_all(run_t *R) {
  for (int l = R->nl - 2; l >= 0; --l) commmean(R, l);
  bc_state(R);
  for (int l = 0; l < R->nl - 1; ++l) commup(R, l);
}

/* Initial state (Sect. 3.4): rho0, e0 = rho0 c_s^2 / (gamma (gamma-1)), the
 * uniform wind (-V, 0, 0) everywhere; the density of every active cell of
 * level l and active index a = i + nx (j + ny k) is multiplied by
 * 1 + A (2U - 1), U the uniform number number l 2^40 + a of the stream. */
static void init_state(run_t *R) {
  for (int l = 0; l < R->nl; ++l) {
    lev_t *L = &R->lev[l];
    for (size_t c = 0; c < L->vol; ++c) {
      L->st[S_RHO][c] = R->p.rho0;
      L->st[S_E][c] = R->e0;
      L->st[S_VX][c] = -R->V;
      L->st[S_VY][c] = 0.0;
      L->st[S_VZ][c] = 0.0;
    }
    if (R->p.noise_amp != 0.0)
      for (int k = 0; k < L->n[2]; ++k)
        for (int j = 0; j < L->n[1]; ++j)
          for (int i = 0; i < L->n[0]; ++i) {
            uint64_t a = ((uint64_t)k * (uint64_t)L->n[1] + (uint64_t)j) * (uint64_t)L->n[0] + (uint64_t)i;
            double U = uniform01(R->p.seed, ((uint64_t)l << 40) + a);
            L->st[S_RHO][IX(L, i, j, k)] = R->p.rho0 * (1.0 + R->p.noise_amp * (2.0 * U - 1.0));
          }
  }
  restrict_prolong_all(R);
}

static void cov_box(const run_t *R, int lc, int o[3], int h[3]) {
  const lev_t *C = &R->lev[lc], *F = &R->lev[lc + 1];
  for (int d = 0; d < 3; ++d) {
    h[d] = F->n[d] / 2;
    o[d] = R->anch[d] ? 0 : (C->n[d] - h[d]) / 2;  /* quadrant: from the mirror plane */
  }
}

/* ============================================================== C API */

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

void dfo_destroy(void *h);

void *dfo_create(const dfo_params *p) {
  if (p->nlevels < 1 || p->nlevels > DFO_MAXLEV) return NULL;
  if (p->nx1 > 0) {
    /* finer levels: even halves that fit inside level 0 around its centre */
    const int n0[3] = {p->nx, p->ny, p->nz}, n1[3] = {p->nx1, p->ny1, p->nz1};
    for (int d = 0; d < 3; ++d)
      if (n1[d] % 4 || n1[d] / 2 > n0[d] || (n0[d] - n1[d] / 2) % 2) return NULL;
  }
  run_t *R = (run_t *)calloc(1, sizeof(run_t));
  R->p = *p;
  R->nl = p->nlevels;
  for (int m = 0; m < DFO_MAXLEV; ++m) R->xi[m] = 2;
  R->V = p->mach * p->cs;
  R->e0 = p->rho0 * p->cs * p->cs / (p->gamma * (p->gamma - 1.0));
  /* quadrant: y and z start at the perturber's mirror planes (the paper's
   * x, y > 0 with its flow along z is here y, z > 0 with the flow along x);
   * its boundaries are those of the boundary list */
  if (p->quadrant && p->bcmode != 1) { free(R); return NULL; }
  R->anch[0] = 0;
  R->anch[1] = R->anch[2] = p->quadrant ? 1 : 0;
  R->mult = p->quadrant ? 4.0 : 1.0;
  for (int l = 0; l < R->nl; ++l) {
    lev_t *L = &R->lev[l];
    L->n[0] = p->nx; L->n[1] = p->ny; L->n[2] = p->nz;
    if (l > 0 && p->nx1 > 0) { L->n[0] = p->nx1; L->n[1] = p->ny1; L->n[2] = p->nz1; }
    L->g = (l == 0) ? p->g0 : p->gf;
    for (int d = 0; d < 3; ++d) L->org[d] = R->anch[d] ? 0.0 : 0.5 * (double)L->n[d];
    L->vol = 1;
    for (int d = 0; d < 3; ++d) { L->s[d] = L->n[d] + 2 * L->g; L->vol *= (size_t)L->s[d]; }
    L->dx = p->dx0 / (double)(1L << l);
    for (int f = 0; f < NSTATE; ++f) L->st[f] = zalloc(L->vol);
    for (int q = 0; q < NQ; ++q) {
      L->q[q] = zalloc(L->vol); L->qn[q] = zalloc(L->vol);
      L->fl[q] = zalloc(L->vol); L->sp[q] = zalloc(L->vol);
    }
    L->tmp = zalloc(L->vol);
    for (int d = 0; d < 3; ++d) {
      int t1, t2;
      tdims(d, &t1, &t2);
      for (int side = 0; side < 2; ++side)
        for (int q = 0; q < NQ; ++q) L->acc[d][side][q] = zalloc((size_t)L->n[t1] * L->n[t2]);
    }
    L->hw = zalloc((size_t)L->n[0] * L->n[1] * L->n[2]);
    heat_weights(R, l);
  }
  init_state(R);
  return R;
}

void dfo_destroy(void *h) {
  run_t *R = (run_t *)h;
  if (!R) return;
  for (int l = 0; l < R->nl; ++l) {
    lev_t *L = &R->lev[l];
    for (int f = 0; f < NSTATE; ++f) free(L->st[f]);
    for (int q = 0; q < NQ; ++q) { free(L->q[q]); free(L->qn[q]); free(L->fl[q]); free(L->sp[q]); }
    free(L->tmp);
    for (int d = 0; d < 3; ++d)
      for (int side = 0; side < 2; ++side)
        for (int q = 0; q < NQ; ++q) free(L->acc[d][side][q]);
    free(L->hw);
  }
  free(R);
}

/* one coarse step: time-step rule, recursive cycle from level 0 */
void dfo_step(void *h, int n) {
  run_t *R = (run_t *)h;
  for (int s = 0; s < n; ++s) {
    double dt = dt_rule(R);
    cycle(R, 0, dt);
    R->t += dt;
    R->dt_last = dt;
    R->nsteps++;
  }
}

double dfo_time(void *h) { return ((run_t *)h)->t; }
double dfo_dt(void *h) { return dt_rule((run_t *)h); }

/* sub-steps per level of the last coarse step (nl-1 entries) */
void dfo_schedule(void *h, int *xi) {
  run_t *R = (run_t *)h;
  for (int m = 0; m < R->nl - 1; ++m) xi[m] = R->xi[m];
}

/* the criterion alone, for given per-level limits and costs (tests) */
void dfo_choose_schedule(int nl, const double *dtl, const double *cost, int use_criterion, int *xi) {
  choose_schedule(nl, dtl, cost, use_criterion, xi);
}

/* OpenMP threads of the cell loops (timing only; results do not depend on it) */
void dfo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
void dfo_force(void *h, double out[3]) { force((run_t *)h, out); }
void dfo_totals(void *h, double out[4]) { totals((run_t *)h, out); }

/* copy one field of one level: whole allocated array (ghosts=1) or the active
 * entries (cells 0..n-1; a face field's own axis is 0..n-1 too), x fastest */
static int field_ok(run_t *R, int l, int f) { return l >= 0 && l < R->nl && f >= 0 && f < NSTATE; }

int dfo_get_field(void *h, int l, int f, double *out, int ghosts) {
  run_t *R = (run_t *)h;
  if (!field_ok(R, l, f)) return -1;
  lev_t *L = &R->lev[l];
  if (ghosts) { memcpy(out, L->st[f], L->vol * sizeof(double)); return 0; }
  size_t a = 0;
  for (int k = 0; k < L->n[2]; ++k)
    for (int j = 0; j < L->n[1]; ++j)
      for (int i = 0; i < L->n[0]; ++i) out[a++] = L->st[f][IX(L, i, j, k)];
  return 0;
}

int dfo_set_field(void *h, int l, int f, const double *in, int ghosts) {
  run_t *R = (run_t *)h;
  if (!field_ok(R, l, f)) return -1;
  lev_t *L = &R->lev[l];
  if (ghosts) { memcpy(L->st[f], in, L->vol * sizeof(double)); return 0; }
  size_t a = 0;
  for (int k = 0; k < L->n[2]; ++k)
    for (int j = 0; j < L->n[1]; ++j)
      for (int i = 0; i < L->n[0]; ++i) L->st[f][IX(L, i, j, k)] = in[a++];
  return 0;
}

/* face field entry n along its own axis (the last active face) */
int dfo_get_lastface(void *h, int l, int f, double *out) {
  run_t *R = (run_t *)h;
  if (!field_ok(R, l, f) || f < S_VX) return -1;
  lev_t *L = &R->lev[l];
  int dn = f - S_VX, t1, t2;
  tdims(dn, &t1, &t2);
  size_t a = 0;
  for (int b2 = 0; b2 < L->n[t2]; ++b2)
    for (int b1 = 0; b1 < L->n[t1]; ++b1) {
      int id[3];
      id[dn] = L->n[dn]; id[t1] = b1; id[t2] = b2;
      out[a++] = L->st[f][IX(L, id[0], id[1], id[2])];
    }
  return 0;
}

int dfo_set_lastface(void *h, int l, int f, const double *in) {
  run_t *R = (run_t *)h;
  if (!field_ok(R, l, f) || f < S_VX) return -1;
  lev_t *L = &R->lev[l];
  int dn = f - S_VX, t1, t2;
  tdims(dn, &t1, &t2);
  size_t a = 0;
  for (int b2 = 0; b2 < L->n[t2]; ++b2)
    for (int b1 = 0; b1 < L->n[t1]; ++b1) {
      int id[3];
      id[dn] = L->n[dn]; id[t1] = b1; id[t2] = b2;
      L->st[f][IX(L, id[0], id[1], id[2])] = in[a++];
    }
  return 0;
}

/* make the hierarchy consistent after fields were set: restrict every level
 * onto its parent (finest first), refill level-0 ghosts, prolong ghosts */
void dfo_sync(void *h) { restrict_prolong_all((run_t *)h); }
void dfo_commup(void *h, int lc) { commup((run_t *)h, lc); }
/* test helper: interpolate every entry of level lc+1 (active ones too) */
void dfo_prolong_all(void *h, int lc) {
  run_t *R = (run_t *)h;
  commup_fill(R, lc, 1);
  if (R->anch[1] || R->anch[2]) mirror_fill(R, lc + 1);
}
void dfo_commmean(void *h, int lc) { commmean((run_t *)h, lc); }

/* single-level stage harness (level 0), with the boundary fills the step
 * performs before each stage:
 *   1 kick(dt)  2 compression(dt)  3 diffusion(dt)  4 heat(dt)
 *   5 transport(dt)  6 compression+diffusion+heat(dt)  7 full level step(dt) */
int dfo_stage(void *h, int stage, double dt) {
  run_t *R = (run_t *)h;
  switch (stage) {
    case 1: bc_state(R); kick(R, 0, dt); break;
    case 2: bc_state(R); compress(R, 0, dt); break;
    case 3: bc_state(R); diffuse(R, 0, dt); break;
    case 4: heat(R, 0, dt); break;
    case 5: bc_state(R); transport(R, 0, dt); break;
    case 6: bc_state(R); compress(R, 0, dt); bc_state(R); diffuse(R, 0, dt); heat(R, 0, dt); break;
    case 7: if (R->nl != 1) return -1; hydro_step(R, 0, dt); R->t += dt; break;
    case 8: bc_state(R); viscosity(R, 0, dt); break;
    default: return -1;
  }
  bc_state(R);
  return 0;
}

/* the heat-release weights of one level (active cells, x fastest) */
int dfo_heat_weights(void *h, int l, double *out) {
  run_t *R = (run_t *)h;
  if (l < 0 || l >= R->nl) return -1;
  lev_t *L = &R->lev[l];
  memcpy(out, L->hw, (size_t)L->n[0] * L->n[1] * L->n[2] * sizeof(double));
  return 0;
}
