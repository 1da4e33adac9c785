// dfk.hip -- gfx950 kernels of libdfmesh (FP64 storage).
//
// The update of one level over a step dt follows the staging list of Velasco
// Romero & Masset (2018), Sect. 3.3, with the split source step of eq. 15:
//   kick(dt/2) -> compression, diffusion, heat release (dt) -> transport (dt)
//   -> kick(dt/2)
// Every kernel is a coalesced sweep over x-fastest arrays: blocks of 64 x 4
// threads cover 64 consecutive x entries of 4 rows; the grid's z dimension
// walks planes.  Level 0 reads its outer boundary conditions on the fly
// (clamped indices, inflow constants at x_max), so it stores no ghost data;
// finer levels advance their whole ghost shell, filled once per parent step.
#include "dfk.h"

namespace dfk {

namespace {

constexpr int BX = 64, BY = 4;

struct Box {
  int lo[3], hi[3];
};

inline bool empty_grid(const dim3 &g) { return g.x == 0; }

// Kernels over a box launch a 1-D grid of tiles of 64 x 4 entries (x fastest)
// times one plane.  The hardware hands workgroups to the 8 XCDs round-robin
// (workgroup h runs on XCD h % 8); thread_cell gives each XCD one contiguous
// range of tiles: a band of rows through all planes, walked plane by plane
// (x-tile fastest, then y-tile within the band, then plane), so the neighbour
// planes a stencil reads are in its own L2 (a few planes of one band fit
// there) and neighbour rows are too except at band edges.
inline dim3 grid_of(const Box &b) {
  int ex = b.hi[0] - b.lo[0], ey = b.hi[1] - b.lo[1], ez = b.hi[2] - b.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return dim3(0, 1, 1);
  long n = (long)((ex + BX - 1) / BX) * ((ey + BY - 1) / BY) * ez;
  return dim3((unsigned)n, 1, 1);
}

__device__ __forceinline__ bool thread_cell(const Box &b, int &i, int &j, int &k) {
  const unsigned nbx = (unsigned)(b.hi[0] - b.lo[0] + BX - 1) / BX;
  const unsigned nby = (unsigned)(b.hi[1] - b.lo[1] + BY - 1) / BY;
  const unsigned N = gridDim.x, h = blockIdx.x;
  const unsigned nbz = N / (nbx * nby);
  // contiguous tile range of this workgroup's XCD
  const unsigned q = N / 8, r = N % 8, x = h % 8, s = h / 8;
  unsigned L = (x < r) ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
  // 8 bands of y-tiles (sizes differ by at most one); a band's tiles are
  // ordered x-tile fastest, then y-tile, then plane
  const unsigned hq = nby / 8, hr = nby % 8;
  unsigned band = 0, y0 = 0, hb = hq + (hr > 0);
  for (unsigned bb = 0; bb < 8; ++bb) {
    hb = hq + (bb < hr ? 1u : 0u);
    unsigned nt = nbx * hb * nbz;
    if (L < nt || bb == 7) {
      band = bb;
      break;
    }
    L -= nt;
    y0 += hb;
  }
  (void)band;
  const unsigned bx = L % nbx, t = L / nbx;
  const unsigned by = y0 + t % hb, bz = t / hb;
  i = b.lo[0] + (int)(bx * BX + threadIdx.x);
  j = b.lo[1] + (int)(by * BY + threadIdx.y);
  k = b.lo[2] + (int)bz;
  return i < b.hi[0] && j < b.hi[1];
}

__device__ __forceinline__ long lin(const Geo &G, int i, int j, int k) {
  return G.off + i + (long)j * G.sy + (long)k * G.sz;
}

__device__ __forceinline__ long dstride(const Geo &G, int d) {
  return d == 0 ? 1L : (d == 1 ? G.sy : G.sz);
}

// cell-centre coordinate: the perturber is the central vertex of the level
__device__ __forceinline__ double xcen(const Geo &G, int d, int i) {
  return ((double)i - 0.5 * (double)G.n[d] + 0.5) * G.dx;
}

// Plummer potential -GM / sqrt(r^2 + eps^2) at a cell centre (eq. 16)
__device__ __forceinline__ double phi_at(const Geo &G, const Phys &P, int i, int j, int k) {
  double x = xcen(G, 0, i), y = xcen(G, 1, j), z = xcen(G, 2, k);
  return -P.GM / sqrt(x * x + y * y + z * z + P.eps2);
}

// van Leer's harmonic limited difference
__device__ __forceinline__ double vleer(double a, double b) {
  return (a * b > 0.0) ? 2.0 * a * b / (a + b) : 0.0;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Level-0 centred read with the outer boundary conditions: inflow state
// beyond x_max, zero-gradient copy of the nearest active cell elsewhere.
__device__ __forceinline__ double cread(const double *q, const Geo &G, int i, int j, int k, double qin) {
  if (i >= G.n[0]) return qin;
  i = i < 0 ? 0 : i;
  j = clampi(j, 0, G.n[1] - 1);
  k = clampi(k, 0, G.n[2] - 1);
  return q[lin(G, i, j, k)];
}

// Level-0 read of the velocity normal to faces of dimension d (active faces
// 0..n along d): the wind -V (x) or 0 (y, z) beyond x_max, copies elsewhere.
__device__ __forceinline__ double fread_bc(const double *v, const Geo &G, int d, int i, int j, int k,
                                           double V) {
  if (d == 0) {
    if (i > G.n[0]) return -V;
    i = i < 0 ? 0 : i;
  } else {
    if (i >= G.n[0]) return 0.0;
    i = i < 0 ? 0 : i;
  }
  j = clampi(j, 0, G.n[1] - (d == 1 ? 0 : 1));
  k = clampi(k, 0, G.n[2] - (d == 2 ? 0 : 1));
  return v[lin(G, i, j, k)];
}

__device__ __forceinline__ double q_inflow(const Phys &P, int m) {
  return m == 0 ? P.rho0 : (m == 1 ? P.e0 : ((m == 2 || m == 3) ? P.rho0 * (-P.V) : 0.0));
}

// ------------------------------------------------------------------ init

// SplitMix64 finaliser (Steele, Lea & Flood 2014); output n of the stream
// with seed s is mix(s + (n+1) * 0x9e3779b97f4a7c15).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

struct InitArgs {
  Box b;
  double *rho, *e, *vx, *vy, *vz;
  uint64_t seed;
  double amp;
};

__global__ void __launch_bounds__(BX * BY) k_init(Geo G, Phys P, InitArgs A) {
  int i, j, k;
  if (!thread_cell(A.b, i, j, k)) return;
  long c = lin(G, i, j, k);
  double r = P.rho0;
  bool active = i >= 0 && j >= 0 && k >= 0 && i < G.n[0] && j < G.n[1] && k < G.n[2];
  if (active && A.amp != 0.0) {
    uint64_t a = ((uint64_t)k * (uint64_t)G.n[1] + (uint64_t)j) * (uint64_t)G.n[0] + (uint64_t)i;
    uint64_t n = ((uint64_t)G.level << 40) + a;
    uint64_t z = mix64(A.seed + (n + 1ULL) * 0x9e3779b97f4a7c15ULL);
    double U = (double)(z >> 11) * 0x1.0p-53;
    r = P.rho0 * (1.0 + A.amp * (2.0 * U - 1.0));
  }
  A.rho[c] = r;
  A.e[c] = P.e0;
  A.vx[c] = -P.V;
  A.vy[c] = 0.0;
  A.vz[c] = 0.0;
}

// ------------------------------------------------------------------ kick

struct KickArgs {
  Box b;                 // union of the three face ranges
  int flo[3][3], fhi[3][3];  // [normal dir][dim] face ranges
  const double *q[NQ];   // rho, e (and the momenta when rebuilding)
  double *v[3];
  const double *dtp;
  double fac;
};

// Velocity source S(h) (eq. 15): each face velocity receives
// -h [ (gamma-1)(e_c - e_m) / (dx rho_face) + (Phi_c - Phi_m) / dx ].
// REBUILD first sets the face velocity from the transported momenta,
// (P+_m + P-_c) / (rho_m + rho_c).  KICK = false skips the source.
template <bool BC, bool REBUILD, bool KICK>
__global__ void __launch_bounds__(BX * BY) k_kick(Geo G, Phys P, KickArgs A) {
  int i, j, k;
  if (!thread_cell(A.b, i, j, k)) return;
  const double h = A.fac * A.dtp[0];
  const double *rho = A.q[0], *e = A.q[1];
  long c = lin(G, i, j, k);
  double rc = 0.0, ec = 0.0, phic = 0.0;
  bool need_c = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    bool in = i >= A.flo[d][0] && i < A.fhi[d][0] && j >= A.flo[d][1] && j < A.fhi[d][1] &&
              k >= A.flo[d][2] && k < A.fhi[d][2];
    need_c |= in;
  }
  if (!need_c) return;
  if (BC) {
    rc = cread(rho, G, i, j, k, P.rho0);
    ec = cread(e, G, i, j, k, P.e0);
  } else {
    rc = rho[c];
    ec = e[c];
  }
  if (KICK) phic = phi_at(G, P, i, j, k);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    bool in = i >= A.flo[d][0] && i < A.fhi[d][0] && j >= A.flo[d][1] && j < A.fhi[d][1] &&
              k >= A.flo[d][2] && k < A.fhi[d][2];
    if (!in) continue;
    int im = i - (d == 0), jm = j - (d == 1), km = k - (d == 2);
    long m = c - dstride(G, d);
    double rm, em;
    if (BC) {
      rm = cread(rho, G, im, jm, km, P.rho0);
      em = cread(e, G, im, jm, km, P.e0);
    } else {
      rm = rho[m];
      em = e[m];
    }
    double vf;
    if (REBUILD) {
      const double *pm = A.q[2 + 2 * d], *pp = A.q[3 + 2 * d];
      double ppm, pmc;
      if (BC) {
        ppm = cread(pp, G, im, jm, km, q_inflow(P, 3 + 2 * d));
        pmc = cread(pm, G, i, j, k, q_inflow(P, 2 + 2 * d));
      } else {
        ppm = pp[m];
        pmc = pm[c];
      }
      vf = (ppm + pmc) / (rm + rc);
    } else {
      vf = A.v[d][c];
    }
    if (KICK) {
      double rface = 0.5 * (rm + rc);
      double gradp = P.gm1 * (ec - em) / (G.dx * rface);
      double gradphi = (phic - phi_at(G, P, im, jm, km)) / G.dx;
      vf = vf - h * (gradp + gradphi);
    }
    if (BC && d == 0 && i == G.n[0]) vf = -P.V;  // injection face at x_max
    A.v[d][c] = vf;
  }
}

// ------------------------------------------------------------ compression

struct CellArgs {
  Box b;
  const double *rho;
  double *e;
  const double *v[3];
  const double *dtp;
  double fac;
};

// Compressional heating (SubStep3): e <- e (1 - a) / (1 + a),
// a = (gamma - 1) dt div(v) / 2, from the cell's six face velocities.
__global__ void __launch_bounds__(BX * BY) k_compress(Geo G, Phys P, CellArgs A) {
  int i, j, k;
  if (!thread_cell(A.b, i, j, k)) return;
  const double dt = A.fac * A.dtp[0];
  long c = lin(G, i, j, k);
  double divv = ((A.v[0][c + 1] - A.v[0][c]) + (A.v[1][c + G.sy] - A.v[1][c]) +
                 (A.v[2][c + G.sz] - A.v[2][c])) / G.dx;
  double a = 0.5 * P.gm1 * dt * divv;
  A.e[c] = A.e[c] * (1.0 - a) / (1.0 + a);
}

// ---------------------------------------------------- diffusion + heat

struct DiffArgs {
  Box b;
  const double *rho, *e;
  double *eo;
  const double *hw;
  int hw_n[3], hw_lo[3];  // weight box extent and its first active index per dimension
  const double *dtp;
  double fac;
  int do_diff, do_heat;
};

// Thermal diffusion (eqs. 19-22, energy flux down the gradient of e/rho with
// coefficient chi rho0) and heat release L dt w_c / dx^3 (Sect. 3.4).
template <bool BC>
__global__ void __launch_bounds__(BX * BY) k_diffuse_heat(Geo G, Phys P, DiffArgs A) {
  int i, j, k;
  if (!thread_cell(A.b, i, j, k)) return;
  const double dt = A.fac * A.dtp[0];
  long c = lin(G, i, j, k);
  double ec = A.e[c];
  double en = ec;
  if (A.do_diff) {
    double Tc = ec / A.rho[c];
    double lap = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double Tm, Tp;
      if (BC) {
        int im = i - (d == 0), jm = j - (d == 1), km = k - (d == 2);
        int ip = i + (d == 0), jp = j + (d == 1), kp = k + (d == 2);
        Tm = cread(A.e, G, im, jm, km, P.e0) / cread(A.rho, G, im, jm, km, P.rho0);
        Tp = cread(A.e, G, ip, jp, kp, P.e0) / cread(A.rho, G, ip, jp, kp, P.rho0);
      } else {
        long s = dstride(G, d);
        Tm = A.e[c - s] / A.rho[c - s];
        Tp = A.e[c + s] / A.rho[c + s];
      }
      lap += (Tp - Tc) - (Tc - Tm);
    }
    en = ec + dt * (P.chi * P.rho0) * lap / (G.dx * G.dx);
  }
  if (A.do_heat && A.hw_n[0] > 0) {
    int a = i - A.hw_lo[0], b = j - A.hw_lo[1], d = k - A.hw_lo[2];
    if (a >= 0 && b >= 0 && d >= 0 && a < A.hw_n[0] && b < A.hw_n[1] && d < A.hw_n[2] &&
        i >= 0 && j >= 0 && k >= 0 && i < G.n[0] && j < G.n[1] && k < G.n[2]) {
      double w = A.hw[((long)d * A.hw_n[1] + b) * A.hw_n[0] + a];
      if (w != 0.0) en += P.L * dt * w / (G.dx * G.dx * G.dx);
    }
  }
  A.eo[c] = en;
}

// -------------------------------------------------------------- transport

struct PassArgs {
  Box b;
  const double *qi[NQ];
  double *qo[NQ];
  const double *v[3];     // face velocities after the first kick
  const double *dtp;
  double fac;
  double *acc;            // this level's frontier accumulators (fine levels) or null
  const double *facc;     // the finer level's accumulators (coarse levels) or null
  int fn[3];              // finer level's active cells (for accumulator strides)
};

// Offsets of the cell at o along DIR from (i,j,k) for level 0, with the
// boundary conditions: returns false for an inflow ghost (beyond x_max).
template <int DIR, bool BC>
__device__ __forceinline__ bool cell_at(const Geo &G, int i, int j, int k, int o, long &c) {
  int ii = i + (DIR == 0 ? o : 0), jj = j + (DIR == 1 ? o : 0), kk = k + (DIR == 2 ? o : 0);
  if (BC) {
    if (ii >= G.n[0]) return false;
    ii = ii < 0 ? 0 : ii;
    jj = clampi(jj, 0, G.n[1] - 1);
    kk = clampi(kk, 0, G.n[2] - 1);
  }
  c = lin(G, ii, jj, kk);
  return true;
}

// upwind van Leer face value from the specific values s[0..3] of the cells
// -2..+1 around the face (offsets relative to the face's high-side cell)
__device__ __forceinline__ double face_value(double sm2, double sm1, double s0, double sp1, double a,
                                             double nu) {
  if (a > 0.0) return sm1 + 0.5 * vleer(s0 - sm1, sm1 - sm2) * (1.0 - nu);
  return s0 - 0.5 * vleer(sp1 - s0, s0 - sm1) * (1.0 + nu);
}

// One dimensional pass of the van Leer upwind transport along DIR for the cell
// (i,j,k): transfers through its two faces, M = face(rho) a dt dx^2 and
// face(q/rho) M, then q -= (right - left) / dx^3.  The face values use the
// limited differences of the upwind cell and the Courant number a dt / dx.
// The quantities are processed one at a time so that only the densities, their
// reciprocals and the two mass transfers stay live across the loop.  In the
// first (x) pass the momenta are built from the face velocities, whose values
// are the momenta's specific values.
template <int DIR, bool BC, bool FIRST>
__global__ void __launch_bounds__(BX * BY) k_pass(Geo G, Phys P, PassArgs A) {
  int i, j, k;
  if (!thread_cell(A.b, i, j, k)) return;
  const double dt = A.fac * A.dtp[0];
  const double dx = G.dx;
  const double mfac = dt * dx * dx;
  const double ivol = 1.0 / (dx * dx * dx);
  long cc[5];
  bool in[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) in[o] = cell_at<DIR, BC>(G, i, j, k, o - 2, cc[o]);
  double r[5], ir[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    r[o] = in[o] ? A.qi[0][cc[o]] : P.rho0;
    ir[o] = 1.0 / r[o];
  }
  const long c = lin(G, i, j, k);
  const long st = dstride(G, DIR);
  const double aL = A.v[DIR][c], aR = A.v[DIR][c + st];
  const double nuL = aL * dt / dx, nuR = aR * dt / dx;
  const double ML = face_value(r[0], r[1], r[2], r[3], aL, nuL) * aL * mfac;
  const double MR = face_value(r[1], r[2], r[3], r[4], aR, nuR) * aR * mfac;

  const int id[3] = {i, j, k};
  constexpr int T1 = (DIR == 0) ? 1 : 0;
  constexpr int T2 = (DIR == 2) ? 1 : 2;
  const int cd = id[DIR];
  // flux matching on the frontier of the finer level: the sum of its 4 faces
  // over its 2 sub-cycles replaces this level's transfers there
  int side_L = -1, side_R = -1;
  long fbase = 0;
  long fnt = 0;
  if (A.facc) {
    int o1 = G.n[T1] / 4, o2 = G.n[T2] / 4;
    int t1 = id[T1] - o1, t2 = id[T2] - o2;
    if (t1 >= 0 && t2 >= 0 && t1 < G.n[T1] / 2 && t2 < G.n[T2] / 2) {
      int lo = G.n[DIR] / 4, hi = (3 * G.n[DIR]) / 4;
      if (cd == lo || cd == hi) side_L = (cd == hi);
      if (cd + 1 == lo || cd + 1 == hi) side_R = (cd + 1 == hi);
      fnt = (long)A.fn[T1] * A.fn[T2];
      fbase = (long)(2 * t2) * A.fn[T1] + 2 * t1;
    }
  }
  auto fine_sum = [&](int side, int m) {
    const double *a = A.facc + ((long)(DIR * 2 + side) * NQ + m) * fnt + fbase;
    return (a[0] + a[1]) + (a[A.fn[T1]] + a[A.fn[T1] + 1]);
  };
  // this (fine) level's own frontier: accumulate its transfers there
  long acc_i = -1;
  int acc_side = -1;
  long acc_nt = 0;
  if (A.acc) {
    int t1 = id[T1], t2 = id[T2];
    if (t1 >= 0 && t2 >= 0 && t1 < G.n[T1] && t2 < G.n[T2] && (cd == 0 || cd == G.n[DIR] - 1)) {
      acc_nt = (long)G.n[T1] * G.n[T2];
      acc_i = (long)t2 * G.n[T1] + t1;
      acc_side = (cd == 0) ? 0 : 1;
    }
  }
  auto finish = [&](int m, double own, double FL, double FR) {
    if (side_L >= 0) FL = fine_sum(side_L, m);
    if (side_R >= 0) FR = fine_sum(side_R, m);
    if (acc_side == 0) A.acc[((long)(DIR * 2 + 0) * NQ + m) * acc_nt + acc_i] += FL;
    if (acc_side == 1) A.acc[((long)(DIR * 2 + 1) * NQ + m) * acc_nt + acc_i] += FR;
    A.qo[m][c] = own - (FR - FL) * ivol;
  };
  finish(0, r[2], ML, MR);

#pragma unroll 1
  for (int m = 1; m < NQ; ++m) {
    double sv[5];
    double own;
    if (FIRST && m >= 2) {
      // momentum P = rho v of a face velocity: its specific value is v itself
      const int d = (m - 2) >> 1;
      const bool hi = (m & 1);
      const double *vd = A.v[d];
      const long off = hi ? dstride(G, d) : 0;
#pragma unroll
      for (int o = 0; o < 5; ++o) sv[o] = in[o] ? vd[cc[o] + off] : (d == 0 ? -P.V : 0.0);
      own = r[2] * sv[2];
    } else {
      const double *q = A.qi[m];
      double qv[5];
#pragma unroll
      for (int o = 0; o < 5; ++o) qv[o] = in[o] ? q[cc[o]] : q_inflow(P, m);
#pragma unroll
      for (int o = 0; o < 5; ++o) sv[o] = qv[o] * ir[o];
      own = qv[2];
    }
    double FL = face_value(sv[0], sv[1], sv[2], sv[3], aL, nuL) * ML;
    double FR = face_value(sv[1], sv[2], sv[3], sv[4], aR, nuR) * MR;
    finish(m, own, FL, FR);
  }
}

// Streaming form of the y and z passes.  A thread owns one column segment
// [c0, c1) along DIR (lanes along x, so every load is coalesced) and walks it
// once: each cell is loaded once, each limited difference and each face
// transfer is computed once, and the cell is written as soon as its right face
// is known.  The eight quantities are split over two waves of the block: one
// moves rho, e, P-x, P+x, the other P-y, P+y, P-z, P+z (both compute the mass
// transfers they scale).
struct MarchArgs {
  int lo[3], hi[3];    // cells to update; DIR is the walked dimension
  int chunk;           // cells per segment
  const double *qi[NQ];
  double *qo[NQ];
  const double *v;     // face velocity normal to DIR (after the first kick)
  const double *dtp;
  double fac;
  double *acc;         // this level's frontier accumulators (fine levels) or null
  const double *facc;  // the finer level's accumulators or null
  int fn[3];
};

template <int DIR, bool BC>
__global__ void __launch_bounds__(256) k_march(Geo G, Phys P, MarchArgs A) {
  constexpr int TD = (DIR == 1) ? 2 : 1;   // transverse dimension walked by blocks
  constexpr int T1 = (DIR == 0) ? 1 : 0;   // transverse dimensions of a face, in order
  constexpr int T2 = (DIR == 2) ? 1 : 2;
  const int lane = threadIdx.x, ty = threadIdx.y;
  const int grp = ty & 1;
  const int nbx = (A.hi[0] - A.lo[0] + 63) / 64;
  const int ntb = (A.hi[TD] - A.lo[TD] + 1) / 2;
  const unsigned h = blockIdx.x;
  const int bx = (int)(h % (unsigned)nbx);
  const unsigned r1 = h / (unsigned)nbx;
  const int tb = (int)(r1 % (unsigned)ntb);
  const int ch = (int)(r1 / (unsigned)ntb);
  const int i = A.lo[0] + bx * 64 + lane;
  const int t = A.lo[TD] + tb * 2 + (ty >> 1);
  if (i >= A.hi[0] || t >= A.hi[TD]) return;
  const int c0 = A.lo[DIR] + ch * A.chunk;
  const int c1 = min(c0 + A.chunk, A.hi[DIR]);
  if (c0 >= c1) return;

  const double dt = A.fac * A.dtp[0];
  const double dx = G.dx;
  const double mfac = dt * dx * dx, ivol = 1.0 / (dx * dx * dx), cour = dt / dx;
  const long st = dstride(G, DIR);
  // linear index of the cell at position c along DIR in this column
  int id3[3];
  id3[0] = i;
  id3[TD] = t;
  id3[DIR] = 0;
  const long base = lin(G, id3[0], id3[1], id3[2]);
  auto cidx = [&](int c) -> long {
    if (BC) c = clampi(c, 0, G.n[DIR] - 1);
    return base + (long)c * st;
  };
  // quantities of this wave: q[0] is always rho
  const int mq[4] = {grp ? 4 : 1, grp ? 5 : 2, grp ? 6 : 3, grp ? 7 : -1};
  const int nq = grp ? 4 : 3;

  // frontier bookkeeping (transverse position of this column's faces)
  const int tv1 = id3[T1], tv2 = id3[T2];
  bool ov = false;
  long fbase = 0, fnt = 0;
  int flo = 0, fhi = 0;
  if (A.facc) {
    int a1 = tv1 - G.n[T1] / 4, a2 = tv2 - G.n[T2] / 4;
    if (a1 >= 0 && a2 >= 0 && a1 < G.n[T1] / 2 && a2 < G.n[T2] / 2) {
      ov = true;
      fnt = (long)A.fn[T1] * A.fn[T2];
      fbase = (long)(2 * a2) * A.fn[T1] + 2 * a1;
      flo = G.n[DIR] / 4;
      fhi = (3 * G.n[DIR]) / 4;
    }
  }
  const bool acc_col = A.acc && tv1 >= 0 && tv2 >= 0 && tv1 < G.n[T1] && tv2 < G.n[T2];
  const long acc_nt = (long)G.n[T1] * G.n[T2];
  const long acc_i = (long)tv2 * G.n[T1] + tv1;
  // final transfer of quantity m through face f, given the solver's value
  auto fix = [&](int f, int m, double F) -> double {
    if (ov && (f == flo || f == fhi)) {
      const double *a = A.facc + ((long)(DIR * 2 + (f == fhi)) * NQ + m) * fnt + fbase;
      F = (a[0] + a[1]) + (a[A.fn[T1]] + a[A.fn[T1] + 1]);
    }
    if (acc_col && f >= c0 && f < c1 && (f == 0 || f == G.n[DIR]))
      A.acc[((long)(DIR * 2 + (f != 0)) * NQ + m) * acc_nt + acc_i] += F;
    return F;
  };
  auto upwind = [&](double sl, double dl, double sr, double dr, double a, double nu) {
    return (a > 0.0) ? sl + 0.5 * dl * (1.0 - nu) : sr - 0.5 * dr * (1.0 + nu);
  };

  // window: specific values at c, c+1 (s0, s1), limited difference at c (d0),
  // transfer through face c (F0); index 0 is rho
  double s0[5], s1[5], d0[5], F0[5];
  {
    double sm2[5], sm1[5];
    const long im2 = cidx(c0 - 2), im1 = cidx(c0 - 1), i0 = cidx(c0), ip1 = cidx(c0 + 1);
    const double r_m2 = A.qi[0][im2], r_m1 = A.qi[0][im1], r_0 = A.qi[0][i0], r_p1 = A.qi[0][ip1];
    const double ir_m2 = 1.0 / r_m2, ir_m1 = 1.0 / r_m1, ir_0 = 1.0 / r_0, ir_p1 = 1.0 / r_p1;
    sm2[0] = r_m2; sm1[0] = r_m1; s0[0] = r_0; s1[0] = r_p1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= nq) break;
      const double *q = A.qi[mq[u]];
      sm2[u + 1] = q[im2] * ir_m2;
      sm1[u + 1] = q[im1] * ir_m1;
      s0[u + 1] = q[i0] * ir_0;
      s1[u + 1] = q[ip1] * ir_p1;
    }
    const double a = A.v[i0], nu = a * cour;
    double M = 0.0;
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      if (u > nq) break;
      const double dm1 = vleer(s0[u] - sm1[u], sm1[u] - sm2[u]);
      d0[u] = vleer(s1[u] - s0[u], s0[u] - sm1[u]);
      const double fv = upwind(sm1[u], dm1, s0[u], d0[u], a, nu);
      if (u == 0) {
        M = fv * a * mfac;
        F0[0] = grp ? M : fix(c0, 0, M);  // rho belongs to the first wave
      } else {
        F0[u] = fix(c0, mq[u - 1], fv * M);
      }
    }
  }
  // raw values of cell c+2, loaded one iteration ahead of their use
  double nx[5];
  {
    const long ip2 = cidx(c0 + 2);
    nx[0] = A.qi[0][ip2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (u < nq) nx[u + 1] = A.qi[mq[u]][ip2];
  }
  for (int c = c0; c < c1; ++c) {
    const long ic = cidx(c), ip3 = cidx(c + 3);
    // issue this iteration's independent loads first: the cell's own values,
    // its right face velocity and the cell two steps ahead
    double own[5], nn[5];
    const double a = A.v[base + (long)(c + 1) * st];
    own[0] = A.qi[0][ic];
    nn[0] = A.qi[0][ip3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < nq) {
        own[u + 1] = A.qi[mq[u]][ic];
        nn[u + 1] = A.qi[mq[u]][ip3];
      }
    }
    const double ir2 = 1.0 / nx[0];
    double s2[5];
    s2[0] = nx[0];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (u < nq) s2[u + 1] = nx[u + 1] * ir2;
    const double nu = a * cour;
    double M = 0.0;
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      if (u > nq) break;
      const double d1 = vleer(s2[u] - s1[u], s1[u] - s0[u]);
      const double fv = upwind(s0[u], d0[u], s1[u], d1, a, nu);
      double F1;
      if (u == 0) {
        M = fv * a * mfac;
        F1 = grp ? M : fix(c + 1, 0, M);
      } else {
        F1 = fix(c + 1, mq[u - 1], fv * M);
      }
      const int m = (u == 0) ? 0 : mq[u - 1];
      if (u > 0 || grp == 0) A.qo[m][ic] = own[u] - (F1 - F0[u]) * ivol;
      F0[u] = F1;
      d0[u] = d1;
      s0[u] = s1[u];
      s1[u] = s2[u];
    }
#pragma unroll
    for (int u = 0; u < 5; ++u) nx[u] = nn[u];
  }
}

// ------------------------------------------------------------ CommUp

struct UpArgs {
  const double *Q;   // coarse field
  double *out;       // fine field
  int stag;          // -1 centred, else the face normal
  double qin;        // inflow value of a centred field (coarse level 0)
  Box b;             // fine entries
};

// One 1-D step of the prolongation along dimension d: value at the fine
// position from three consecutive coarse values around the host.
__device__ __forceinline__ double up1d(bool stag_axis, int odd, double m, double c, double p) {
  if (stag_axis) return odd ? 0.5 * (c + p) : c;
  return c + vleer(p - c, c - m) * (odd ? 0.25 : -0.25);
}

__device__ __forceinline__ int fdiv2(int i) { return (i >= 0) ? i / 2 : -((1 - i) / 2); }

// CommUp (Sect. 3.2.1): every fine entry outside the fine active set from the
// 27 coarse entries around its host, interpolating along z, then y, then x.
template <bool CBC>
__global__ void __launch_bounds__(BX * BY) k_commup(Geo Gc, Geo Gf, Phys P, UpArgs A) {
  int i, j, k;
  if (!thread_cell(A.b, i, j, k)) return;
  const int id[3] = {i, j, k};
  bool active = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int hi = Gf.n[d] + (d == A.stag ? 1 : 0);
    if (id[d] < 0 || id[d] >= hi) active = false;
  }
  if (active) return;
  int H[3], odd[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    H[d] = Gc.n[d] / 4 + fdiv2(id[d]);
    odd[d] = id[d] - 2 * fdiv2(id[d]);
  }
  auto C = [&](int a, int b, int cc) -> double {
    int ci = H[0] + a, cj = H[1] + b, ck = H[2] + cc;
    if (CBC) {
      if (A.stag < 0) return cread(A.Q, Gc, ci, cj, ck, A.qin);
      return fread_bc(A.Q, Gc, A.stag, ci, cj, ck, P.V);
    }
    return A.Q[lin(Gc, ci, cj, ck)];
  };
  double r[3];
#pragma unroll
  for (int a = -1; a <= 1; ++a) {
    double qz[3];
#pragma unroll
    for (int b = -1; b <= 1; ++b) qz[b + 1] = up1d(A.stag == 2, odd[2], C(a, b, -1), C(a, b, 0), C(a, b, 1));
    r[a + 1] = up1d(A.stag == 1, odd[1], qz[0], qz[1], qz[2]);
  }
  A.out[lin(Gf, i, j, k)] = up1d(A.stag == 0, odd[0], r[0], r[1], r[2]);
}

// ------------------------------------------------------------ CommMean

struct MeanArgs {
  const double *Q;   // fine field
  double *out;       // coarse field
  int stag;
  Box b;             // coarse covered entries, relative to the covered box
};

// CommMean (Sect. 3.2.2): covered coarse cells take the mean of their 8 fine
// cells, covered coarse faces the mean of their 4 coincident fine faces.
__global__ void __launch_bounds__(BX * BY) k_commmean(Geo Gf, Geo Gc, MeanArgs A) {
  int I, J, K;
  if (!thread_cell(A.b, I, J, K)) return;
  long f = lin(Gf, 2 * I, 2 * J, 2 * K);
  double val;
  if (A.stag < 0) {
    const double *q = A.Q;
    long sx = 1, sy = Gf.sy, sz = Gf.sz;
    val = (((q[f] + q[f + sx]) + (q[f + sy] + q[f + sx + sy])) +
           ((q[f + sz] + q[f + sx + sz]) + (q[f + sy + sz] + q[f + sx + sy + sz]))) * 0.125;
  } else {
    long e1 = (A.stag == 0) ? Gf.sy : 1;
    long e2 = (A.stag == 2) ? Gf.sy : Gf.sz;
    const double *q = A.Q;
    val = ((q[f] + q[f + e1]) + (q[f + e2] + q[f + e1 + e2])) * 0.25;
  }
  A.out[lin(Gc, Gc.n[0] / 4 + I, Gc.n[1] / 4 + J, Gc.n[2] / 4 + K)] = val;
}

// -------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

struct RedArgs {
  Box b;
  const double *rho, *e, *v[3];
  double *part;      // 3 doubles per block
  Scal *S;
  int cov_lo[3], cov_hi[3];  // covered cells (empty if no finer level)
};

__device__ __forceinline__ bool is_covered(const RedArgs &A, int i, int j, int k) {
  return i >= A.cov_lo[0] && i < A.cov_hi[0] && j >= A.cov_lo[1] && j < A.cov_hi[1] && k >= A.cov_lo[2] &&
         k < A.cov_hi[2];
}

// block sum of three values into part[3*block]; fixed order for a fixed grid
__device__ void block_sum3(double a, double b, double c, double *part) {
  __shared__ double sh[3][BX * BY / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  int t = threadIdx.y * BX + threadIdx.x;
  int w = t / 64, l = t % 64;
  if (l == 0) {
    sh[0][w] = a;
    sh[1][w] = b;
    sh[2][w] = c;
  }
  __syncthreads();
  if (t == 0) {
    long blk = blockIdx.x;
    double s0 = 0, s1 = 0, s2 = 0;
    for (int q = 0; q < BX * BY / 64; ++q) {
      s0 += sh[0][q];
      s1 += sh[1][q];
      s2 += sh[2][q];
    }
    part[3 * blk + 0] = s0;
    part[3 * blk + 1] = s1;
    part[3 * blk + 2] = s2;
  }
}

// Force of the gas on the perturber, eq. 18: G M (rho - rho0) dV r / (r^2+eps^2)^{3/2}
// over uncovered active cells (the uniform part sums to zero by symmetry).
__global__ void __launch_bounds__(BX * BY) k_force(Geo G, Phys P, RedArgs A) {
  int i, j, k;
  bool ok = thread_cell(A.b, i, j, k);
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (ok && !is_covered(A, i, j, k)) {
    double x = xcen(G, 0, i), y = xcen(G, 1, j), z = xcen(G, 2, k);
    double d2 = x * x + y * y + z * z + P.eps2;
    double vol = G.dx * G.dx * G.dx;
    double w = P.GM * (A.rho[lin(G, i, j, k)] - P.rho0) * vol / (d2 * sqrt(d2));
    fx = w * x;
    fy = w * y;
    fz = w * z;
  }
  block_sum3(fx, fy, fz, A.part);
}

// mass, internal energy and kinetic energy (face velocities averaged to centres)
__global__ void __launch_bounds__(BX * BY) k_totals(Geo G, Phys P, RedArgs A) {
  int i, j, k;
  bool ok = thread_cell(A.b, i, j, k);
  double m = 0.0, ei = 0.0, ek = 0.0;
  if (ok && !is_covered(A, i, j, k)) {
    long c = lin(G, i, j, k);
    double vol = G.dx * G.dx * G.dx;
    double r = A.rho[c];
    double v2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double vc = 0.5 * (A.v[d][c] + A.v[d][c + dstride(G, d)]);
      v2 += vc * vc;
    }
    m = r * vol;
    ei = A.e[c] * vol;
    ek = 0.5 * r * v2 * vol;
  }
  (void)P;
  block_sum3(m, ei, ek, A.part);
}

// fixed-order sum of the partials of all levels (one block of 256 threads)
struct FinalArgs {
  const double *part[MAXLEV];
  int npart[MAXLEV];
  int nl;
  double *out;   // 3 doubles
  Scal *S;       // with flog: append (out, t) to the ring
  double *flog;
};

__global__ void __launch_bounds__(256) k_final3(FinalArgs A) {
  __shared__ double sh[3][4];
  double s[3] = {0.0, 0.0, 0.0};
  for (int l = 0; l < A.nl; ++l)
    for (int b = threadIdx.x; b < A.npart[l]; b += 256) {
      s[0] += A.part[l][3 * b + 0];
      s[1] += A.part[l][3 * b + 1];
      s[2] += A.part[l][3 * b + 2];
    }
#pragma unroll
  for (int q = 0; q < 3; ++q) s[q] = wave_sum(s[q]);
  int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0)
    for (int q = 0; q < 3; ++q) sh[q][w] = s[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < 3; ++q) A.out[q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
    if (A.flog) {
      unsigned int n = A.S->nlog;
      double *e = A.flog + 4 * (size_t)(n % FLOG);
      for (int q = 0; q < 3; ++q) e[q] = A.out[q];
      e[3] = A.S->t;
      A.S->nlog = n + 1;
    }
  }
}

// Largest signal speed c_s + |v| over the active cells and their faces, and
// the health check (density and energy positive and finite).
__global__ void __launch_bounds__(BX * BY) k_signal(Geo G, Phys P, RedArgs A) {
  int i, j, k;
  bool ok = thread_cell(A.b, i, j, k);
  double sig = 0.0;
  int bad = 0;
  if (ok) {
    long c = lin(G, i, j, k);
    double r = A.rho[c], en = A.e[c];
    if (!(r > 0.0) || !(en > 0.0) || !isfinite(r) || !isfinite(en)) bad = 1;
    double cs = sqrt(P.gamma * P.gm1 * en / r);
    double vm = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double a = fabs(A.v[d][c]), b = fabs(A.v[d][c + dstride(G, d)]);
      vm = fmax(vm, fmax(a, b));
    }
    sig = cs + vm;
    if (!isfinite(sig)) bad = 1;
  }
  sig = wave_max(bad ? 0.0 : sig);
  bool anybad = __any(bad);
  __shared__ double sh[BX * BY / 64];
  int t = threadIdx.y * BX + threadIdx.x;
  if ((t % 64) == 0) {
    sh[t / 64] = sig;
    if (anybad) atomicOr(&A.S->health, 1);
  }
  __syncthreads();
  if (t == 0) {
    double m = sh[0];
    for (int q = 1; q < BX * BY / 64; ++q) m = fmax(m, sh[q]);
    long blk = blockIdx.x;
    A.part[blk] = m;  // per-block maximum; reduced by k_dt_final
  }
}

struct DtArgs {
  double dx[MAXLEV];
  const double *part[MAXLEV];  // per-block maximum signal speeds of each level
  int npart[MAXLEV];
  int nl;
  int advance;
};

// coarse step cfl * min_l 2^l min(dx_l / smax_l, dx_l^2 / (6 chi)) (eq. 55, xi = 2)
__global__ void __launch_bounds__(256) k_dt_final(Phys P, DtArgs A, Scal *S) {
  __shared__ double sh[4];
  __shared__ double smax[MAXLEV];
  for (int l = 0; l < A.nl; ++l) {
    double m = 0.0;
    for (int b = threadIdx.x; b < A.npart[l]; b += 256) m = fmax(m, A.part[l][b]);
    m = wave_max(m);
    if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) smax[l] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double best = INFINITY;
  for (int l = 0; l < A.nl; ++l) {
    double dtl = A.dx[l] / smax[l];
    if (P.chi > 0.0) dtl = fmin(dtl, A.dx[l] * A.dx[l] / (6.0 * P.chi));
    dtl = ldexp(dtl, l);
    best = fmin(best, dtl);
  }
  double dt0 = P.cfl * best;
  for (int l = 0; l < A.nl; ++l) S->dt[l] = ldexp(dt0, -l);
  if (A.advance) S->t += dt0;
}

__global__ void k_zero(double *p, size_t n) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) p[t] = 0.0;
}

// every stored entry (level 0 stores cells 0..n-1 and faces 0..n)
Box full_box(const Geo &G) {
  Box b;
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = -G.g;
    b.hi[d] = G.s[d] - G.g;
  }
  return b;
}
Box active_box(const Geo &G) {
  Box b;
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = 0;
    b.hi[d] = G.n[d];
  }
  return b;
}
Box uniform_box(const Geo &G, int lo_off, int hi_off) {
  Box b;
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = -G.g + lo_off;
    b.hi[d] = G.n[d] + G.g - hi_off;
  }
  return b;
}

}  // namespace

// launch only non-empty grids
#define DFK_LAUNCH(K, GR, BL, ST, ...)                                   \
  do {                                                                   \
    dim3 g_ = (GR);                                                      \
    if (!empty_grid(g_)) hipLaunchKernelGGL(K, g_, BL, 0, ST, __VA_ARGS__); \
  } while (0)

// ======================================================================
// launchers

void init_state(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, uint64_t seed,
                double amp) {
  InitArgs A;
  A.b = full_box(G);
  A.rho = B.q[cur][0];
  A.e = B.q[cur][1];
  A.vx = B.v[0];
  A.vy = B.v[1];
  A.vz = B.v[2];
  A.seed = seed;
  A.amp = amp;
  DFK_LAUNCH(k_init, grid_of(A.b), dim3(BX, BY), st, G, P, A);
}

static void kick_common(hipStream_t st, const Geo &G, const Phys &P, const double *const *q, double **v,
                        const double *dtp, double fac, bool rebuild, bool do_kick) {
  KickArgs A;
  for (int d = 0; d < 3; ++d)
    for (int e = 0; e < 3; ++e) {
      if (G.bc) {
        A.flo[d][e] = 0;
        A.fhi[d][e] = G.n[e] + (d == e ? 1 : 0);
      } else if (!rebuild) {
        A.flo[d][e] = -G.g + (d == e ? 1 : 0);
        A.fhi[d][e] = G.n[e] + G.g;
      } else {
        A.flo[d][e] = -G.g + (d == e ? 3 : 2);
        A.fhi[d][e] = G.n[e] + G.g - 3;
      }
    }
  for (int e = 0; e < 3; ++e) {
    A.b.lo[e] = A.flo[0][e] < A.flo[1][e] ? A.flo[0][e] : A.flo[1][e];
    A.b.lo[e] = A.b.lo[e] < A.flo[2][e] ? A.b.lo[e] : A.flo[2][e];
    A.b.hi[e] = A.fhi[0][e] > A.fhi[1][e] ? A.fhi[0][e] : A.fhi[1][e];
    A.b.hi[e] = A.b.hi[e] > A.fhi[2][e] ? A.b.hi[e] : A.fhi[2][e];
  }
  for (int m = 0; m < NQ; ++m) A.q[m] = q[m];
  for (int d = 0; d < 3; ++d) A.v[d] = v[d];
  A.dtp = dtp;
  A.fac = fac;
  dim3 gr = grid_of(A.b), bl(BX, BY);
  if (G.bc) {
    if (rebuild && do_kick) DFK_LAUNCH((k_kick<true, true, true>), gr, bl, st, G, P, A);
    else if (rebuild) DFK_LAUNCH((k_kick<true, true, false>), gr, bl, st, G, P, A);
    else DFK_LAUNCH((k_kick<true, false, true>), gr, bl, st, G, P, A);
  } else {
    if (rebuild && do_kick) DFK_LAUNCH((k_kick<false, true, true>), gr, bl, st, G, P, A);
    else if (rebuild) DFK_LAUNCH((k_kick<false, true, false>), gr, bl, st, G, P, A);
    else DFK_LAUNCH((k_kick<false, false, true>), gr, bl, st, G, P, A);
  }
}

void kick(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp, double fac) {
  kick_common(st, G, P, B.q[cur], B.v, dtp, fac, false, true);
}

void rebuild_kick(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src, const double *dtp,
                  double fac, bool do_kick) {
  kick_common(st, G, P, B.q[src], B.v, dtp, fac, true, do_kick);
}

void compress(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
              double fac) {
  CellArgs A;
  A.b = G.bc ? active_box(G) : uniform_box(G, 0, 1);
  A.rho = B.q[cur][0];
  A.e = B.q[cur][1];
  for (int d = 0; d < 3; ++d) A.v[d] = B.v[d];
  A.dtp = dtp;
  A.fac = fac;
  DFK_LAUNCH(k_compress, grid_of(A.b), dim3(BX, BY), st, G, P, A);
}

void diffuse_heat(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
                  double fac, bool do_diff, bool do_heat) {
  DiffArgs A;
  A.b = G.bc ? active_box(G) : uniform_box(G, 1, 1);
  A.rho = B.q[cur][0];
  A.e = B.q[cur][1];
  A.eo = B.etmp;
  A.hw = B.hw;
  for (int d = 0; d < 3; ++d) {
    A.hw_n[d] = B.hw_n[d];
    A.hw_lo[d] = G.n[d] / 2 - B.hw_n[d] / 2;
  }
  A.dtp = dtp;
  A.fac = fac;
  A.do_diff = do_diff && P.chi > 0.0;
  A.do_heat = do_heat && P.L != 0.0;
  if (G.bc) DFK_LAUNCH(k_diffuse_heat<true>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  else DFK_LAUNCH(k_diffuse_heat<false>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
}

void transport_pass(hipStream_t st, int dir, const Geo &G, const Phys &P, LevBufs &B, int src,
                    const double *dtp, double fac, const Geo *Gf, const double *fine_acc) {
  PassArgs A;
  if (G.bc) {
    A.b = active_box(G);
  } else {
    // in-bounds ranges that cover every entry the active cells depend on
    for (int d = 0; d < 3; ++d) {
      if (d == dir) {
        A.b.lo[d] = -G.g + 2;
        A.b.hi[d] = G.n[d] + G.g - 3;
      } else if (dir == 0) {
        A.b.lo[d] = -G.g;
        A.b.hi[d] = G.n[d] + G.g - 1;
      } else if (d < dir) {
        A.b.lo[d] = -G.g + 2;
        A.b.hi[d] = G.n[d] + G.g - 3;
      } else {
        A.b.lo[d] = -G.g;
        A.b.hi[d] = G.n[d] + G.g - 1;
      }
    }
  }
  for (int m = 0; m < NQ; ++m) {
    A.qi[m] = B.q[src][m];
    A.qo[m] = B.q[1 - src][m];
  }
  for (int d = 0; d < 3; ++d) A.v[d] = B.v[d];
  A.dtp = dtp;
  A.fac = fac;
  A.acc = G.level > 0 ? B.acc : nullptr;
  A.facc = (G.has_fine && fine_acc) ? fine_acc : nullptr;
  for (int d = 0; d < 3; ++d) A.fn[d] = Gf ? Gf->n[d] : 0;
  if (dir == 0) {
    dim3 gr = grid_of(A.b), bl(BX, BY);
    if (G.bc) DFK_LAUNCH((k_pass<0, true, true>), gr, bl, st, G, P, A);
    else DFK_LAUNCH((k_pass<0, false, true>), gr, bl, st, G, P, A);
    return;
  }
  MarchArgs M;
  for (int d = 0; d < 3; ++d) {
    M.lo[d] = A.b.lo[d];
    M.hi[d] = A.b.hi[d];
    M.fn[d] = A.fn[d];
  }
  const int ext = M.hi[dir] - M.lo[dir];
  M.chunk = ext <= 16 ? ext : 16;
  for (int m = 0; m < NQ; ++m) {
    M.qi[m] = A.qi[m];
    M.qo[m] = A.qo[m];
  }
  M.v = A.v[dir];
  M.dtp = A.dtp;
  M.fac = A.fac;
  M.acc = A.acc;
  M.facc = A.facc;
  const int td = (dir == 1) ? 2 : 1;
  const long nbx = (M.hi[0] - M.lo[0] + 63) / 64;
  const long ntb = (M.hi[td] - M.lo[td] + 1) / 2;
  const long nch = (ext + M.chunk - 1) / M.chunk;
  dim3 gr((unsigned)(nbx * ntb * nch)), bl(64, 4);
  if (ext <= 0) return;
  if (G.bc) {
    if (dir == 1) DFK_LAUNCH((k_march<1, true>), gr, bl, st, G, P, M);
    else DFK_LAUNCH((k_march<2, true>), gr, bl, st, G, P, M);
  } else {
    if (dir == 1) DFK_LAUNCH((k_march<1, false>), gr, bl, st, G, P, M);
    else DFK_LAUNCH((k_march<2, false>), gr, bl, st, G, P, M);
  }
}

void zero(hipStream_t st, double *p, size_t n) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}

void commup(hipStream_t st, const Geo &Gc, const Phys &P, LevBufs &Bc, int curc, const Geo &Gf, LevBufs &Bf,
            int curf) {
  for (int f = 0; f < NSTATE; ++f) {
    UpArgs A;
    A.stag = f >= 2 ? f - 2 : -1;
    A.Q = f == 0 ? Bc.q[curc][0] : (f == 1 ? Bc.q[curc][1] : Bc.v[f - 2]);
    A.out = f == 0 ? Bf.q[curf][0] : (f == 1 ? Bf.q[curf][1] : Bf.v[f - 2]);
    A.qin = f == 0 ? P.rho0 : P.e0;
    A.b = full_box(Gf);
    if (Gc.bc) DFK_LAUNCH(k_commup<true>, grid_of(A.b), dim3(BX, BY), st, Gc, Gf, P, A);
    else DFK_LAUNCH(k_commup<false>, grid_of(A.b), dim3(BX, BY), st, Gc, Gf, P, A);
  }
}

void commmean(hipStream_t st, const Geo &Gf, LevBufs &Bf, int curf, const Geo &Gc, LevBufs &Bc, int curc) {
  for (int f = 0; f < NSTATE; ++f) {
    MeanArgs A;
    A.stag = f >= 2 ? f - 2 : -1;
    A.Q = f == 0 ? Bf.q[curf][0] : (f == 1 ? Bf.q[curf][1] : Bf.v[f - 2]);
    A.out = f == 0 ? Bc.q[curc][0] : (f == 1 ? Bc.q[curc][1] : Bc.v[f - 2]);
    for (int d = 0; d < 3; ++d) {
      A.b.lo[d] = 0;
      A.b.hi[d] = Gc.n[d] / 2 + (d == A.stag ? 1 : 0);
    }
    DFK_LAUNCH(k_commmean, grid_of(A.b), dim3(BX, BY), st, Gf, Gc, A);
  }
}

size_t part_count(const Geo &G) {
  Box b = active_box(G);
  dim3 g = grid_of(b);
  return (size_t)g.x * g.y * g.z;
}

static RedArgs red_args(const Geo &G, LevBufs &B, int cur) {
  RedArgs A;
  A.b = active_box(G);
  A.rho = B.q[cur][0];
  A.e = B.q[cur][1];
  for (int d = 0; d < 3; ++d) A.v[d] = B.v[d];
  A.part = B.part;
  A.S = nullptr;
  for (int d = 0; d < 3; ++d) {
    if (G.has_fine) {
      A.cov_lo[d] = G.n[d] / 4;
      A.cov_hi[d] = (3 * G.n[d]) / 4;
    } else {
      A.cov_lo[d] = 0;
      A.cov_hi[d] = 0;
    }
  }
  return A;
}

void signal_speed(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, Scal *S) {
  RedArgs A = red_args(G, B, cur);
  A.S = S;
  DFK_LAUNCH(k_signal, grid_of(A.b), dim3(BX, BY), st, G, P, A);
}

void dt_final(hipStream_t st, const Geo *G, const LevBufs *B, int nl, const Phys &P, Scal *S, int advance) {
  DtArgs A;
  for (int l = 0; l < MAXLEV; ++l) {
    A.dx[l] = l < nl ? G[l].dx : 0.0;
    A.part[l] = l < nl ? B[l].part : nullptr;
    A.npart[l] = l < nl ? (int)part_count(G[l]) : 0;
  }
  A.nl = nl;
  A.advance = advance;
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, st, P, A, S);
}

int force_partials(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur) {
  RedArgs A = red_args(G, B, cur);
  DFK_LAUNCH(k_force, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  return (int)part_count(G);
}

int totals_partials(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur) {
  RedArgs A = red_args(G, B, cur);
  DFK_LAUNCH(k_totals, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  return (int)part_count(G);
}

void force_final(hipStream_t st, double *const *parts, const int *nparts, int nl, Scal *S, int slot,
                 double *flog) {
  FinalArgs A;
  for (int l = 0; l < MAXLEV; ++l) {
    A.part[l] = l < nl ? parts[l] : nullptr;
    A.npart[l] = l < nl ? nparts[l] : 0;
  }
  A.nl = nl;
  A.out = slot == 1 ? S->totals : S->force;
  A.S = S;
  A.flog = slot == 2 ? flog : nullptr;
  hipLaunchKernelGGL(k_final3, dim3(1), dim3(256), 0, st, A);
}

}  // namespace dfk
