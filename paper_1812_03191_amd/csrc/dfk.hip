// dfk.hip -- gfx950 kernels of libdfmesh.
//
// The update of one level over a step dt follows the staging list of Velasco
// Romero & Masset (2018), Sect. 3.3, with the split source step of eq. 15:
//   kick(dt/2) -> compression, diffusion, heat release (dt) -> transport (dt)
//   -> kick(dt/2)
//
// Storage and arithmetic.  Every field is stored as its departure from the
// uniform background (rho0, e0, wind (-V, 0, 0), momenta rho0 (-V, 0, 0)) in
// the run's storage type T: double (FP64 runs) or float (FP32 runs).  The
// stencils are written for departures: the uniform background transfer is the
// same through every face and cancels from every flux difference, so it is
// never formed, and the potential difference across a face is taken in a form
// free of cancellation.  Forces, totals and the time step are reduced in FP64.
//
// Launch shape.  Box kernels launch a 1-D grid of 64 x 4 tiles times one plane;
// level 0 reads its outer boundary conditions on the fly (clamped indices, a
// zero departure beyond the inflow face), so it stores no ghost data; finer
// levels advance their whole ghost shell, filled once per parent step.
#include "dfk.h"

#include <cstdlib>
#include <cstring>
#include <type_traits>

namespace dfk {

namespace {

constexpr int BX = 64, BY = 4;

struct Box {
  int lo[3], hi[3];
};

inline bool empty_grid(const dim3 &g) { return g.x == 0; }

// The hardware hands workgroups to the 8 XCDs round-robin (workgroup h runs
// on XCD h % 8).  thread_cell gives each XCD one contiguous range of tiles: a
// band of rows through all planes, walked plane by plane (x-tile fastest, then
// y-tile within the band, then plane), so the neighbour planes a stencil
// reads are in its own L2 (a few planes of one band fit there) and neighbour
// rows are too except at band edges.
inline dim3 grid_of(const Box &b) {
  int ex = b.hi[0] - b.lo[0], ey = b.hi[1] - b.lo[1], ez = b.hi[2] - b.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return dim3(0, 1, 1);
  long n = (long)((ex + BX - 1) / BX) * ((ey + BY - 1) / BY) * ez;
  return dim3((unsigned)n, 1, 1);
}

// A block's place in its launch: the hardware's, or, in a launch that
// carries the blocks of several runs (the engine's batched stages), its place
// among its own run's blocks.
struct Blk {
  unsigned id, n;
};
__device__ __forceinline__ Blk grid_blk() { return Blk{blockIdx.x, gridDim.x}; }

__device__ __forceinline__ bool thread_cell(const Box &b, int &i, int &j, int &k, Blk bk = grid_blk()) {
  const unsigned nbx = (unsigned)(b.hi[0] - b.lo[0] + BX - 1) / BX;
  const unsigned nby = (unsigned)(b.hi[1] - b.lo[1] + BY - 1) / BY;
  const unsigned N = bk.n, h = bk.id;
  const unsigned nbz = N / (nbx * nby);
  const unsigned q = N / 8, r = N % 8, x = h % 8, s = h / 8;
  unsigned L = (x < r) ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
  const unsigned hq = nby / 8, hr = nby % 8;
  unsigned y0 = 0, hb = hq + (hr > 0);
  for (unsigned bb = 0; bb < 8; ++bb) {
    hb = hq + (bb < hr ? 1u : 0u);
    unsigned nt = nbx * hb * nbz;
    if (L < nt || bb == 7) break;
    L -= nt;
    y0 += hb;
  }
  const unsigned bx = L % nbx, t = L / nbx;
  const unsigned by = y0 + t % hb, bz = t / hb;
  i = b.lo[0] + (int)(bx * BX + threadIdx.x);
  j = b.lo[1] + (int)(by * BY + threadIdx.y);
  k = b.lo[2] + (int)bz;
  return i < b.hi[0] && j < b.hi[1];
}

// Flat tiles, for the box kernels whose lanes do not exchange values along x
// (and for the level-0 pair kernels, whose lanes check for it): the (x, row)
// entries of a plane are numbered row by row and each wave takes 64
// consecutive ones, so that rows whose length is not a multiple of 64 share
// waves (a row of 64 entries is one wave, and the tiles are those of
// thread_cell); blocks of four waves go to the XCDs in bands through all
// planes as there.  A lane's previous lane then holds the previous entry of
// its row unless the lane is the first of its wave or its entry the first of
// its row.  With WS = BX - 1 entries per wave, the waves overlap by one entry:
// the last lane holds the entry after the wave's own (the next wave's first).
template <int WS = BX>
inline dim3 grid_of_flat(const Box &b) {
  const long ex = b.hi[0] - b.lo[0], ey = b.hi[1] - b.lo[1], ez = b.hi[2] - b.lo[2];
  if (ex <= 0 || ey <= 0 || ez <= 0) return dim3(0, 1, 1);
  return dim3((unsigned)((ex * ey + WS * BY - 1) / (WS * BY) * ez), 1, 1);
}

template <int WS = BX>
__device__ __forceinline__ bool thread_cell_flat(const Box &b, int &i, int &j, int &k, Blk bk = grid_blk()) {
  const unsigned ex = (unsigned)(b.hi[0] - b.lo[0]), ey = (unsigned)(b.hi[1] - b.lo[1]);
  const unsigned nby = (ex * ey + WS * BY - 1) / (WS * BY);  // blocks per plane
  const unsigned N = bk.n, h = bk.id;
  const unsigned nbz = N / nby;
  const unsigned q = N / 8, r = N % 8, x = h % 8, s = h / 8;
  unsigned L = (x < r) ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
  const unsigned hq = nby / 8, hr = nby % 8;
  unsigned y0 = 0, hb = hq + (hr > 0);
  for (unsigned bb = 0; bb < 8; ++bb) {
    hb = hq + (bb < hr ? 1u : 0u);
    unsigned nt = hb * nbz;
    if (L < nt || bb == 7) break;
    L -= nt;
    y0 += hb;
  }
  const unsigned by = y0 + L % hb, bz = L / hb;
  const unsigned f = by * (WS * BY) + threadIdx.y * WS + threadIdx.x;
  i = b.lo[0] + (int)(f % ex);
  j = b.lo[1] + (int)(f / ex);
  k = b.lo[2] + (int)bz;
  return f < ex * ey;
}

// Element indices are 32-bit (a field holds fewer than 2^31 entries, checked
// when a mesh is created): with a uniform 64-bit base in scalar registers the
// loads and stores then take a 32-bit per-lane offset, with no 64-bit address
// arithmetic per lane.
using idx_t = int;

__device__ __forceinline__ idx_t lin(const Geo &G, int i, int j, int k) {
  return (idx_t)G.off + i + j * (idx_t)G.sy + k * (idx_t)G.sz;
}

__device__ __forceinline__ idx_t dstride(const Geo &G, int d) {
  return d == 0 ? 1 : (d == 1 ? (idx_t)G.sy : (idx_t)G.sz);
}

// Load and store at a non-negative element index whose byte offset fits 32
// bits (every field is smaller than 4 GiB): the address is a uniform base plus
// an unsigned 32-bit lane offset, which the hardware adds itself.
template <typename T>
__device__ __forceinline__ T gld(const T *p, idx_t i) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) +
                                      (unsigned)i * (unsigned)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void gst(T *p, idx_t i, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(p) + (unsigned)i * (unsigned)sizeof(T)) = v;
}

// W adjacent cells of a row in one lane: T itself, or a two-element vector
// whose loads and stores are single 8- or 16-byte accesses (the first cell's
// index is even and rows start 128-byte aligned)
template <typename T, int W>
struct lanes_of {
  using type = T;
};
template <>
struct lanes_of<double, 2> {
  using type = double __attribute__((ext_vector_type(2)));
};
template <>
struct lanes_of<float, 2> {
  using type = float __attribute__((ext_vector_type(2)));
};

// a * b + c with one rounding, per element of a lane vector
template <typename V>
__device__ __forceinline__ V fmav(V a, V b, V c) {
  return __builtin_elementwise_fma(a, b, c);
}

template <typename V, typename T>
__device__ __forceinline__ V gldv(const T *p, idx_t i) {
  return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(p) + (unsigned)i * (unsigned)sizeof(T));
}
template <typename V, typename T>
__device__ __forceinline__ void gstv(T *p, idx_t i, V v) {
  *reinterpret_cast<V *>(reinterpret_cast<char *>(p) + (unsigned)i * (unsigned)sizeof(T)) = v;
}

// W per-cell values of a lane as its lanes_of vector
template <typename V, typename T, int W>
__device__ __forceinline__ V to_lanes(const T (&a)[W]) {
  if constexpr (W == 1) {
    return a[0];
  } else {
    V v;
    v.x = a[0];
    v.y = a[1];
    return v;
  }
}

template <typename V, typename T, int W>
__device__ __forceinline__ void from_lanes(V v, T (&a)[W]) {
  if constexpr (W == 1) {
    a[0] = v;
  } else {
    a[0] = v.x;
    a[1] = v.y;
  }
}

// cell-centre coordinate: the perturber is the central vertex of the level
template <typename T>
__device__ __forceinline__ T xcen(const Geo &G, int d, int i) {
  return (T)(((double)i - G.org[d] + 0.5) * G.dx);
}

// Quotient and square root in the storage type, from the hardware reciprocal
// and reciprocal square root instead of the correctly rounded expansions: in
// FP64 the hardware reciprocal (relative error up to 4.6e-8, measured on
// gfx950) takes one Newton step and the quotient is the dividend times it
// (within 2.2e-15 of the quotient, measured over 4 M divisors; a second step
// would reach about an ulp), the square root one Goldschmidt step and one
// residual correction (within an ulp); in FP32 both are the single hardware
// instructions (about 1 ulp each).  Every use has a normal
// positive operand or divisor (densities and energies near their background,
// squared distances of at least a quarter cell, sums of two slopes of one
// sign; a van Leer quotient of slopes of opposite signs is selected away).
__device__ __forceinline__ double qdiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return a * r;
}
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
template <typename V>
__device__ __forceinline__ V qdiv(V a, V b) {
  return V{qdiv(a.x, b.x), qdiv(a.y, b.y)};  // two-element vectors, per element
}
__device__ __forceinline__ double qsqrt(double x) {
  // hardware reciprocal square root, one of Goldschmidt's steps towards
  // g = sqrt(x), h = 1/(2 sqrt(x)), one residual correction (within an ulp,
  // as with two steps: measured over 4 M arguments on gfx950)
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return fma(fma(-g, g, x), h, g);
}
__device__ __forceinline__ float qsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
template <typename V>
__device__ __forceinline__ V qsqrtv(V x) {
  V r;
  r.x = qsqrt(x.x);  // two-element vectors, per element
  r.y = qsqrt(x.y);
  return r;
}

// van Leer's harmonic limited difference; evaluated without a branch (the
// quotient of the discarded side is selected away)
template <typename T>
__device__ __forceinline__ T vleer(T a, T b) {
  const T p = a * b;
  const T r = qdiv(T(2) * p, a + b);
  return p > T(0) ? r : T(0);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// mirror image of a ghost index across the low (idx < 0) or high (idx >= n) side
__device__ __forceinline__ int mirror_idx(int idx, int n) {
  return idx < 0 ? -1 - idx : (idx >= n ? 2 * n - 1 - idx : idx);
}

// Level-0 read of a centred departure with the outer boundary conditions
// (M: the level's bc).  bc 1: zero departure (the inflow state) beyond x_max, the nearest active
// cell elsewhere (zero-gradient outflow).  bc 2: zero departure (the
// background) beyond both flow ends, mirror images across the walls.  (For
// momenta only the ones normal to x read ghosts here, which hold the
// background at the flow ends in both modes.)
template <int M, typename T>
__device__ __forceinline__ T cread(const T *q, const Geo &G, int i, int j, int k) {
  if (M == 2) {
    if (i < 0 || i >= G.n[0]) return T(0);
    return q[lin(G, i, mirror_idx(j, G.n[1]), mirror_idx(k, G.n[2]))];
  }
  if (i >= G.n[0]) return T(0);
  i = i < 0 ? 0 : i;
  j = clampi(j, 0, G.n[1] - 1);
  k = clampi(k, 0, G.n[2] - 1);
  return q[lin(G, i, j, k)];
}

// Level-0 read of the velocity departure normal to faces of dimension d
// (active faces 0..n along d; M: the level's bc).  bc 1: zero beyond x_max, copies elsewhere.
// bc 2: zero (the wind) beyond both flow ends for x faces, mirror images
// across the flow ends for the tangential ones; across a wall the normal
// velocity is reversed (zero on the wall) and the tangential ones mirrored.
template <int M, typename T>
__device__ __forceinline__ T fread_bc(const T *v, const Geo &G, int d, int i, int j, int k) {
  if (M == 2) {
    T sgn = T(1);
    if (d == 0) {
      if (i < 0 || i > G.n[0]) return T(0);
    } else {
      i = mirror_idx(i, G.n[0]);
    }
    int id[3] = {i, j, k};
#pragma unroll
    for (int e = 1; e < 3; ++e) {
      if (d == e) {
        if (id[e] < 0) { id[e] = -id[e]; sgn = -sgn; }
        else if (id[e] > G.n[e]) { id[e] = 2 * G.n[e] - id[e]; sgn = -sgn; }
      } else {
        id[e] = mirror_idx(id[e], G.n[e]);
      }
    }
    return sgn * v[lin(G, id[0], id[1], id[2])];
  }
  if (d == 0) {
    if (i > G.n[0]) return T(0);
  } else if (i >= G.n[0]) {
    return T(0);
  }
  i = i < 0 ? 0 : i;
  j = clampi(j, 0, G.n[1] - (d == 1 ? 0 : 1));
  k = clampi(k, 0, G.n[2] - (d == 2 ? 0 : 1));
  return v[lin(G, i, j, k)];
}

// background of the wind along dimension d and of the transported quantities
__device__ __forceinline__ double vback(const Phys &P, int d) { return d == 0 ? -P.V : 0.0; }
__device__ __forceinline__ double qback(const Phys &P, int m) {
  return m == 0 ? P.rho0 : (m == 1 ? P.e0 : ((m == 2 || m == 3) ? -P.rho0 * P.V : 0.0));
}
// background specific value q0 / rho0
__device__ __forceinline__ double sback(const Phys &P, int m) {
  return m == 1 ? P.e0 / P.rho0 : ((m == 2 || m == 3) ? -P.V : 0.0);
}

// Neighbour exchange inside a wave through the data-parallel-primitive lane
// shifts: from_left gives every lane the value of the lane below it, from_right
// that of the lane above it (the end lanes receive 0).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ float dpp_t(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}

template <int CTRL>
__device__ __forceinline__ double dpp_t(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;

template <typename T>
__device__ __forceinline__ T from_left(T v) { return dpp_t<DPP_WAVE_SHR1>(v); }

template <typename T>
__device__ __forceinline__ T from_right(T v) { return dpp_t<DPP_WAVE_SHL1>(v); }

// ------------------------------------------------------------------ init

// SplitMix64 finaliser (Steele, Lea & Flood 2014); output n of the stream
// with seed s is mix(s + (n+1) * 0x9e3779b97f4a7c15).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

template <typename T>
struct InitArgs {
  Box b;
  T *rho, *e, *vx, *vy, *vz;
  uint64_t seed;
  double amp;
};

// uniform background (zero departures) plus the density noise of the active
// cells: rho = rho0 (1 + A (2U - 1))
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_init(Geo G, Phys P, InitArgs<T> A) {
  int i, j, k;
  if (!thread_cell(A.b, i, j, k)) return;
  idx_t c = lin(G, i, j, k);
  double dr = 0.0;
  bool active = i >= 0 && j >= 0 && k >= 0 && i < G.n[0] && j < G.n[1] && k < G.n[2];
  if (active && A.amp != 0.0) {
    uint64_t a = ((uint64_t)k * (uint64_t)G.n[1] + (uint64_t)j) * (uint64_t)G.n[0] + (uint64_t)i;
    uint64_t n = ((uint64_t)G.level << 40) + a;
    uint64_t z = mix64(A.seed + (n + 1ULL) * 0x9e3779b97f4a7c15ULL);
    double U = (double)(z >> 11) * 0x1.0p-53;
    dr = P.rho0 * (A.amp * (2.0 * U - 1.0));
  }
  A.rho[c] = (T)dr;
  A.e[c] = T(0);
  A.vx[c] = T(0);
  A.vy[c] = T(0);
  A.vz[c] = T(0);
}

// ------------------------------------------------------------------ kick

template <typename T>
struct KickArgs {
  Box b;                     // union of the three face ranges
  int flo[3][3], fhi[3][3];  // [normal dir][dim] face ranges
  const T *q[NQ];            // rho, e (and the momenta when rebuilding)
  T *v[3];                   // face velocities written
  const T *vin[3];           // face velocities read (v itself, or the set a fused kick reads from)
  const double *dtp;
  double fac;
  Scal *slots;               // non-null: the step length from slots->smax (single-level runs)
  // with the compression fused (level 0): the compressed energy departures
  // (a buffer other than q[1], which every thread reads for the kick), the
  // compression's share of the step length, and the force log of the last
  // step's state (non-null log: the first block logs it, as k_compress2 does)
  T *eo;
  double cfac;
  Scal *log;
  const double *part;
  int npart;
  double *flog;
};

// Velocity source S(h) (eq. 15): each face velocity receives
// -h [ (gamma-1)(e_c - e_m) / (dx rho_face) + (Phi_c - Phi_m) / dx ],
// with Phi = -GM / sqrt(r^2 + eps^2) (eq. 16).  Since only the coordinate
// along the face normal differs between the two cells,
// (Phi_c - Phi_m)/dx = GM (x_c + x_m) / (d_c d_m (d_c + d_m)).
// REBUILD first sets the face velocity from the transported momenta,
// (P+_m + P-_c) / (rho_m + rho_c).  KICK = false skips the source.
template <typename T, bool REBUILD, bool KICK>
__global__ void __launch_bounds__(BX * BY) k_kick(Geo G, Phys P, KickArgs<T> A) {
  int i, j, k;
  if (!thread_cell_flat(A.b, i, j, k)) return;
  bool need = false;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    need |= i >= A.flo[d][0] && i < A.fhi[d][0] && j >= A.flo[d][1] && j < A.fhi[d][1] &&
            k >= A.flo[d][2] && k < A.fhi[d][2];
  if (!need) return;
  const T h = (T)(A.fac * A.dtp[0]);
  const T rho0 = (T)P.rho0, gm1 = (T)P.gm1, GM = (T)P.GM, eps2 = (T)P.eps2, dx = (T)G.dx;
  const T *rho = A.q[0], *e = A.q[1];
  const idx_t c = lin(G, i, j, k);
  const T drc = rho[c], dec = e[c];
  const T xc[3] = {xcen<T>(G, 0, i), xcen<T>(G, 1, j), xcen<T>(G, 2, k)};
  const T r2c = xc[0] * xc[0] + xc[1] * xc[1] + xc[2] * xc[2] + eps2;
  const T dcen = qsqrt(r2c);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    bool in = i >= A.flo[d][0] && i < A.fhi[d][0] && j >= A.flo[d][1] && j < A.fhi[d][1] &&
              k >= A.flo[d][2] && k < A.fhi[d][2];
    if (!in) continue;
    const int im = i - (d == 0), jm = j - (d == 1), km = k - (d == 2);
    const idx_t m = c - dstride(G, d);
    const T drm = rho[m], dem = e[m];
    T vf;
    if (REBUILD) {
      const T *pm = A.q[2 + 2 * d], *pp = A.q[3 + 2 * d];
      const T ppm = pp[m], pmc = pm[c];
      const T vb = (T)vback(P, d);
      vf = qdiv(ppm + pmc - vb * (drm + drc), T(2) * rho0 + drm + drc);
    } else {
      vf = A.v[d][c];
    }
    if (KICK) {
      const T rface = rho0 + T(0.5) * (drm + drc);
      const T gradp = qdiv(gm1 * (dec - dem), dx * rface);
      const T xm = xc[d] - dx;
      const T dm = qsqrt(r2c - xc[d] * xc[d] + xm * xm);
      const T gradphi = qdiv(GM * (xc[d] + xm), dm * dcen * (dm + dcen));
      vf = vf - h * (gradp + gradphi);
    }
    A.v[d][c] = vf;
  }
}

// The first kick and the compression of a finer level in one launch (as
// kick_compress on level 0): a cell of the kick's union box kicks its low
// faces that lie in their ranges into A.v, reading the faces from A.vin; a
// cell of the compression box cb also compresses its energy into A.eo, from
// the six kicked faces around it.  The waves take 63 cells of the box's flat
// numbering each and their last lane the cell after them, so that the high x
// face of a cell is the low face its next lane kicked (a cell of cb is never
// the last of its row); the high y and z faces the cell kicks again, by the
// expression of the cell above, with every distance formed from the cells'
// own coordinates (the same value).  A face of the union box outside its
// range is copied unkicked (what the separate kick leaves there).
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_kick_compress_fine(Geo G, Phys P, KickArgs<T> A, Box cb, Box ub) {
#pragma clang fp contract(off)
  int i, j, k;
  // no lane leaves before the exchange along x: a lane past the box takes
  // the box's first cell and writes nothing
  const bool inb = thread_cell_flat<BX - 1>(ub, i, j, k);
  const bool own = inb && threadIdx.x < BX - 1;
  if (!inb) {
    i = ub.lo[0];
    j = ub.lo[1];
    k = ub.lo[2];
  }
  const T h = (T)(A.fac * A.dtp[0]);
  const T rho0 = (T)P.rho0, gm1 = (T)P.gm1, GM = (T)P.GM, eps2 = (T)P.eps2, dx = (T)G.dx;
  const T *rho = A.q[0], *e = A.q[1];
  const idx_t c = lin(G, i, j, k);
  const int id[3] = {i, j, k};
  auto in_range = [&](int d, int a, int b, int cc) {
    return a >= A.flo[d][0] && a < A.fhi[d][0] && b >= A.flo[d][1] && b < A.fhi[d][1] && cc >= A.flo[d][2] &&
           cc < A.fhi[d][2];
  };
  const bool comp =
      own && i >= cb.lo[0] && i < cb.hi[0] && j >= cb.lo[1] && j < cb.hi[1] && k >= cb.lo[2] && k < cb.hi[2];
  const T xc[3] = {xcen<T>(G, 0, i), xcen<T>(G, 1, j), xcen<T>(G, 2, k)};
  // distance of the cell whose coordinate along d is xd (the others the cell's)
  auto dist = [&](int d, T xd) -> T {
    const T x = d == 0 ? xd : xc[0], y = d == 1 ? xd : xc[1], z = d == 2 ? xd : xc[2];
    return qsqrt(fmav<T>(x, x, fmav<T>(y, y, fmav<T>(z, z, eps2))));
  };
  // the face between cells m (below) and u (above) along d
  auto kicked = [&](T vf, T drm, T dem, T dru, T deu, T xm, T xu, T dm, T du) -> T {
    const T rface = fmav<T>(T(0.5), drm + dru, rho0);
    const T gradp = qdiv(gm1 * (deu - dem), dx * rface);
    const T gradphi = qdiv(GM * (xu + xm), dm * du * (dm + du));
    return fmav<T>(-h, gradp + gradphi, vf);
  };
  const T drc = rho[c], dec = e[c];
  const T dcen = dist(0, xc[0]);
  T vlo[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const idx_t s = dstride(G, d);
    vlo[d] = A.vin[d][c];
    if (inb && in_range(d, i, j, k)) {
      const T xm = xcen<T>(G, d, id[d] - 1);
      vlo[d] = kicked(vlo[d], rho[c - s], e[c - s], drc, dec, xm, xc[d], dist(d, xm), dcen);
    }
    if (own) A.v[d][c] = vlo[d];
  }
  const T vhx = from_right(vlo[0]);
  if (comp) {
    T divv = T(0) + (vhx - vlo[0]);
#pragma unroll
    for (int d = 1; d < 3; ++d) {
      const idx_t s = dstride(G, d);
      T vhi = A.vin[d][c + s];
      if (in_range(d, id[0], id[1] + (d == 1), id[2] + (d == 2))) {
        const T xu = xcen<T>(G, d, id[d] + 1);
        vhi = kicked(vhi, drc, dec, rho[c + s], e[c + s], xc[d], xu, dcen, dist(d, xu));
      }
      divv += vhi - vlo[d];
    }
    const T dt = (T)(A.cfac * A.dtp[0]);
    const T a = T(0.5) * (T)P.gm1 * dt * qdiv(divv, dx);
    A.eo[c] = qdiv(fmav<T>(dec, T(1) - a, -(T(2) * a * (T)P.e0)), T(1) + a);
  }
}

// ------------------------------------------------- artificial viscosity

template <typename T>
struct ViscArgs {
  int lo[3], hi[3];          // union of the ranges below
  int elo[3], ehi[3];        // cells whose energy changes
  int flo[3][3], fhi[3][3];  // [normal dir][dim] faces that change
  const T *rho;
  T *e;
  const T *v[3];
  T *vn[3];                  // new face velocities
  const double *dtp;
  double fac;
};

// Von Neumann-Richtmyer viscosity of ZEUS (Stone & Norman 1992) as the
// SubStep2 that the staging list of Sect. 3.3 names: per dimension d and cell
// c, dv = v_d(high face) - v_d(low face) and q_d = C2 rho dv^2 where dv < 0,
// else 0; e -= dt sum_d q_d dv / dx; v_d(face) -= dt (q_d(c) - q_d(c-1)) /
// (dx rho_face).  All from the values before the stage: the new velocities go
// to vn.  On level 0 the boundary faces (the injection face, walls under bc 2)
// keep their values, and cells and faces past the boundary read its ghosts.
template <typename T, int BC>
__global__ void __launch_bounds__(BX * BY) k_visc(Geo G, Phys P, ViscArgs<T> A) {
  int id[3];
  if (!thread_cell_flat(Box{{A.lo[0], A.lo[1], A.lo[2]}, {A.hi[0], A.hi[1], A.hi[2]}}, id[0], id[1], id[2])) return;
  const T dt = (T)(A.fac * A.dtp[0]);
  const T c2 = (T)P.visc, rho0 = (T)P.rho0, dx = (T)G.dx;
  auto rho_at = [&](int i, int j, int k) -> T { return BC ? cread<BC>(A.rho, G, i, j, k) : A.rho[lin(G, i, j, k)]; };
  auto v_at = [&](int d, int i, int j, int k) -> T {
    return BC ? fread_bc<BC>(A.v[d], G, d, i, j, k) : A.v[d][lin(G, i, j, k)];
  };
  // q_d and dv_d of the cell at p
  auto qd = [&](int d, const int *p, T &dv) -> T {
    const T lo = v_at(d, p[0], p[1], p[2]);
    const T hi = v_at(d, p[0] + (d == 0), p[1] + (d == 1), p[2] + (d == 2));
    dv = hi - lo;
    return dv < T(0) ? c2 * (rho0 + rho_at(p[0], p[1], p[2])) * dv * dv : T(0);
  };
  const idx_t c = lin(G, id[0], id[1], id[2]);
  bool ecell = true;
#pragma unroll
  for (int e = 0; e < 3; ++e) ecell = ecell && id[e] >= A.elo[e] && id[e] < A.ehi[e];
  if (ecell) {
    T de = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T dv;
      const T q = qd(d, id, dv);
      de += q * dv;
    }
    A.e[c] = A.e[c] - qdiv(dt * de, dx);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    bool in = true;
#pragma unroll
    for (int e = 0; e < 3; ++e) in = in && id[e] >= A.flo[d][e] && id[e] < A.fhi[d][e];
    if (!in) continue;
    const T vold = A.v[d][c];
    T vnew = vold;
    const bool fixed = BC && ((d == 0 && id[0] == G.n[0]) ||
                              (BC == 2 && d > 0 && (id[d] == 0 || id[d] == G.n[d])));
    if (!fixed) {
      int m[3] = {id[0] - (d == 0), id[1] - (d == 1), id[2] - (d == 2)};
      T dvc, dvm;
      const T qc = qd(d, id, dvc), qm = qd(d, m, dvm);
      const T rface = rho0 + T(0.5) * (rho_at(m[0], m[1], m[2]) + rho_at(id[0], id[1], id[2]));
      vnew = vold - qdiv(dt * (qc - qm), dx * rface);
    }
    A.vn[d][c] = vnew;
  }
}

template <typename T>
__global__ void __launch_bounds__(BX * BY) k_copy_faces(Geo G, Box b, T *dst, const T *src) {
  int i, j, k;
  if (!thread_cell_flat(b, i, j, k)) return;
  const idx_t c = lin(G, i, j, k);
  dst[c] = src[c];
}

// ------------------------------------------------------------ compression

template <typename T>
struct CellArgs {
  Box b;
  T *e;
  const T *v[3];
  const double *dtp;
  double fac;
  Scal *log;                 // non-null: clear log->smax and log a pending force (first block)
  const double *part;        // the force partials: three planes of npart values
  int npart;
  double *flog;
};

// Compressional heating (SubStep3): e <- e (1 - a) / (1 + a),
// a = (gamma - 1) dt div(v) / 2; for the departure de = e - e0:
// de <- (de (1 - a) - 2 a e0) / (1 + a).
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_compress(Geo G, Phys P, CellArgs<T> A) {
  int i, j, k;
  if (!thread_cell_flat(A.b, i, j, k)) return;
  const T dt = (T)(A.fac * A.dtp[0]);
  const idx_t c = lin(G, i, j, k);
  const T divv = qdiv((A.v[0][c + 1] - A.v[0][c]) + (A.v[1][c + G.sy] - A.v[1][c]) +
                           (A.v[2][c + G.sz] - A.v[2][c]),
                       (T)G.dx);
  const T a = T(0.5) * (T)P.gm1 * dt * divv;
  const T de = A.e[c];
  A.e[c] = qdiv(de * (T(1) - a) - T(2) * a * (T)P.e0, T(1) + a);
}

template <int NT>
__device__ void log_pending_body(const double *part, int n, Scal *S, double *flog);

// The same on level 0 with two adjacent cells per lane (even row length; the
// box's x range counts pairs): every field moves as one 8- or 16-byte access.
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_compress2(Geo G, Phys P, CellArgs<T> A) {
  using V = typename lanes_of<T, 2>::type;
  int p, j, k;
  if (thread_cell_flat(A.b, p, j, k)) {
    const T dt = (T)(A.fac * A.dtp[0]);
    const idx_t c = lin(G, 2 * p, j, k);
    const V vx0 = gldv<V>(A.v[0], c);
    V vx1;
    vx1.x = vx0.y;
    vx1.y = gld(A.v[0], c + 2);
    const V divv = qdiv((vx1 - vx0) + (gldv<V>(A.v[1], c + (idx_t)G.sy) - gldv<V>(A.v[1], c)) +
                            (gldv<V>(A.v[2], c + (idx_t)G.sz) - gldv<V>(A.v[2], c)),
                        V((T)G.dx));
    const V a = T(0.5) * (T)P.gm1 * dt * divv;
    const V de = gldv<V>(A.e, c);
    gstv<V>(A.e, c, qdiv(de * (T(1) - a) - T(2) * a * (T)P.e0, T(1) + a));
  }
  if (A.log && blockIdx.x == 0) {
    // the kick of this step has read the slots: clear them for this step's
    // end-of-step pass, and log the force of the last step's state
    for (int q = threadIdx.y * BX + threadIdx.x; q < NSLOT; q += BX * BY) A.log->smax[q] = 0ull;
    log_pending_body<BX * BY>(A.part, A.npart, A.log, A.flog);
  }
}

// ---------------------------------------------------- diffusion + heat

template <typename T>
struct DiffArgs {
  Box b;
  const T *rho, *e;
  T *eo;
  const double *hw;
  int hw_n[3], hw_lo[3];  // weight box extent and its first active index per dimension
  const double *dtp;
  double fac;
  int do_diff, do_heat;
  Scal *clear;  // non-null (level 0 after a fused kick and compression): the first block clears clear->smax
};

// departure of e/rho from e0/rho0
template <typename T>
__device__ __forceinline__ T dtemp(T dr, T de, T rho0, T e0) {
  return qdiv(rho0 * de - e0 * dr, rho0 * (rho0 + dr));
}

// Thermal diffusion (eqs. 19-22, energy flux down the gradient of e/rho with
// coefficient chi rho0) and heat release L dt w_c / dx^3 (Sect. 3.4), on a
// finer level (its ghost shell holds every neighbour).
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_diffuse_heat(Geo G, Phys P, DiffArgs<T> A) {
  int i, j, k;
  if (!thread_cell_flat(A.b, i, j, k)) return;
  const T dt = (T)(A.fac * A.dtp[0]);
  const T rho0 = (T)P.rho0, e0 = (T)P.e0;
  const idx_t c = lin(G, i, j, k);
  const T dec = A.e[c];
  T en = dec;
  if (A.do_diff) {
    const T Tc = dtemp(A.rho[c], dec, rho0, e0);
    T lap = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const idx_t s = dstride(G, d);
      const T Tm = dtemp(A.rho[c - s], A.e[c - s], rho0, e0);
      const T Tp = dtemp(A.rho[c + s], A.e[c + s], rho0, e0);
      lap += (Tp - Tc) - (Tc - Tm);
    }
    en = dec + qdiv(dt * (T)(P.chi * P.rho0) * lap, (T)(G.dx * G.dx));
  }
  if (A.do_heat && A.hw_n[0] > 0) {
    // quadrant: the entries beyond a mirror plane are the images of the
    // level's cells and are heated as their cells are
    const int jj = (G.anch[1] && j < 0) ? -1 - j : j, kk = (G.anch[2] && k < 0) ? -1 - k : k;
    const int a = i - A.hw_lo[0], b = jj - A.hw_lo[1], d = kk - A.hw_lo[2];
    if (a >= 0 && b >= 0 && d >= 0 && a < A.hw_n[0] && b < A.hw_n[1] && d < A.hw_n[2] && i >= 0 && jj >= 0 &&
        kk >= 0 && i < G.n[0] && jj < G.n[1] && kk < G.n[2]) {
      const double w = A.hw[((long)d * A.hw_n[1] + b) * A.hw_n[0] + a];
      if (w != 0.0) en += (T)(P.L * (A.fac * A.dtp[0]) * w / (G.dx * G.dx * G.dx));
    }
  }
  A.eo[c] = en;
}

// The same on level 0, whose boundary conditions it applies on read, with two
// adjacent cells per lane (level-0 rows have an even length; the box's x
// range counts pairs): the pair's own fields and its y and z neighbours move
// as 8- or 16-byte accesses, the x neighbours of the pair are the other cell
// of the pair and one cell on each side.
template <typename T, int BC>
__device__ __forceinline__ void diffuse_heat2_body(Geo G, Phys P, DiffArgs<T> A, Blk bk) {
  using V = typename lanes_of<T, 2>::type;
  int p, j, k;
  const bool ok = thread_cell_flat(A.b, p, j, k, bk);
  if (A.clear && bk.id == 0) {
    // the kick of this step has read the slots: clear them for this step's
    // end-of-step pass
    for (int q = threadIdx.y * BX + threadIdx.x; q < NSLOT; q += BX * BY) A.clear->smax[q] = 0ull;
  }
  if (!ok) return;
  const int i = 2 * p;
  const T dt = (T)(A.fac * A.dtp[0]);
  const T rho0 = (T)P.rho0, e0 = (T)P.e0;
  const idx_t c = lin(G, i, j, k);
  const V de = gldv<V>(A.e, c);
  V en = de;
  if (A.do_diff) {
    auto tv = [&](V r, V e) -> V { return qdiv(rho0 * e - e0 * r, rho0 * (rho0 + r)); };
    const V Tc = tv(gldv<V>(A.rho, c), de);
    // x: past x_max (and past x_min under bc 2) the background, else the
    // nearest active cell (as k_diffuse_heat)
    V Tl, Tr;
    Tl.y = Tc.x;
    Tr.x = Tc.y;
    if (BC == 2 && i == 0) {
      Tl.x = T(0);
    } else {
      const idx_t cm = i > 0 ? c - 1 : c;
      Tl.x = dtemp(gld(A.rho, cm), gld(A.e, cm), rho0, e0);
    }
    Tr.y = i + 1 == G.n[0] - 1 ? T(0) : dtemp(gld(A.rho, c + 2), gld(A.e, c + 2), rho0, e0);
    V lap = V(0);
    lap += (Tr - Tc) - (Tc - Tl);
#pragma unroll
    for (int d = 1; d < 3; ++d) {
      const int id = d == 1 ? j : k;
      const idx_t s = dstride(G, d);
      const idx_t cm = id > 0 ? c - s : c, cp = id < G.n[d] - 1 ? c + s : c;
      const V Tm = tv(gldv<V>(A.rho, cm), gldv<V>(A.e, cm)), Tp = tv(gldv<V>(A.rho, cp), gldv<V>(A.e, cp));
      lap += (Tp - Tc) - (Tc - Tm);
    }
    en = de + qdiv(dt * (T)(P.chi * P.rho0) * lap, V((T)(G.dx * G.dx)));
  }
  if (A.do_heat && A.hw_n[0] > 0) {
    const int b = j - A.hw_lo[1], d = k - A.hw_lo[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int a = i + q - A.hw_lo[0];
      if (a >= 0 && b >= 0 && d >= 0 && a < A.hw_n[0] && b < A.hw_n[1] && d < A.hw_n[2]) {
        const double w = A.hw[((long)d * A.hw_n[1] + b) * A.hw_n[0] + a];
        if (w != 0.0) en[q] += (T)(P.L * (A.fac * A.dtp[0]) * w / (G.dx * G.dx * G.dx));
      }
    }
  }
  gstv<V>(A.eo, c, en);
}

template <typename T, int BC>
__global__ void __launch_bounds__(BX * BY) k_diffuse_heat2(Geo G, Phys P, DiffArgs<T> A) {
  diffuse_heat2_body<T, BC>(G, P, A, grid_blk());
}

// -------------------------------------------------------------- transport

template <typename T>
struct PassArgs {
  Box b;
  const T *qi[NQ];
  T *qo[NQ];
  const T *v[3];     // face velocity departures after the first kick
  const double *dtp;
  double fac;
  T *acc;            // this level's frontier accumulators (fine levels) or null
  const T *facc;     // the finer level's accumulators (coarse levels) or null
  int fn[3];         // finer level's active cells (accumulator strides)
};

// Cell of the x pass at row (j, k) and x: false where level 0's boundary
// holds the background (beyond x_max; under bc 2 beyond both flow ends), else
// the cell to read (the nearest active one under bc 1).
template <int BC>
__device__ __forceinline__ bool xcell_at(const Geo &G, int x, int j, int k, idx_t &c) {
  if (BC) {
    if (x >= G.n[0] || (BC == 2 && x < 0)) return false;
    x = x < 0 ? 0 : x;
  }
  c = lin(G, x, j, k);
  return true;
}

// Wave-tiled form of the x pass.  A wave holds 64 consecutive cells of one
// row, of which lanes 2..61 own their cell (tiles overlap by 4 cells): every
// lane forms the specific value of its cell and the limited difference there
// once, takes its neighbours' through lane shifts, computes the transfer
// through its left face, and the owning lanes take the right face's transfer
// from the lane above.  Arithmetic and its order are those of k_pass.
constexpr int XT = 60;

__host__ __device__ inline Box xtile_box(const Box &b) {
  Box v = b;
  const int ex = b.hi[0] - b.lo[0];
  v.lo[0] = 0;
  v.hi[0] = ex > 0 ? ((ex + XT - 1) / XT) * BX : 0;
  return v;
}

template <typename T, int BC>
__global__ void __launch_bounds__(BX * BY) k_xpass(Geo G, Phys P, PassArgs<T> A) {
  int iv, j, k;
  if (!thread_cell(xtile_box(A.b), iv, j, k)) return;
  const int lane = threadIdx.x;
  const int x = A.b.lo[0] - 2 + (iv / BX) * XT + lane;
  // lanes past the last cell's neighbours read that neighbour (never used)
  const int xl = min(x, A.b.hi[0] + 1);
  const bool owner = lane >= 2 && lane < 2 + XT && x < A.b.hi[0];
  const T dt = (T)(A.fac * A.dtp[0]);
  const T dx = (T)G.dx;
  const T mfac = dt * dx * dx, ivol = T(1) / (dx * dx * dx);
  const T rho0 = (T)P.rho0;
  const T vb = (T)vback(P, 0);
  idx_t c;
  const bool in = xcell_at<BC>(G, xl, j, k, c);
  // momenta tangential to x beyond a flow end under bc 2: the mirror cell's
  idx_t ct = c;
  bool int_ = in;
  if (BC == 2 && !in) {
    ct = lin(G, mirror_idx(xl, G.n[0]), j, k);
    int_ = true;
  }
  const T dr = in ? gld(A.qi[0], c) : T(0);
  const T irr = qdiv(T(1), rho0 * (rho0 + dr));
  // velocity departure on the left face (faces lo..hi are the ones used)
  const T da = gld(A.v[0], lin(G, clampi(x, A.b.lo[0], A.b.hi[0]), j, k));
  const T a = vb + da, nu = a * (dt / dx);
  const T hl = T(0.5) * (T(1) - nu), hh = T(0.5) * (T(1) + nu);
  const T M0 = rho0 * vb * mfac;
  auto left_face = [&](T sv) -> T {
    const T sm = from_left(sv), sp = from_right(sv);
    const T d = vleer(sp - sv, sv - sm);
    const T dm = from_left(d);
    const T lo = sm + dm * hl, hi = sv - d * hh;
    return a > T(0) ? lo : hi;
  };
  const T dM = (rho0 * da + left_face(dr) * a) * mfac;
  const T M = M0 + dM;

  // flux matching on the frontier of the finer level (its 4 faces over its 2
  // sub-cycles replace this level's transfer) and this level's own frontier
  bool fine_face = false;
  int side = 0;
  long fbase = 0, fnt = 0;
  if (A.facc) {
    const int a1 = j - G.co[1], a2 = k - G.co[2];
    const int lo = G.co[0], hi = G.co[0] + G.cn[0];
    if (a1 >= 0 && a2 >= 0 && a1 < G.cn[1] && a2 < G.cn[2] && (x == lo || x == hi)) {
      fine_face = true;
      side = (x == hi);
      fnt = (long)A.fn[1] * A.fn[2];
      fbase = (long)(2 * a2) * A.fn[1] + 2 * a1;
    }
  }
  long acc_i = -1, acc_nt = 0;
  int acc_side = -1;
  if (A.acc && owner && j >= 0 && k >= 0 && j < G.n[1] && k < G.n[2] &&
      (x == 0 || x == G.n[0] - 1)) {
    acc_nt = (long)G.n[1] * G.n[2];
    acc_i = (long)k * G.n[1] + j;
    acc_side = (x == 0) ? 0 : 1;
  }
  const idx_t co = lin(G, x, j, k);
  auto finish = [&](int m, T own, T FL) {
    if (fine_face) {
      const T *f = A.facc + ((long)side * NQ + m) * fnt + fbase;
      FL = (f[0] + f[1]) + (f[A.fn[1]] + f[A.fn[1] + 1]);
    }
    const T FR = from_right(FL);
    if (acc_side == 0) A.acc[((long)0 * NQ + m) * acc_nt + acc_i] += FL;
    if (acc_side == 1) A.acc[((long)1 * NQ + m) * acc_nt + acc_i] += FR;
    if (owner) gst(A.qo[m], co, own - (FR - FL) * ivol);
  };
  finish(0, dr, dM);

#pragma unroll 1
  for (int m = 1; m < NQ; ++m) {
    T sv, own;
    if (m >= 2) {
      // momentum P = rho v of a face velocity: its specific value is v itself
      const int d = (m - 2) >> 1;
      const idx_t off = (m & 1) ? dstride(G, d) : 0;
      if (d == 0) sv = in ? gld(A.v[d], c + off) : T(0);
      else sv = int_ ? gld(A.v[d], ct + off) : T(0);
      own = rho0 * sv + dr * ((T)vback(P, d) + sv);
    } else {
      const T dq = in ? gld(A.qi[m], c) : T(0);
      sv = (rho0 * dq - (T)qback(P, m) * dr) * irr;
      own = dq;
    }
    finish(m, own, (T)sback(P, m) * dM + left_face(sv) * M);
  }
}

// Row form of the x pass for level 0 when a row has at most 64 R cells and R
// divides it: one wave holds a whole row, lane l the R consecutive cells
// R l .. R l + R - 1, so the neighbours of a cell are in its own lane or, at
// the lane's ends, in the adjacent lane (one lane shift per exchanged value
// for R cells).  The boundary conditions give what lies beyond the row: at
// x_min the outflow copy (the specific value of cell -1 is that of cell 0,
// the limited difference there is zero); at x_max, cells n, n+1 hold zero
// departures and the injection face carries no departure transfer.  Cells
// past n inside the wave are those ghost cells.  Arithmetic and its order are
// those of k_xpass.
__host__ __device__ inline Box xrow_box(const Box &b) {
  Box v = b;
  v.lo[0] = 0;
  v.hi[0] = (b.hi[0] > b.lo[0]) ? BX : 0;
  return v;
}

// lane shift with a fill value for the lane that has no source
template <int CTRL>
__device__ __forceinline__ float dpp_fill(float v, float fill) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                               __builtin_bit_cast(int, v), CTRL, 0xf, 0xf,
                                                               false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_fill(double v, double fill) {
  const long long b = __builtin_bit_cast(long long, v), f = __builtin_bit_cast(long long, fill);
  const int lo = __builtin_amdgcn_update_dpp((int)f, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// the value of the cell before each of the lane's R cells (fill for cell -1)
template <typename T, int R>
__device__ __forceinline__ void row_left(const T (&v)[R], T (&out)[R], T fill) {
  out[0] = dpp_fill<DPP_WAVE_SHR1>(v[R - 1], fill);
#pragma unroll
  for (int r = 1; r < R; ++r) out[r] = v[r - 1];
}

// the value of the cell after each of the lane's R cells (fill past the wave)
template <typename T, int R>
__device__ __forceinline__ void row_right(const T (&v)[R], T (&out)[R], T fill) {
#pragma unroll
  for (int r = 0; r + 1 < R; ++r) out[r] = v[r + 1];
  out[R - 1] = dpp_fill<DPP_WAVE_SHL1>(v[0], fill);
}

// R consecutive entries from an R-aligned index (R a power of two)
template <typename T, int R>
__device__ __forceinline__ void row_load(const T *p, idx_t c, T (&out)[R]) {
  typedef T vec __attribute__((ext_vector_type(R)));
  const vec w = *reinterpret_cast<const vec *>(reinterpret_cast<const char *>(p) +
                                                (unsigned)c * (unsigned)sizeof(T));
#pragma unroll
  for (int r = 0; r < R; ++r) out[r] = w[r];
}

template <typename T, int R>
__device__ __forceinline__ void row_store(T *p, idx_t c, const T (&v)[R]) {
  typedef T vec __attribute__((ext_vector_type(R)));
  vec w;
#pragma unroll
  for (int r = 0; r < R; ++r) w[r] = v[r];
  *reinterpret_cast<vec *>(reinterpret_cast<char *>(p) + (unsigned)c * (unsigned)sizeof(T)) = w;
}

// x pass of one level-0 row held by one wave, R cells per lane (lane l owns
// cells R l .. R l + R - 1; lanes past the row end hold zero departures, the
// inflow state beyond x_max): from the row's density and left-face velocity
// departures (dr, da, set by the caller) the mass transfers through every left
// face, then per quantity its transfers and updated departures.
template <typename T, int R>
struct XRow {
  T dr[R], da[R];
  T dt, dx, rho0, ivol, mfac, M0, irr[R], a[R], hl[R], hh[R], dM[R], M[R];

  // face velocities and Courant numbers of the row
  __device__ __forceinline__ void flow(const Geo &G, const Phys &P, T dt_) {
#pragma clang fp contract(off)
    dt = dt_;
    dx = (T)G.dx;
    mfac = dt * dx * dx;
    const T cour = dt / dx;
    ivol = T(1) / (dx * dx * dx);
    rho0 = (T)P.rho0;
    const T vb = (T)vback(P, 0);
    M0 = rho0 * vb * mfac;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      a[r] = vb + da[r];
      const T nu = a[r] * cour;
      hl[r] = fmav<T>(T(-0.5), nu, T(0.5));  // (1 -+ nu)/2, exact halvings of the rounded 1 -+ nu
      hh[r] = fmav<T>(T(0.5), nu, T(0.5));
    }
  }
  // the mass transfers through the left faces (departures dm_)
  __device__ __forceinline__ void take_mass(const T (&dm_)[R]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      dM[r] = dm_[r];
      M[r] = M0 + dM[r];
    }
  }
  __device__ __forceinline__ void mass() {
#pragma clang fp contract(off)
    T fv[R], dm_[R];
    left_faces(dr, fv);
#pragma unroll
    for (int r = 0; r < R; ++r) dm_[r] = fmav<T>(fv[r], a[r], rho0 * da[r]) * mfac;
    take_mass(dm_);
  }
  __device__ __forceinline__ void recip() {
#pragma clang fp contract(off)
#pragma unroll
    for (int r = 0; r < R; ++r) irr[r] = qdiv(T(1), rho0 * (rho0 + dr[r]));
  }
  __device__ __forceinline__ void begin(const Geo &G, const Phys &P, T dt_) {
    flow(G, P, dt_);
    recip();
    mass();
  }
  // left-face value of the upwind van Leer reconstruction of s, per cell
  __device__ __forceinline__ void left_faces(const T (&sv)[R], T (&fv)[R]) const {
#pragma clang fp contract(off)
    T sl[R], sr[R], d[R], dl[R];
    row_left<T, R>(sv, sl, sv[0]);
    row_right<T, R>(sv, sr, T(0));
#pragma unroll
    for (int r = 0; r < R; ++r) d[r] = vleer(sr[r] - sv[r], sv[r] - sl[r]);
    row_left<T, R>(d, dl, T(0));
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // both upwind values, then a select (a branch per face costs more)
      const T lo = fmav<T>(dl[r], hl[r], sl[r]), hi = fmav<T>(-d[r], hh[r], sv[r]);
      fv[r] = a[r] > T(0) ? lo : hi;
    }
  }
  // specific value and own departure of quantity m >= 1 from its input: the
  // energy departure (m = 1) or the face velocity whose momentum it is
  __device__ __forceinline__ void quantity(const Phys &P, int m, const T (&in)[R], T (&sv)[R],
                                           T (&own)[R]) const {
#pragma clang fp contract(off)
    if (m >= 2) {
      // momentum P = rho v of a face velocity: its specific value is v itself
      const T vbd = (T)vback(P, (m - 2) >> 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        sv[r] = in[r];
        own[r] = fmav<T>(dr[r], vbd + sv[r], rho0 * sv[r]);
      }
    } else {
      const T q0 = (T)qback(P, m);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        sv[r] = fmav<T>(rho0, in[r], -(q0 * dr[r])) * irr[r];
        own[r] = in[r];
      }
    }
  }
  // transfers of quantity m through the left faces
  __device__ __forceinline__ void transfers(const Phys &P, int m, const T (&sv)[R], T (&F)[R]) const {
#pragma clang fp contract(off)
    T fv[R];
    left_faces(sv, fv);
    const T s0 = (T)sback(P, m);
#pragma unroll
    for (int r = 0; r < R; ++r) F[r] = fmav<T>(s0, dM[r], fv[r] * M[r]);
  }
  // updated departures from the left-face transfers (none through x_max)
  __device__ __forceinline__ void update(const T (&own)[R], const T (&FL)[R], T (&out)[R]) const {
#pragma clang fp contract(off)
    T FR[R];
    row_right<T, R>(FL, FR, T(0));
#pragma unroll
    for (int r = 0; r < R; ++r) out[r] = fmav<T>(-(FR[r] - FL[r]), ivol, own[r]);
  }
};

// input of quantity m >= 1 of the row of level 0 at index c (first cell of the
// lane): the energy departure, or the face velocity whose momentum it is (the
// right x face from the next lane's left face, zero past x_max)
template <typename T, int R>
__device__ __forceinline__ void xrow_input(const Geo &G, const PassArgs<T> &A, int m, idx_t c, bool live,
                                           const T (&da)[R], T (&in)[R]) {
  if (m == 3) {
    row_right<T, R>(da, in, T(0));
    return;
  }
  if (m == 2) {
#pragma unroll
    for (int r = 0; r < R; ++r) in[r] = da[r];
    return;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) in[r] = T(0);
  if (!live) return;
  if (m == 1) {
    row_load<T, R>(A.qi[1], c, in);
  } else {
    const int d = (m - 2) >> 1;
    row_load<T, R>(A.v[d], c + ((m & 1) ? dstride(G, d) : 0), in);
  }
}

template <typename T, int R>
__global__ void __launch_bounds__(BX * BY) k_xrow(Geo G, Phys P, PassArgs<T> A) {
  int lane, j, k;
  if (!thread_cell(xrow_box(A.b), lane, j, k)) return;
  const int n = G.n[0];
  const int x0 = R * lane;
  const bool live = x0 < n;  // the lane's cells are active (R divides n)
  const idx_t c = lin(G, x0, j, k);
  XRow<T, R> X;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    X.dr[r] = T(0);
    X.da[r] = T(0);
  }
  if (live) {
    row_load<T, R>(A.qi[0], c, X.dr);
    row_load<T, R>(A.v[0], c, X.da);  // left faces x0 .. x0+R-1 (all <= n - 1)
  }
  X.begin(G, P, (T)(A.fac * A.dtp[0]));
  // flux matching on the frontier of the finer level
  const bool ov = A.facc && j - G.co[1] >= 0 && k - G.co[2] >= 0 && j - G.co[1] < G.cn[1] && k - G.co[2] < G.cn[2];
  const int flo = G.co[0], fhi = G.co[0] + G.cn[0];
  const long fnt = (long)A.fn[1] * A.fn[2];
  const long fbase = (long)(2 * (k - G.co[2])) * A.fn[1] + 2 * (j - G.co[1]);
  auto finish = [&](int m, const T (&own)[R], T (&FL)[R]) {
    if (ov) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = x0 + r;
        if (x == flo || x == fhi) {
          const T *f = A.facc + ((long)(x == fhi) * NQ + m) * fnt + fbase;
          FL[r] = (f[0] + f[1]) + (f[A.fn[1]] + f[A.fn[1] + 1]);
        }
      }
    }
    T out[R];
    X.update(own, FL, out);
    if (live) row_store<T, R>(A.qo[m], c, out);
  };
  {
    T F[R];
#pragma unroll
    for (int r = 0; r < R; ++r) F[r] = X.dM[r];
    finish(0, X.dr, F);
  }

#pragma unroll 1
  for (int m = 1; m < NQ; ++m) {
    T in[R], sv[R], own[R], F[R];
    xrow_input<T, R>(G, A, m, c, live, X.da, in);
    X.quantity(P, m, in, sv, own);
    X.transfers(P, m, sv, F);
    finish(m, own, F);
  }
}

// Row form of the x pass on a finer level (no boundary conditions: the
// stored row holds the ghost cells): one wave per row, lane l the R cells
// xs + R l .. xs + R l + R - 1 from the R-aligned start xs <= lo - 2, so that
// the wave covers the cells [lo - 2, hi + 2) every update of [lo, hi) reads.
// The arithmetic is XRow's (that of k_xpass); the cells outside [lo, hi) are
// computed and not written, and the frontier transfers are taken (the finer
// level's sums at the covered box's faces) and accumulated (this level's own
// at faces 0 and n) as k_xpass does.
template <typename T, int R>
__global__ void __launch_bounds__(BX * BY) k_xrow_fine(Geo G, Phys P, PassArgs<T> A, int xs) {
  int lane, j, k;
  if (!thread_cell_flat(xrow_box(A.b), lane, j, k)) return;
  const int n = G.n[0];
  const int x0 = xs + R * lane;
  // the lane's cells lie within the row's padded storage, which starts px
  // entries before x = 0 (loads past it are not made; the padding is read as
  // the neighbours of cells outside the range the update reads)
  const int px = (int)(G.off - (long)G.g * (G.sy + G.sz));
  const bool live = x0 >= -px && x0 + R <= (int)G.sy - px;
  const idx_t c = lin(G, x0, j, k);
  XRow<T, R> X;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    X.dr[r] = T(0);
    X.da[r] = T(0);
  }
  if (live) {
    row_load<T, R>(A.qi[0], c, X.dr);
    row_load<T, R>(A.v[0], c, X.da);
  }
  X.begin(G, P, (T)(A.fac * A.dtp[0]));
  const bool ov = A.facc && j - G.co[1] >= 0 && k - G.co[2] >= 0 && j - G.co[1] < G.cn[1] && k - G.co[2] < G.cn[2];
  const int flo = G.co[0], fhi = G.co[0] + G.cn[0];
  const long fnt = (long)A.fn[1] * A.fn[2];
  const long fbase = (long)(2 * (k - G.co[2])) * A.fn[1] + 2 * (j - G.co[1]);
  const bool accrow = A.acc && j >= 0 && k >= 0 && j < G.n[1] && k < G.n[2];
  const long acc_nt = (long)G.n[1] * G.n[2], acc_i = (long)k * G.n[1] + j;
  // the lane's cells all inside the updated range: one vector store
  const bool inner = x0 >= A.b.lo[0] && x0 + R <= A.b.hi[0];
  auto finish = [&](int m, const T (&own)[R], T (&FL)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int x = x0 + r;
      if (ov && (x == flo || x == fhi)) {
        const T *f = A.facc + ((long)(x == fhi) * NQ + m) * fnt + fbase;
        FL[r] = (f[0] + f[1]) + (f[A.fn[1]] + f[A.fn[1] + 1]);
      }
      if (accrow && (x == 0 || x == n)) A.acc[((long)(x == n) * NQ + m) * acc_nt + acc_i] += FL[r];
    }
    T out[R];
    X.update(own, FL, out);
    if (inner) {
      row_store<T, R>(A.qo[m], c, out);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (x0 + r >= A.b.lo[0] && x0 + r < A.b.hi[0]) A.qo[m][c + r] = out[r];
    }
  };
  {
    T F[R];
#pragma unroll
    for (int r = 0; r < R; ++r) F[r] = X.dM[r];
    finish(0, X.dr, F);
  }

#pragma unroll 1
  for (int m = 1; m < NQ; ++m) {
    T in[R], sv[R], own[R], F[R];
    xrow_input<T, R>(G, A, m, c, live, X.da, in);
    X.quantity(P, m, in, sv, own);
    X.transfers(P, m, sv, F);
    finish(m, own, F);
  }
}

// Streaming form of the y and z passes.  A thread owns one column segment
// [c0, c1) along DIR (lanes along x, so every load is coalesced) and walks it
// once: each cell is loaded once (one iteration ahead of its use), each limited
// difference and each face transfer is computed once, and the cell is written
// as soon as its right face is known.  The eight quantities are split over two
// waves of the block: one moves rho, e, P-x, P+x, the other P-y, P+y, P-z, P+z
// (both compute the mass transfers they scale).  A lane may own W = 2 adjacent
// columns, whose cells then move as one 8- or 16-byte access.
template <typename T>
struct MarchArgs {
  int lo[3], hi[3];   // cells to update; DIR is the walked dimension
  int chunk;          // cells per segment
  const T *qi[NQ];
  T *qo[NQ];
  const T *v;         // face velocity departure normal to DIR
  const double *dtp;
  double fac;
  T *acc;
  const T *facc;
  int fn[3];
};

// Transported quantities of group GRP of NG (u = 0.. of the group; entries
// past the group's count are unused): two groups {e, P-x, P+x} and {P-y, P+y,
// P-z, P+z}, or four groups {e}, {P-x, P+x}, {P-y, P+y}, {P-z, P+z}.  Every
// group also transports the density (its mass transfers carry the others);
// the first one stores it.
// NG = 3 is the one group {e, P+y} of the neighbour row a fused z finish
// walks for the y faces of its first row.
constexpr int group_q(int NG, int GRP, int u) {
  return NG == 2 ? (GRP ? 4 + u : (u < 3 ? 1 + u : 1))
                 : (NG == 3 ? (u == 1 ? 5 : 1) : (GRP == 0 ? 1 : (u < 2 ? 2 * GRP + u : 1)));
}
constexpr int group_n(int NG, int GRP) { return NG == 2 ? (GRP ? 4 : 3) : (NG == 3 ? 2 : (GRP ? 2 : 1)); }

// Rows of a column read from the transported set (the y and z passes): the
// raw departures of row c (w[0] the density, w[1..] the group's quantities)
// through level 0's boundary rules.  bc 1 clamps c to the active range; bc 2:
// across a wall (DIR is y or z) every quantity takes its mirror image, and the
// two momenta normal to the wall swap and change sign.
template <typename T, typename V, int DIR, int BC, int GRP, int NG>
struct ColSrc {
  const T *rho;
  const T *qin[4];
  idx_t base, st;
  int n;
  __device__ __forceinline__ V ld(int u, int c) const {  // u < 0: the density
    constexpr bool walls = BC == 2;
    // group wg holds P-, P+ normal to DIR at u = pa, pa + 1
    constexpr int wg = NG == 2 ? 1 : (DIR == 1 ? 2 : 3);
    constexpr int pa = NG == 2 ? ((DIR == 1) ? 0 : 2) : 0;
    const T *q = u < 0 ? rho : qin[u];
    if (walls && (c < 0 || c >= n)) {
      // rows c0-2 .. c1+1 have a mirror image in the active range for n >= 2;
      // the row c1+2 fetched past the last one (never used) may not (n = 2)
      // and is kept in range
      const idx_t m = base + clampi(mirror_idx(c, n), 0, n - 1) * st;
      if (GRP == wg && (u == pa || u == pa + 1)) return -gldv<V>(qin[u ^ 1], m);
      return gldv<V>(q, m);
    }
    if (BC) c = clampi(c, 0, n - 1);
    return gldv<V>(q, base + c * st);
  }
  __device__ __forceinline__ void get(int c, V (&w)[5]) {
    w[0] = ld(-1, c);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (u < group_n(NG, GRP)) w[u + 1] = ld(u, c);
  }
};

// One column segment [c0, c1) of the quantity group GRP of NG at in-plane
// position (i, t), W adjacent columns per lane.  The rows come from src, in
// increasing order c0-2, c0-1, ..., each requested one iteration ahead of its
// use; lanes that are not live (past the row end) neither read nor write.
// FRONT: the level has frontier transfers (a finer level's sums to take, or
// its own to accumulate); without them the solver's transfers stand.
template <typename T, int DIR, int BC, int GRP, bool FRONT, int W, int NG, typename Src, typename Sink>
__device__ __forceinline__ void march_column(const Geo &G, const Phys &P, const MarchArgs<T> &A,
                                             int i, int t, int c0, int c1, Src &src, Sink &snk, bool live) {
  // the transfer through a segment's first face is formed before the walk and
  // again, by the segment below, inside it: with no implicit contraction and
  // the fused products written out, both give the same value, so the results
  // do not depend on where segments start
#pragma clang fp contract(off)
  static_assert(W == 1 || !FRONT, "frontier transfers are per column");
  using V = typename lanes_of<T, W>::type;  // the W adjacent columns of a lane
  constexpr int TD = (DIR == 1) ? 2 : 1;
  constexpr int T1 = (DIR == 0) ? 1 : 0;
  constexpr int T2 = (DIR == 2) ? 1 : 2;
  const T dt = (T)(A.fac * A.dtp[0]);
  const T dx = (T)G.dx;
  const T mfac = dt * dx * dx, ivol = T(1) / (dx * dx * dx), cour = dt / dx;
  const T rho0 = (T)P.rho0;
  const T vb = (T)vback(P, DIR);
  const T M0 = rho0 * vb * mfac;
  const idx_t st = dstride(G, DIR);
  int id3[3];
  id3[0] = i;
  id3[TD] = t;
  id3[DIR] = 0;
  const idx_t base = lin(G, id3[0], id3[1], id3[2]);
  auto cidx = [&](int c) -> idx_t {
    if (BC) c = clampi(c, 0, G.n[DIR] - 1);
    return base + c * st;
  };
  constexpr int mq[4] = {group_q(NG, GRP, 0), group_q(NG, GRP, 1), group_q(NG, GRP, 2), group_q(NG, GRP, 3)};
  constexpr int nq = group_n(NG, GRP);
  // the momenta across the wind (P-y .. P+z) have a zero background, and
  // only x carries a background velocity: those terms are dropped outright
  constexpr bool zq[4] = {mq[0] >= 4, mq[1] >= 4, mq[2] >= 4, mq[3] >= 4};
  constexpr bool wind = DIR == 0;
  T q0[4], sb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    q0[u] = (T)qback(P, mq[u]);
    sb[u] = (T)sback(P, mq[u]);
  }

  const int tv1 = id3[T1], tv2 = id3[T2];
  bool ov = false;
  long fbase = 0, fnt = 0;
  int flo = 0, fhi = 0;
  if (FRONT && A.facc) {
    const int a1 = tv1 - G.co[T1], a2 = tv2 - G.co[T2];
    if (a1 >= 0 && a2 >= 0 && a1 < G.cn[T1] && a2 < G.cn[T2]) {
      ov = true;
      fnt = (long)A.fn[T1] * A.fn[T2];
      fbase = (long)(2 * a2) * A.fn[T1] + 2 * a1;
      flo = G.co[DIR];
      fhi = G.co[DIR] + G.cn[DIR];
    }
  }
  const bool acc_col = FRONT && live && A.acc && tv1 >= 0 && tv2 >= 0 && tv1 < G.n[T1] && tv2 < G.n[T2];
  const long acc_nt = (long)G.n[T1] * G.n[T2];
  const long acc_i = (long)tv2 * G.n[T1] + tv1;
  // final transfer of quantity m through face f, given the solver's value
  auto fix = [&](int f, int m, V F) -> V {
    if constexpr (!FRONT) {
      return F;
    } else {
      if (ov && (f == flo || f == fhi)) {
        const T *a = A.facc + ((long)(DIR * 2 + (f == fhi)) * NQ + m) * fnt + fbase;
        F = (a[0] + a[1]) + (a[A.fn[T1]] + a[A.fn[T1] + 1]);
      }
      if (acc_col && f >= c0 && f < c1 && (f == 0 || f == G.n[DIR]))
        A.acc[((long)(DIR * 2 + (f != 0)) * NQ + m) * acc_nt + acc_i] += F;
      return F;
    }
  };
  // the face's weights hl = (1 - nu)/2, hh = (1 + nu)/2 are exact halvings
  auto upwind = [&](V sl, V dl, V sr, V dr, V a, V hl, V hh) -> V {
    const V lo = fmav<V>(dl, hl, sl), hi = fmav<V>(-dr, hh, sr);
    return a > T(0) ? lo : hi;
  };
  // numerator of the departure of quantity u's specific value from raw
  // departures (q, rho): times 1/(rho0 rho) it is the value
  auto numer = [&](int u, V q, V r) -> V { return zq[u] ? rho0 * q : fmav<V>(V(rho0), q, -(q0[u] * r)); };
  // limited difference at a cell of value s from its left neighbour's value sl
  // and its right neighbour's numerator and reciprocal (xr, ir): the right
  // difference takes the neighbour's value unrounded, the left one the values
  auto limited = [&](V xr, V ir, V s, V sl) -> V { return vleer(fmav<V>(xr, ir, -s), s - sl); };
  // Courant weights of a face: (1 -+ nu)/2, exact halvings of the rounded 1 -+ nu
  auto weights = [&](V a, V &hl, V &hh) {
    const V nu = a * cour;
    hl = fmav<V>(V(-0.5), nu, V(0.5));
    hh = fmav<V>(V(0.5), nu, V(0.5));
  };
  // velocity departure on face c (normal to DIR)
  auto face = [&](int c) -> V { return live ? gldv<V>(A.v, base + c * st) : V(0); };

  // window: departures of the specific values at c, c+1 (s0, s1; index 0 is
  // the density departure), limited difference at c (d0), transfer through
  // face c (F0); raw departures of cells c, c+1, c+2 (w0, w1, w2) and the
  // velocity departure on face c+1 (va), all fetched at least one iteration
  // ahead of their use
  V s0[5], s1[5], d0[5], F0[5], w0[5], w1[5], w2[5];
  V va;
  {
    // the density (u = 0) is its own value: numerator the raw departure,
    // reciprocal 1
    V rm2[5], rm1[5], sm2[5], sm1[5], x0[5], x1[5];
    src.get(c0 - 2, rm2);
    src.get(c0 - 1, rm1);
    src.get(c0, w0);
    src.get(c0 + 1, w1);
    const V ir_m2 = qdiv(V(1), rho0 * (rho0 + rm2[0])), ir_m1 = qdiv(V(1), rho0 * (rho0 + rm1[0]));
    const V ir_0 = qdiv(V(1), rho0 * (rho0 + w0[0])), ir_p1 = qdiv(V(1), rho0 * (rho0 + w1[0]));
    sm2[0] = rm2[0]; sm1[0] = rm1[0]; s0[0] = x0[0] = w0[0]; s1[0] = x1[0] = w1[0];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u >= nq) break;
      sm2[u + 1] = numer(u, rm2[u + 1], rm2[0]) * ir_m2;
      sm1[u + 1] = numer(u, rm1[u + 1], rm1[0]) * ir_m1;
      x0[u + 1] = numer(u, w0[u + 1], w0[0]);
      x1[u + 1] = numer(u, w1[u + 1], w1[0]);
      s0[u + 1] = x0[u + 1] * ir_0;
      s1[u + 1] = x1[u + 1] * ir_p1;
    }
    const V da = face(c0);
    const V a = wind ? vb + da : da;
    V hl, hh;
    weights(a, hl, hh);
    V dM = V(0), M = V(0);
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      if (u > nq) break;
      const V dm1 = limited(x0[u], u ? ir_0 : V(1), sm1[u], sm2[u]);
      d0[u] = limited(x1[u], u ? ir_p1 : V(1), s0[u], sm1[u]);
      const V fv = upwind(sm1[u], dm1, s0[u], d0[u], a, hl, hh);
      if (u == 0) {
        dM = fmav<V>(fv, a, rho0 * da) * mfac;
        M = wind ? M0 + dM : dM;
        F0[0] = GRP ? dM : fix(c0, 0, dM);  // the density belongs to the first group
      } else {
        F0[u] = fix(c0, mq[u - 1], zq[u - 1] ? fv * M : fmav<V>(V(sb[u - 1]), dM, fv * M));
      }
    }
    src.get(c0 + 2, w2);
    va = face(c0 + 1);
  }
  for (int c = c0; c < c1; ++c) {
    const idx_t ic = cidx(c);
    // next iteration's rows: cell c+3 and face c+2 (one row past the last
    // needed one, c1+1, is fetched and not used: no branch splits the body)
    V nn[5];
    src.get(c + 3, nn);
    const V vn = face(min(c + 2, c1));
    const V ir2 = qdiv(V(1), rho0 * (rho0 + w2[0]));
    V s2[5], x2[5];
    s2[0] = x2[0] = w2[0];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < nq) {
        x2[u + 1] = numer(u, w2[u + 1], w2[0]);
        s2[u + 1] = x2[u + 1] * ir2;
      }
    }
    const V da = va;
    const V a = wind ? vb + da : da;
    V hl, hh;
    weights(a, hl, hh);
    V dM = V(0), M = V(0);
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      if (u > nq) break;
      const V d1 = limited(x2[u], u ? ir2 : V(1), s1[u], s0[u]);
      const V fv = upwind(s0[u], d0[u], s1[u], d1, a, hl, hh);
      V F1;
      if (u == 0) {
        dM = fmav<V>(fv, a, rho0 * da) * mfac;
        M = wind ? M0 + dM : dM;
        F1 = GRP ? dM : fix(c + 1, 0, dM);
      } else {
        F1 = fix(c + 1, mq[u - 1], zq[u - 1] ? fv * M : fmav<V>(V(sb[u - 1]), dM, fv * M));
      }
      snk.put(u, ic, fmav<V>(-(F1 - F0[u]), V(ivol), w0[u]));
      F0[u] = F1;
      d0[u] = d1;
      s0[u] = s1[u];
      s1[u] = s2[u];
    }
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      w0[u] = w1[u];
      w1[u] = w2[u];
      w2[u] = nn[u];
    }
    va = vn;
    snk.done(c);
  }
}

// The usual sink of a column walk: cell c's new departures of the group's
// quantities (u = 1..) and, for the first group, of the density (u = 0) go to
// the output set.
template <typename T, typename V, int GRP, int NG>
struct OutSink {
  T *q[5];
  bool live;
  __device__ __forceinline__ OutSink(const MarchArgs<T> &A, bool lv) : live(lv) {
    q[0] = A.qo[0];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u + 1] = A.qo[group_q(NG, GRP, u)];
  }
  __device__ __forceinline__ void put(int u, idx_t ic, V val) {
    if ((u > 0 || GRP == 0) && live) gstv<V>(q[u], ic, val);
  }
  __device__ __forceinline__ void done(int) {}
};

// Rows of a finer level's column for the y pass, x-updated on the fly: row r
// of plane t comes from the x pass (XRow's arithmetic, that of k_xrow_fine)
// of the density and the group's quantities on a tile of 64 consecutive x
// cells, lane l the cell x0 = xa - 2 + l.  The tile's x pass is exact on the
// lanes 2 .. 60, the ones the walk stores: their stencils lie in the tile
// (P+x is read from the next lane's left face, which lane 63 has not).
// The x faces take the finer level's sums on the frontier and add this
// level's own transfers at faces 0 and n to the accumulators, as the separate
// x pass does, once: on owned rows (those of the walk's segment) and interior
// lanes, the density by the first group only.
template <typename T, int GRP, int NG>
struct XFineSrc {
  const Geo *G;
  const Phys *P;
  const PassArgs<T> *A;
  T dt;
  int t, x0, c0, c1, rmax;
  bool in_row, own;  // the lane's cell lies in the stored row; it is an interior lane
  // inputs of the next row (loaded while the walk uses this one): density,
  // left x-face velocity, the group's own inputs
  T ndr, nda, nin[4];
  // the row fetched past the last one needed is not used: kept in storage
  __device__ __forceinline__ idx_t at(int r) const { return lin(*G, x0, min(r, rmax), t); }
  __device__ __forceinline__ void load(int r) {
    const PassArgs<T> &a = *A;
    const idx_t c = at(r);
    ndr = in_row ? a.qi[0][c] : T(0);
    nda = in_row ? a.v[0][c] : T(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      nin[u] = T(0);
      if (u < group_n(NG, GRP)) {
        const int m = group_q(NG, GRP, u);
        if (m == 1) {
          nin[u] = in_row ? a.qi[1][c] : T(0);
        } else if (m >= 4) {
          const int d = (m - 2) >> 1;
          nin[u] = in_row ? a.v[d][c + ((m & 1) ? dstride(*G, d) : 0)] : T(0);
        }
      }
    }
  }
  __device__ __forceinline__ void get(int r, T (&w)[5]) {
    const Geo &g = *G;
    const PassArgs<T> &a = *A;
    const int rr = min(r, rmax);
    XRow<T, 1> X;
    X.dr[0] = ndr;
    X.da[0] = nda;
    T in0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) in0[u] = nin[u];
    load(r + 1);
    X.begin(g, *P, dt);
    const int n = g.n[0];
    const bool ov = a.facc && rr - g.co[1] >= 0 && t - g.co[2] >= 0 && rr - g.co[1] < g.cn[1] &&
                    t - g.co[2] < g.cn[2] && (x0 == g.co[0] || x0 == g.co[0] + g.cn[0]);
    const bool acc = a.acc && own && rr >= c0 && rr < c1 && rr >= 0 && t >= 0 && rr < g.n[1] && t < g.n[2] &&
                     (x0 == 0 || x0 == n);
    auto finish = [&](int m, const T (&own_)[1], T (&FL)[1]) -> T {
      if (ov) {
        const long fnt = (long)a.fn[1] * a.fn[2];
        const long fbase = (long)(2 * (t - g.co[2])) * a.fn[1] + 2 * (rr - g.co[1]);
        const T *f = a.facc + ((long)(x0 != g.co[0]) * NQ + m) * fnt + fbase;
        FL[0] = (f[0] + f[1]) + (f[a.fn[1]] + f[a.fn[1] + 1]);
      }
      if (acc && (m > 0 || GRP == 0))
        a.acc[((long)(x0 == n) * NQ + m) * ((long)g.n[1] * g.n[2]) + (long)t * g.n[1] + rr] += FL[0];
      T out[1];
      X.update(own_, FL, out);
      return out[0];
    };
    {
      T F[1] = {X.dM[0]};
      w[0] = finish(0, X.dr, F);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < group_n(NG, GRP)) {
        const int m = group_q(NG, GRP, u);
        T in[1], sv[1], own_[1], F[1];
        if (m == 3) row_right<T, 1>(X.da, in, T(0));
        else if (m == 2) in[0] = X.da[0];
        else in[0] = in0[u];
        X.quantity(*P, m, in, sv, own_);
        X.transfers(*P, m, sv, F);
        w[u + 1] = finish(m, own_, F);
      }
    }
  }
};

// Fused x and y passes of a finer level: one block per (x tile, y segment,
// plane), one wave per quantity group, each walking the y pass of its tile's
// 64 columns over rows that its own source x-updates on the fly (the density
// is x-passed and walked by every group; a row's inputs are loaded one row
// ahead).  Only the y pass's results reach HBM, on interior lanes within the
// updated box; the frontier transfers of both passes are taken and
// accumulated as by the separate passes.  NG quantity groups: two (the
// density walked twice) or four (walked four times, fewer registers).
// With four groups (FP64), the cells of a row past its whole tiles (at most
// XF_HALF of them) take half a wave: the blocks after those of the whole
// tiles hold these tails of two planes, lanes 0-31 the first and 32-63 the
// second, each half a tile of its own (the lane shifts across the halves
// reach only their edge lanes, which store nothing); with a longer tail, or
// two groups, it is one more whole tile.  (On 4 levels of 128^3, whose rows
// end in 12-24 such cells, this ran the FP64 coarse step 0.9 % faster and the
// FP32 one 0.5 % slower.)
constexpr int XF_TILE = BX - 5;        // x cells a tile stores
constexpr int XF_HALF = BX / 2 - 5;    // and a half-wave tile
template <typename T, int NG>
__global__ void __launch_bounds__(64 * NG) __attribute__((amdgpu_waves_per_eu(4)))
k_xyfine(Geo G, Phys P, PassArgs<T> A, MarchArgs<T> M, int ntiles, int nseg, int tail) {
  const int lane = threadIdx.x;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const unsigned h = blockIdx.x;
  const unsigned np = (unsigned)(M.hi[2] - M.lo[2]);
  const unsigned nfull = (unsigned)ntiles * (unsigned)nseg * np;
  int seg, t, xa, lx, width;
  if (NG == 2 || h < nfull) {
    const int xt = (int)(h % (unsigned)ntiles);
    const unsigned r1 = h / (unsigned)ntiles;
    seg = (int)(r1 % (unsigned)nseg);
    t = M.lo[2] + (int)(r1 / (unsigned)nseg);
    xa = M.lo[0] + XF_TILE * xt;
    lx = lane;
    width = XF_TILE;
  } else {
    const unsigned h2 = h - nfull;
    seg = (int)(h2 % (unsigned)nseg);
    t = M.lo[2] + 2 * (int)(h2 / (unsigned)nseg) + (lane >> 5);
    xa = M.lo[0] + XF_TILE * ntiles;
    lx = lane & 31;
    width = tail;
  }
  // a second half past the last plane walks the last plane again, storing nothing
  const bool tin = NG == 2 || t < M.hi[2];
  t = tin ? t : M.hi[2] - 1;
  const int c0 = M.lo[1] + seg * M.chunk;
  const int c1 = min(c0 + M.chunk, M.hi[1]);
  const int x0 = xa - 2 + lx;
  const int px = (int)(G.off - (long)G.g * (G.sy + G.sz));
  const bool in_row = x0 >= -px && x0 < (int)G.sy - px;
  const bool own = tin && lx >= 2 && lx < 2 + width && x0 < M.hi[0];
  const T dt = (T)(A.fac * A.dtp[0]);
  // rows past the last one the walk reads stay in the stored box
  const int rmax = G.n[1] + G.g - 2;
  auto walk = [&](auto gc) {
    constexpr int g = decltype(gc)::value;
    XFineSrc<T, g, NG> src{&G, &P, &A, dt, t, x0, c0, c1, rmax, in_row, own};
    src.load(c0 - 2);
    OutSink<T, T, g, NG> snk(M, own);
    march_column<T, 1, 0, g, true, 1, NG>(G, P, M, x0, t, c0, c1, src, snk, own);
  };
  if constexpr (NG == 2) {
    if (grp == 0) walk(std::integral_constant<int, 0>{});
    else walk(std::integral_constant<int, 1>{});
  } else {
    if (grp == 0) walk(std::integral_constant<int, 0>{});
    else if (grp == 1) walk(std::integral_constant<int, 1>{});
    else if (grp == 2) walk(std::integral_constant<int, 2>{});
    else walk(std::integral_constant<int, 3>{});
  }
}

template <typename T, int DIR, int BC, bool FRONT, int W>
__global__ void __launch_bounds__(256) k_march(Geo G, Phys P, MarchArgs<T> A) {
  constexpr int TD = (DIR == 1) ? 2 : 1;
  const int lane = threadIdx.x, ty = threadIdx.y;
  // threadIdx.y is the same across a wave (blockDim.x is one wave): reading it
  // from the first lane makes the quantity group, and so every field pointer,
  // a scalar
  const int grp = __builtin_amdgcn_readfirstlane(ty) & 1;
  int i, t, ch;
  if (W == 1) {
    // one column per lane: the (x, transverse) columns of the box numbered x
    // fastest, each wave taking 64 consecutive ones (rows that are not a
    // multiple of 64 long share waves), two waves' worth per block
    const unsigned ex = (unsigned)(A.hi[0] - A.lo[0]), et = (unsigned)(A.hi[TD] - A.lo[TD]);
    const unsigned nt2 = (ex * et + 127) / 128;
    const unsigned h = blockIdx.x;
    ch = (int)(h / nt2);
    const unsigned f = (h % nt2) * 128 + (unsigned)(ty >> 1) * 64 + (unsigned)lane;
    if (f >= ex * et) return;
    i = A.lo[0] + (int)(f % ex);
    t = A.lo[TD] + (int)(f / ex);
  } else {
    const int nbx = (A.hi[0] - A.lo[0] + 64 * W - 1) / (64 * W);
    const int ntb = (A.hi[TD] - A.lo[TD] + 1) / 2;
    const unsigned h = blockIdx.x;
    const int bx = (int)(h % (unsigned)nbx);
    const unsigned r1 = h / (unsigned)nbx;
    const int tb = (int)(r1 % (unsigned)ntb);
    ch = (int)(r1 / (unsigned)ntb);
    i = A.lo[0] + (bx * 64 + lane) * W;  // the lane's first column (W divides the extent)
    t = A.lo[TD] + tb * 2 + (ty >> 1);
    if (i >= A.hi[0] || t >= A.hi[TD]) return;
  }
  const int c0 = A.lo[DIR] + ch * A.chunk;
  const int c1 = min(c0 + A.chunk, A.hi[DIR]);
  if (c0 >= c1) return;
  using V = typename lanes_of<T, W>::type;
  int id3[3];
  id3[0] = i;
  id3[TD] = t;
  id3[DIR] = 0;
  const idx_t base = lin(G, id3[0], id3[1], id3[2]);
  if (grp) {
    ColSrc<T, V, DIR, BC, 1, 2> src{A.qi[0], {A.qi[4], A.qi[5], A.qi[6], A.qi[7]}, base, dstride(G, DIR), G.n[DIR]};
    OutSink<T, V, 1, 2> snk(A, true);
    march_column<T, DIR, BC, 1, FRONT, W, 2>(G, P, A, i, t, c0, c1, src, snk, true);
  } else {
    ColSrc<T, V, DIR, BC, 0, 2> src{A.qi[0], {A.qi[1], A.qi[2], A.qi[3], A.qi[1]}, base, dstride(G, DIR), G.n[DIR]};
    OutSink<T, V, 0, 2> snk(A, true);
    march_column<T, DIR, BC, 0, FRONT, W, 2>(G, P, A, i, t, c0, c1, src, snk, true);
  }
}

// Fused x and y passes with the density's work done once per plane.  Every
// quantity group needs the density's transfers: the mass transfers through the
// x faces of each row, the row's x-updated density and the y pass's reciprocal
// 1/(rho0 rho), and the mass transfers through the y faces.  The first wave of
// a plane (the density leader) computes them one row ahead of the march and
// hands them to the plane's waves (itself included) through LDS, so that the
// waves move only their own quantities; the reciprocal of each row past the
// segment's first ones is formed by the second wave, a row behind the leader
// (whose step is the longest of the four).  Row r sits in slot r mod XY_RS, face
// f in slot f mod XY_FS; one barrier per row orders the hand-over.  The
// arithmetic of every value is that of the separate passes (k_xrow, k_march).
constexpr int XY_RS = 8, XY_FS = 4;

template <typename T, int W>
struct XyShare {
  T *rows;   // [XY_RS][3][W][64]: x-face mass transfers, x-updated density, 1/(rho0 rho)
  T *faces;  // [XY_FS][W][64]: y-face mass transfers
  int lane;
  using V = typename lanes_of<T, W>::type;
  __device__ __forceinline__ T &row(int r, int f, int q) const {
    return rows[(((r & (XY_RS - 1)) * 3 + f) * W + q) * 64 + lane];
  }
  __device__ __forceinline__ T &face(int f, int q) const { return faces[((f & (XY_FS - 1)) * W + q) * 64 + lane]; }
  __device__ __forceinline__ V rowv(int r, int f) const {
    T a[W];
#pragma unroll
    for (int q = 0; q < W; ++q) a[q] = row(r, f, q);
    return to_lanes<V, T, W>(a);
  }
  __device__ __forceinline__ V facev(int f) const {
    T a[W];
#pragma unroll
    for (int q = 0; q < W; ++q) a[q] = face(f, q);
    return to_lanes<V, T, W>(a);
  }
  __device__ __forceinline__ void put_face(int f, V v) const {
    T a[W];
    from_lanes<V, T, W>(v, a);
#pragma unroll
    for (int q = 0; q < W; ++q) face(f, q) = a[q];
  }
};

// density and x-face velocity departures of row r (clamped to the active
// range, as the y pass reads its ghosts under bc 1) of plane t
template <typename T, int W>
__device__ __forceinline__ idx_t xy_row_in(const Geo &G, const PassArgs<T> &A, int r, int t, int x0, bool live,
                                           T (&dr)[W], T (&da)[W]) {
  const idx_t c = lin(G, x0, clampi(r, 0, G.n[1] - 1), t);
#pragma unroll
  for (int q = 0; q < W; ++q) {
    dr[q] = T(0);
    da[q] = T(0);
  }
  if (live) {
    row_load<T, W>(A.qi[0], c, dr);
    row_load<T, W>(A.v[0], c, da);
  }
  return c;
}

// Flux matching under a finer level (FR): the transfers of quantity m
// through the x faces of row r (the row the pass reads: clamped to the active
// range) of plane t that lie on the finer level's frontier become the sums of
// its four fine faces' transfers, as k_xrow takes them.
template <typename T, int W>
__device__ __forceinline__ void xy_front_x(const Geo &G, const PassArgs<T> &A, int m, int r, int t, int x0,
                                           T (&FL)[W]) {
  const int j = clampi(r, 0, G.n[1] - 1);
  if (!(j - G.co[1] >= 0 && t - G.co[2] >= 0 && j - G.co[1] < G.cn[1] && t - G.co[2] < G.cn[2])) return;
  const int flo = G.co[0], fhi = G.co[0] + G.cn[0];
  const long fnt = (long)A.fn[1] * A.fn[2];
  const long fbase = (long)(2 * (t - G.co[2])) * A.fn[1] + 2 * (j - G.co[1]);
#pragma unroll
  for (int q = 0; q < W; ++q) {
    const int x = x0 + q;
    if (x == flo || x == fhi) {
      const T *f = A.facc + ((long)(x == fhi) * NQ + m) * fnt + fbase;
      FL[q] = (f[0] + f[1]) + (f[A.fn[1]] + f[A.fn[1] + 1]);
    }
  }
}

// the leader's x pass of the density of row r: left-face mass transfers and
// x-updated departure into the row's slot, with ir also the reciprocal (FR:
// the update takes the frontier's transfers, the slot the pass's own, which
// the other quantities' transfers are formed from)
template <typename T, int W, bool FR>
__device__ __forceinline__ typename lanes_of<T, W>::type xy_lead_row(const Geo &G, const Phys &P, T dt,
                                                                     const XyShare<T, W> &S, int r,
                                                                     const T (&dr)[W], const T (&da)[W],
                                                                     const PassArgs<T> &A, int t, int x0,
                                                                     bool ir = true) {
  XRow<T, W> X;
#pragma unroll
  for (int q = 0; q < W; ++q) {
    X.dr[q] = dr[q];
    X.da[q] = da[q];
  }
  X.flow(G, P, dt);
  X.mass();
  T out[W];
  if constexpr (FR) {
    T F[W];
#pragma unroll
    for (int q = 0; q < W; ++q) F[q] = X.dM[q];
    xy_front_x<T, W>(G, A, 0, r, t, x0, F);
    X.update(X.dr, F, out);
  } else {
    X.update(X.dr, X.dM, out);
  }
#pragma unroll
  for (int q = 0; q < W; ++q) {
    S.row(r, 0, q) = X.dM[q];
    S.row(r, 1, q) = out[q];
    if (ir) S.row(r, 2, q) = qdiv(T(1), X.rho0 * (X.rho0 + out[q]));
  }
  return to_lanes<typename lanes_of<T, W>::type, T, W>(out);
}

// Rows of a column for the y pass of a group's own quantities: the x pass of
// those quantities on whole level-0 rows, with the row's mass transfers taken
// from the leader; the inputs of the next row are loaded while the y pass uses
// this one.
template <typename T, int W, int GRP, int NG, bool FR>
struct XyOwn {
  using V = typename lanes_of<T, W>::type;
  const Geo *G;
  const Phys *P;
  const PassArgs<T> *A;
  T dt;
  int t, x0;
  bool live;
  T dr[W], da[W], in[4][W];  // inputs of the next row

  __device__ __forceinline__ void load(int r) {
    const idx_t c = xy_row_in<T, W>(*G, *A, r, t, x0, live, dr, da);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < group_n(NG, GRP)) {
        const int m = group_q(NG, GRP, u);
        if (m != 2 && m != 3) xrow_input<T, W>(*G, *A, m, c, live, da, in[u]);
      }
    }
  }
  __device__ __forceinline__ void get(int r, const XyShare<T, W> &S, V (&w)[4]) {
    XRow<T, W> X;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      X.dr[q] = dr[q];
      X.da[q] = da[q];
    }
    X.flow(*G, *P, dt);
    if (group_q(NG, GRP, 0) == 1) X.recip();  // the energy's specific value
    T dm[W];
#pragma unroll
    for (int q = 0; q < W; ++q) dm[q] = S.row(r, 0, q);
    X.take_mass(dm);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < group_n(NG, GRP)) {
        const int m = group_q(NG, GRP, u);
        T inq[W], sv[W], own[W], F[W], out[W];
        if (m == 2 || m == 3) xrow_input<T, W>(*G, *A, m, 0, live, X.da, inq);
        else
#pragma unroll
          for (int q = 0; q < W; ++q) inq[q] = in[u][q];
        X.quantity(*P, m, inq, sv, own);
        X.transfers(*P, m, sv, F);
        if constexpr (FR) xy_front_x<T, W>(*G, *A, m, r, t, x0, F);
        X.update(own, F, out);
        w[u] = to_lanes<V, T, W>(out);
      }
    }
    load(r + 1);
  }
};

// One plane's y segment [c0, c1) of group GRP's own quantities; with LEAD
// also the density (its x pass one row ahead, its y-face transfers one face
// ahead, its update).  Each row is one step that ends in a barrier, so every
// wave of the block meets the same barriers.  The values a step hands to the
// next live in rings of three slots whose roles turn with the step's phase
// (its row's distance from c0, mod 3), so that no value is copied from step
// to step.  put: the lane writes its results (it is live and the plane
// exists).
template <typename T, int W, int GRP, int NG, bool LEAD, bool FR>
__device__ __forceinline__ void xy_shared_group(const Geo &G, const Phys &P, const PassArgs<T> &A,
                                                const MarchArgs<T> &M, T dt, int t, int x0, bool live, bool put,
                                                int c0, int c1, const XyShare<T, W> &S) {
  // a segment's first face is formed here and, by the segment below, in its
  // walk: as in march_column, no implicit contraction, the fused products
  // written out, so that both give the same value
#pragma clang fp contract(off)
  using V = typename lanes_of<T, W>::type;
  constexpr int nq = group_n(NG, GRP);
  constexpr int mq[4] = {group_q(NG, GRP, 0), group_q(NG, GRP, 1), group_q(NG, GRP, 2), group_q(NG, GRP, 3)};
  constexpr bool zq[4] = {mq[0] >= 4, mq[1] >= 4, mq[2] >= 4, mq[3] >= 4};
  const T dx = (T)G.dx;
  const T mfac = dt * dx * dx, ivol = T(1) / (dx * dx * dx), cour = dt / dx;
  const T rho0 = (T)P.rho0;
  const idx_t st = (idx_t)G.sy;
  const idx_t base = lin(G, x0, 0, t);
  T q0[4], sb[4];
  T *qout[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    q0[u] = (T)qback(P, mq[u]);
    sb[u] = (T)sback(P, mq[u]);
    qout[u] = M.qo[mq[u]];
  }
  // the face's weights hl = (1 - nu)/2, hh = (1 + nu)/2 are exact halvings
  // of the rounded 1 -+ nu
  auto upwind = [&](V sl, V dl, V sr, V dr, V a) -> V {
    const V nu = a * cour;
    const V hl = fmav<V>(V(-0.5), nu, V(0.5)), hh = fmav<V>(V(0.5), nu, V(0.5));
    const V lo = fmav<V>(dl, hl, sl), hi = fmav<V>(-dr, hh, sr);
    return a > T(0) ? lo : hi;
  };
  // numerator of a specific value's departure (times 1/(rho0 rho) the value)
  // and the limited difference at a cell from its right neighbour's numerator
  // and reciprocal: the arithmetic of march_column
  auto numer = [&](int u, V q, V r) -> V { return zq[u] ? rho0 * q : fmav<V>(V(rho0), q, -(q0[u] * r)); };
  auto limited = [&](V xr, V ir, V s, V sl) -> V { return vleer(fmav<V>(xr, ir, -s), s - sl); };
  auto face = [&](int c) -> V { return live ? gldv<V>(M.v, base + c * st) : V(0); };
  // mass transfer through a y face from the density around it
  auto mass_y = [&](V a, V sl, V dl, V sr, V dr) -> V {
    return fmav<V>(upwind(sl, dl, sr, dr, a), a, rho0 * a) * mfac;
  };
  // flux matching under a finer level (FR): the transfer of quantity m
  // through y face f of the lane's columns, where that face lies on the finer
  // level's frontier, becomes the sum of its four fine faces' transfers (as in
  // march_column); the mass transfers handed to the other waves stay the
  // pass's own, which their transfers are formed from
  bool ovy[W];
  long fby[W];
  bool anyov = false;
  if constexpr (FR) {
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const int a1 = x0 + q - G.co[0], a2 = t - G.co[2];
      ovy[q] = live && a1 >= 0 && a2 >= 0 && a1 < G.cn[0] && a2 < G.cn[2];
      fby[q] = (long)(2 * a2) * A.fn[0] + 2 * a1;
      anyov |= ovy[q];
    }
  }
  auto fixy = [&](int f, int m, V F) -> V {
    if constexpr (FR) {
      const int fylo = G.co[1], fyhi = G.co[1] + G.cn[1];
      if (anyov && (f == fylo || f == fyhi)) {
        const long fnt = (long)A.fn[0] * A.fn[2];
        T a[W];
        from_lanes<V, T, W>(F, a);
#pragma unroll
        for (int q = 0; q < W; ++q) {
          if (ovy[q]) {
            const T *p = A.facc + ((long)(2 + (f == fyhi)) * NQ + m) * fnt + fby[q];
            a[q] = (p[0] + p[1]) + (p[A.fn[0]] + p[A.fn[0] + 1]);
          }
        }
        return to_lanes<V, T, W>(a);
      }
    }
    return F;
  };

  // leader rings: x-updated density of rows c+1 .. c+3 (rr), its limited
  // difference at c+1 (rd), the mass transfers of faces c, c+1 (rm), the
  // velocity departure of face c+2 (rv); inputs of row c+4 (ldr, lda)
  V rr[3], rd[3], rm[3], rv[3];
  T ldr[W], lda[W];
  if constexpr (LEAD) {
    xy_row_in<T, W>(G, A, c0 - 2, t, x0, live, ldr, lda);
    const V r_m2 = xy_lead_row<T, W, FR>(G, P, dt, S, c0 - 2, ldr, lda, A, t, x0);
    xy_row_in<T, W>(G, A, c0 - 1, t, x0, live, ldr, lda);
    const V r_m1 = xy_lead_row<T, W, FR>(G, P, dt, S, c0 - 1, ldr, lda, A, t, x0);
    xy_row_in<T, W>(G, A, c0, t, x0, live, ldr, lda);
    const V r_0 = xy_lead_row<T, W, FR>(G, P, dt, S, c0, ldr, lda, A, t, x0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xy_row_in<T, W>(G, A, c0 + 1 + k, t, x0, live, ldr, lda);
      rr[k] = xy_lead_row<T, W, FR>(G, P, dt, S, c0 + 1 + k, ldr, lda, A, t, x0, k < 2);
    }
    xy_row_in<T, W>(G, A, c0 + 4, t, x0, live, ldr, lda);
    const V d_m1 = vleer(r_0 - r_m1, r_m1 - r_m2);
    const V d_0 = vleer(rr[0] - r_0, r_0 - r_m1);
    rm[0] = mass_y(face(c0), r_m1, d_m1, r_0, d_0);
    S.put_face(c0, rm[0]);
    rd[0] = vleer(rr[1] - rr[0], rr[0] - r_0);
    rm[1] = mass_y(face(c0 + 1), r_0, d_0, rr[0], rd[0]);
    S.put_face(c0 + 1, rm[1]);
    rv[0] = face(min(c0 + 2, c1));
  }
  __syncthreads();

  // own rings: specific values at c, c+1 (ss), limited difference at c (sd),
  // transfer through face c (sF), x-updated departures of rows c .. c+2 (sw),
  // velocity departure of face c+1 (sv)
  XyOwn<T, W, GRP, NG, FR> src{&G, &P, &A, dt, t, x0, live};
  V ss[3][4], sd[3][4], sF[3][4], sw[3][4], sv[3];
  if constexpr (nq > 0) {
    V wm2[4], wm1[4];
    src.load(c0 - 2);
    src.get(c0 - 2, S, wm2);
    src.get(c0 - 1, S, wm1);
    src.get(c0, S, sw[0]);
    src.get(c0 + 1, S, sw[1]);
    const V r_m2 = S.rowv(c0 - 2, 1), r_m1 = S.rowv(c0 - 1, 1), r_0 = S.rowv(c0, 1), r_p1 = S.rowv(c0 + 1, 1);
    const V i_m2 = S.rowv(c0 - 2, 2), i_m1 = S.rowv(c0 - 1, 2), i_0 = S.rowv(c0, 2), i_p1 = S.rowv(c0 + 1, 2);
    const V a = face(c0);
    const V dM = S.facev(c0);
#pragma unroll
    for (int u = 0; u < nq; ++u) {
      const V sm2 = numer(u, wm2[u], r_m2) * i_m2, sm1 = numer(u, wm1[u], r_m1) * i_m1;
      const V x0 = numer(u, sw[0][u], r_0), x1 = numer(u, sw[1][u], r_p1);
      ss[0][u] = x0 * i_0;
      ss[1][u] = x1 * i_p1;
      const V dm1 = limited(x0, i_0, sm1, sm2);
      sd[0][u] = limited(x1, i_p1, ss[0][u], sm1);
      const V fv = upwind(sm1, dm1, ss[0][u], sd[0][u], a);
      sF[0][u] = fixy(c0, mq[u], zq[u] ? fv * dM : fmav<V>(V(sb[u]), dM, fv * dM));
    }
    src.get(c0 + 2, S, sw[2]);
    sv[0] = face(c0 + 1);
  }

  // row c in phase K0: ring slot K0 holds the oldest value, K1 the next, K2
  // the newest (or the free slot)
  auto step = [&](auto phase, int c) {
    constexpr int K0 = decltype(phase)::value, K1 = (K0 + 1) % 3, K2 = (K0 + 2) % 3;
    const idx_t ic = base + c * st;
    if constexpr (nq > 0) {
      const V r2 = S.rowv(c + 2, 1), ir2 = S.rowv(c + 2, 2);
      const V a = sv[K0];
      sv[K1] = face(min(c + 2, c1));
      const V dM = S.facev(c + 1);
#pragma unroll
      for (int u = 0; u < nq; ++u) {
        const V x2 = numer(u, sw[K2][u], r2);
        ss[K2][u] = x2 * ir2;
        sd[K1][u] = limited(x2, ir2, ss[K1][u], ss[K0][u]);
        const V fv = upwind(ss[K0][u], sd[K0][u], ss[K1][u], sd[K1][u], a);
        sF[K1][u] = fixy(c + 1, mq[u], zq[u] ? fv * dM : fmav<V>(V(sb[u]), dM, fv * dM));
        if (put) gstv<V>(qout[u], ic, fmav<V>(-(sF[K1][u] - sF[K0][u]), V(ivol), sw[K0][u]));
      }
      src.get(c + 3, S, sw[K0]);
    }
    if constexpr (GRP == 1) {
      // the reciprocal of row c+3 (its density came from the leader a step
      // ago), for the y walk one step later; the leader carries more work
#pragma unroll
      for (int q = 0; q < W; ++q) S.row(c + 3, 2, q) = qdiv(T(1), rho0 * (rho0 + S.row(c + 3, 1, q)));
    }
    if constexpr (LEAD) {
      if (put) gstv<V>(M.qo[0], ic, fmav<V>(-(fixy(c + 1, 0, rm[K1]) - fixy(c, 0, rm[K0])), V(ivol), S.rowv(c, 1)));
      rd[K1] = vleer(rr[K2] - rr[K1], rr[K1] - rr[K0]);
      rm[K2] = mass_y(rv[K0], rr[K0], rd[K0], rr[K1], rd[K1]);
      S.put_face(c + 2, rm[K2]);
      rv[K1] = face(min(c + 3, c1));
      rr[K0] = xy_lead_row<T, W, FR>(G, P, dt, S, c + 4, ldr, lda, A, t, x0, false);
      xy_row_in<T, W>(G, A, c + 5, t, x0, live, ldr, lda);
    }
    __syncthreads();
  };
  for (int c = c0; c < c1; c += 3) {
    step(std::integral_constant<int, 0>(), c);
    if (c + 1 < c1) step(std::integral_constant<int, 1>(), c + 1);
    if (c + 2 < c1) step(std::integral_constant<int, 2>(), c + 2);
  }
}

// Fused x and y passes of level 0 without a finer level (bc 1, rows of at most
// 64 W cells): one block per (plane, y segment), one wave per quantity group
// of four, each holding whole rows, W cells per lane; the first group's wave
// leads the density.  Only the y pass's results reach HBM.  Results are those
// of the separate passes up to the pairing of products and sums into fused
// multiply-adds.
template <typename T, int W, bool FULL, bool FR>
__device__ __forceinline__ void xyshared_body(Geo G, Phys P, PassArgs<T> A, MarchArgs<T> M, Blk bk) {
  constexpr int NG = 4;
  __shared__ T rows[XY_RS * 3 * W * 64];
  __shared__ T faces[XY_FS * W * 64];
  const int lane = threadIdx.x;
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int t = (int)(bk.id % (unsigned)G.n[2]), ch = (int)(bk.id / (unsigned)G.n[2]);
  const int c0 = ch * M.chunk;
  const int c1 = min(c0 + M.chunk, G.n[1]);
  if (c0 >= c1) return;  // the whole block
  const int x0 = W * lane;
  const bool live = FULL || x0 < G.n[0];  // FULL: the rows fill the wave exactly
  const T dt = (T)(A.fac * A.dtp[0]);
  const XyShare<T, W> S{rows, faces, lane};
  if (grp == 0) xy_shared_group<T, W, 0, NG, true, FR>(G, P, A, M, dt, t, x0, live, live, c0, c1, S);
  else if (grp == 1) xy_shared_group<T, W, 1, NG, false, FR>(G, P, A, M, dt, t, x0, live, live, c0, c1, S);
  else if (grp == 2) xy_shared_group<T, W, 2, NG, false, FR>(G, P, A, M, dt, t, x0, live, live, c0, c1, S);
  else xy_shared_group<T, W, 3, NG, false, FR>(G, P, A, M, dt, t, x0, live, live, c0, c1, S);
}

template <typename T, int W, bool FULL, bool FR = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_xyshared(Geo G, Phys P, PassArgs<T> A, MarchArgs<T> M) {
  xyshared_body<T, W, FULL, FR>(G, P, A, M, grid_blk());
}

// ------------------------------------------------------------ CommUp

// The five state fields of one CommUp or CommMean in one launch: field f
// takes blocks [start[f], start[f+1]).
template <typename T>
struct UpArgs {
  const T *Q[NSTATE];  // coarse fields: rho, e, vx, vy, vz
  T *out[NSTATE];      // fine fields
  Box b;               // coarse hosts of the fine entries (every field)
  // hosts whose eight children are all active fine cells ([0, n/2) along each
  // axis, relative to b.lo) are not enumerated: the shell around them is, in
  // three parts -- the planes outside them (all rows), the rows outside them
  // in their planes, the hosts outside them in their rows
  int in_lo[3], in_n[3];
  unsigned c1, c2, nshell;
  unsigned nb;         // blocks per field
};

// element f of a five-entry argument array, for a wave-uniform f (a select
// chain rather than an indexed load of the kernel's arguments)
template <typename P>
__device__ __forceinline__ P pick5(const P (&a)[NSTATE], int f) {
  return f == 0 ? a[0] : f == 1 ? a[1] : f == 2 ? a[2] : f == 3 ? a[3] : a[4];
}

// CommUp (Sect. 3.2.1, Fig. 2): every fine entry outside the fine active set
// from the 27 coarse entries around its host, interpolating along z, then y,
// then x.  The background is uniform, so departures interpolate like values.
// One thread per coarse host: its eight fine children share the 27 coarse
// neighbours and, since the limited slope of a 1-D step does not depend on
// which half of the host a child takes, every slope is formed once for both
// children (19 slopes instead of 8 x 13).  A.b counts hosts relative to the
// covered coarse box (host H = Gc.co + h).
template <typename T, int CBC>
__global__ void __launch_bounds__(BX * BY) k_commup(Geo Gc, Geo Gf, UpArgs<T> UA) {
  const int fld = (int)(blockIdx.x / UA.nb);
  struct {
    const T *Q;
    T *out;
    int stag;
  } A{pick5(UA.Q, fld), pick5(UA.out, fld), fld >= 2 ? fld - 2 : -1};
  int h[3];
  {
    const unsigned f = (blockIdx.x % UA.nb) * (BX * BY) + threadIdx.y * BX + threadIdx.x;
    if (f >= UA.nshell) return;
    const unsigned X = (unsigned)(UA.b.hi[0] - UA.b.lo[0]), Y = (unsigned)(UA.b.hi[1] - UA.b.lo[1]);
    unsigned x, y, z;
    if (f < UA.c1) {
      z = f / (X * Y);
      y = (f % (X * Y)) / X;
      x = f % X;
      if ((int)z >= UA.in_lo[2]) z += UA.in_n[2];
    } else if (f < UA.c2) {
      const unsigned g = f - UA.c1, ny = Y - UA.in_n[1];
      z = UA.in_lo[2] + g / (ny * X);
      y = (g % (ny * X)) / X;
      x = g % X;
      if ((int)y >= UA.in_lo[1]) y += UA.in_n[1];
    } else {
      const unsigned g = f - UA.c2, nx = X - UA.in_n[0];
      z = UA.in_lo[2] + g / (UA.in_n[1] * nx);
      y = UA.in_lo[1] + (g % (UA.in_n[1] * nx)) / nx;
      x = g % nx;
      if ((int)x >= UA.in_lo[0]) x += UA.in_n[0];
    }
    h[0] = UA.b.lo[0] + (int)x;
    h[1] = UA.b.lo[1] + (int)y;
    h[2] = UA.b.lo[2] + (int)z;
  }
  // children 2h, 2h+1 along each axis; the host is skipped when all eight are
  // active entries (which the fine level owns)
  bool inner = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int hi = Gf.n[d] + (d == A.stag ? 1 : 0);
    if (2 * h[d] < 0 || 2 * h[d] + 1 >= hi) inner = false;
  }
  if (inner) return;
  const int H0 = Gc.co[0] + h[0], H1 = Gc.co[1] + h[1], H2 = Gc.co[2] + h[2];
  auto C = [&](int a, int b, int cc) -> T {
    const int ci = H0 + a, cj = H1 + b, ck = H2 + cc;
    if (CBC) {
      if (A.stag < 0) return cread<CBC>(A.Q, Gc, ci, cj, ck);
      return fread_bc<CBC>(A.Q, Gc, A.stag, ci, cj, ck);
    }
    return A.Q[lin(Gc, ci, cj, ck)];
  };
  // both children of one 1-D step of the prolongation, from three
  // consecutive coarse values around the host: on centred axes a quarter
  // coarse cell either side of the host centre with van Leer's limited slope;
  // along a face field's own axis the even child is the host face, the odd
  // one the mean of the host face and the next
  auto up2 = [&](bool stag_axis, T m, T c, T p, T &lo, T &hi) {
    if (stag_axis) {
      lo = c;
      hi = T(0.5) * (c + p);
    } else {
      const T sl = vleer(p - c, c - m);
      lo = c + sl * T(-0.25);
      hi = c + sl * T(0.25);
    }
  };
  T qz[2][3][3];  // [z child][x offset][y offset]
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) up2(A.stag == 2, C(a - 1, b - 1, -1), C(a - 1, b - 1, 0), C(a - 1, b - 1, 1),
                                    qz[0][a][b], qz[1][a][b]);
  T r[2][2][3];  // [z child][y child][x offset]
#pragma unroll
  for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
    for (int a = 0; a < 3; ++a) up2(A.stag == 1, qz[o2][a][0], qz[o2][a][1], qz[o2][a][2], r[o2][0][a], r[o2][1][a]);
#pragma unroll
  for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
    for (int o1 = 0; o1 < 2; ++o1) {
      T v[2];
      up2(A.stag == 0, r[o2][o1][0], r[o2][o1][1], r[o2][o1][2], v[0], v[1]);
      const int k = 2 * h[2] + o2, j = 2 * h[1] + o1;
#pragma unroll
      for (int o0 = 0; o0 < 2; ++o0) {
        const int i = 2 * h[0] + o0;
        const int id[3] = {i, j, k};
        bool in = true, active = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          if (id[d] < -Gf.g || id[d] >= Gf.s[d] - Gf.g) in = false;
          if (id[d] < 0 || id[d] >= Gf.n[d] + (d == A.stag ? 1 : 0)) active = false;
        }
        if (in && !active) A.out[lin(Gf, i, j, k)] = v[o0];
      }
    }
}

// ------------------------------------------------------ quadrant images
// The entries of a finer level beyond an anchored face (the perturber's mirror
// plane, Sect. 3.4) as the mirror images of the level's own entries:
// dst = sgn src at the mirror position -- cell j < 0 takes cell -1-j, a face
// normal to the plane j < 0 takes face -j.  One launch per plane, every
// listed field at each position.
template <typename T>
struct MirArgs {
  T *dst[NQ];
  const T *src[NQ];
  T sgn[NQ];
  int face[NQ];  // the field lives on the faces normal to the plane
  int nf;
  int d;         // the plane's normal (1 or 2)
  Box b;         // the entries beyond the plane
};

template <typename T>
__global__ void __launch_bounds__(BX * BY) k_mirror(Geo G, MirArgs<T> A) {
  int i, j, k;
  if (!thread_cell_flat(A.b, i, j, k)) return;
  const int id[3] = {i, j, k};
  const int m = id[A.d];  // < 0
  const idx_t c = lin(G, i, j, k), sd = dstride(G, A.d);
  for (int f = 0; f < A.nf; ++f) {
    const idx_t src = A.face[f] ? c - 2 * m * sd : c + (-1 - 2 * m) * sd;
    A.dst[f][c] = A.sgn[f] * A.src[f][src];
  }
}

// ------------------------------------------------------------ CommMean

template <typename T>
struct MeanArgs {
  const T *Q[NSTATE];      // fine fields
  T *out[NSTATE];          // coarse fields
  Box b;                   // covered coarse cells, relative to the covered box (faces: one more
                           // along their normal)
  unsigned start[NSTATE + 1];
};

// CommMean (Sect. 3.2.2): covered coarse cells take the mean of their 8 fine
// cells, covered coarse faces the mean of their 4 coincident fine faces.
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_commmean(Geo Gf, Geo Gc, MeanArgs<T> MA) {
  const unsigned h = blockIdx.x;
  const int fld = h < MA.start[1] ? 0 : h < MA.start[2] ? 1 : h < MA.start[3] ? 2 : h < MA.start[4] ? 3 : 4;
  const unsigned s0 = fld == 0 ? 0u : fld == 1 ? MA.start[1] : fld == 2 ? MA.start[2] : fld == 3 ? MA.start[3] : MA.start[4];
  const unsigned s1 = fld == 0 ? MA.start[1] : fld == 1 ? MA.start[2] : fld == 2 ? MA.start[3] : fld == 3 ? MA.start[4]
                                                                                                 : MA.start[5];
  struct {
    const T *Q;
    T *out;
    int stag;
  } A{pick5(MA.Q, fld), pick5(MA.out, fld), fld >= 2 ? fld - 2 : -1};
  Box bb = MA.b;
  bb.hi[0] += A.stag == 0 ? 1 : 0;
  bb.hi[1] += A.stag == 1 ? 1 : 0;
  bb.hi[2] += A.stag == 2 ? 1 : 0;
  int I, J, K;
  if (!thread_cell_flat(bb, I, J, K, Blk{h - s0, s1 - s0})) return;
  const idx_t f = lin(Gf, 2 * I, 2 * J, 2 * K);
  const T *q = A.Q;
  T val;
  if (A.stag < 0) {
    const idx_t sx = 1, sy = (idx_t)Gf.sy, sz = (idx_t)Gf.sz;
    val = (((q[f] + q[f + sx]) + (q[f + sy] + q[f + sx + sy])) +
           ((q[f + sz] + q[f + sx + sz]) + (q[f + sy + sz] + q[f + sx + sy + sz]))) * T(0.125);
  } else {
    const idx_t e1 = (A.stag == 0) ? (idx_t)Gf.sy : 1;
    const idx_t e2 = (A.stag == 2) ? (idx_t)Gf.sy : (idx_t)Gf.sz;
    val = ((q[f] + q[f + e1]) + (q[f + e2] + q[f + e1 + e2])) * T(0.25);
  }
  A.out[lin(Gc, Gc.co[0] + I, Gc.co[1] + J, Gc.co[2] + K)] = val;
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

template <typename T>
struct RedArgs {
  Box b;
  const T *rho, *e, *v[3];
  double *part;              // per-block partials: three planes of npart values
  double *spart;             // per-block maximum signal speeds
  int npart;                 // partial slots per plane (the blocks of the one-cell-per-thread grid)
  Scal *S;
  int cov_lo[3], cov_hi[3];  // covered cells (empty if no finer level)
};

template <typename T>
__device__ __forceinline__ bool is_covered(const RedArgs<T> &A, int i, int j, int k) {
  return i >= A.cov_lo[0] && i < A.cov_hi[0] && j >= A.cov_lo[1] && j < A.cov_hi[1] && k >= A.cov_lo[2] &&
         k < A.cov_hi[2];
}

// block sum of three values into part[q * blocks + block]; fixed order for a fixed grid
__device__ void block_sum3(double a, double b, double c, double *part, int npart, Blk bk = grid_blk()) {
  __shared__ double sh[3][BX * BY / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int t = threadIdx.y * BX + threadIdx.x;
  const int w = t / 64, l = t % 64;
  if (l == 0) {
    sh[0][w] = a;
    sh[1][w] = b;
    sh[2][w] = c;
  }
  __syncthreads();
  if (t == 0) {
    const long blk = bk.id;
    double s0 = 0, s1 = 0, s2 = 0;
    for (int q = 0; q < BX * BY / 64; ++q) {
      s0 += sh[0][q];
      s1 += sh[1][q];
      s2 += sh[2][q];
    }
    // three planes of one value per block (coalesced for the final sum)
    const long nb = npart;
    part[blk] = s0;
    part[nb + blk] = s1;
    part[2 * nb + blk] = s2;
  }
}

// Force of the gas on the perturber, eq. 18: G M (rho - rho0) dV r /
// (r^2+eps^2)^{3/2} over uncovered active cells, in FP64 (the uniform part
// sums to zero by symmetry).
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_force(Geo G, Phys P, RedArgs<T> A) {
  int i, j, k;
  const bool ok = thread_cell(A.b, i, j, k);
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (ok && !is_covered(A, i, j, k)) {
    const double x = xcen<double>(G, 0, i), y = xcen<double>(G, 1, j), z = xcen<double>(G, 2, k);
    const double d2 = x * x + y * y + z * z + P.eps2;
    const double vol = G.dx * G.dx * G.dx;
    const double w = P.GM * (double)A.rho[lin(G, i, j, k)] * vol / (d2 * sqrt(d2));
    fx = w * x;
    fy = w * y;
    fz = w * z;
  }
  block_sum3(fx, fy, fz, A.part, A.npart);
}

// mass, internal energy and kinetic energy (face velocities averaged to
// centres), FP64
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_totals(Geo G, Phys P, RedArgs<T> A) {
  int i, j, k;
  const bool ok = thread_cell(A.b, i, j, k);
  double m = 0.0, ei = 0.0, ek = 0.0;
  if (ok && !is_covered(A, i, j, k)) {
    const idx_t c = lin(G, i, j, k);
    const double vol = G.dx * G.dx * G.dx;
    const double r = P.rho0 + (double)A.rho[c];
    double v2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double vc = vback(P, d) + 0.5 * ((double)A.v[d][c] + (double)A.v[d][c + dstride(G, d)]);
      v2 += vc * vc;
    }
    m = r * vol;
    ei = (P.e0 + (double)A.e[c]) * vol;
    ek = 0.5 * r * v2 * vol;
  }
  block_sum3(m, ei, ek, A.part, A.npart);
}

// fixed-order sum of the partials of all levels (one block)
struct FinalArgs {
  const double *part[MAXLEV];
  int npart[MAXLEV];
  int nl;
  double *out;   // 3 doubles
  Scal *S;       // with flog: append (out, t) to the ring
  double *flog;
};

// The one-block kernels that finish a reduction run FT threads: each reads
// its partials (blocks t, t+FT, ...) eight at a time, so that all partials
// of a 128^3 level are in flight at once; the order of the sum is fixed.
constexpr int FT = 1024;
constexpr int FW = FT / 64;

// thread 0: the wave sums sh (in wave order) into out, then the log entry
__device__ void final3_finish(const FinalArgs &A, const double (*sh)[FW]) {
  for (int q = 0; q < 3; ++q) {
    double t = 0.0;
    for (int v = 0; v < FW; ++v) t += sh[q][v];
    A.out[q] = t * (A.out == A.S->totals ? A.S->tmul : A.S->fmul[q]);
  }
  if (A.flog) {
    const unsigned int n = A.S->nlog;
    double *e = A.flog + 4 * (size_t)(n % FLOG);
    for (int q = 0; q < 3; ++q) e[q] = A.out[q];
    e[3] = A.S->t;
    A.S->nlog = n + 1;
    A.S->pending = 0;
  }
}

__device__ void final3_body(const FinalArgs &A) {
  __shared__ double sh[3][FW];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int l = 0; l < A.nl; ++l) {
    const double *p = A.part[l];
    const int n = A.npart[l];
    int b = threadIdx.x;
    for (; b + 7 * FT < n; b += 8 * FT) {
      double x[8][3];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int q = 0; q < 3; ++q) x[u][q] = p[(size_t)q * n + b + u * FT];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s0 += x[u][0];
        s1 += x[u][1];
        s2 += x[u][2];
      }
    }
    for (; b < n; b += FT) {
      s0 += p[b];
      s1 += p[(size_t)n + b];
      s2 += p[2 * (size_t)n + b];
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  const int w = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) {
    sh[0][w] = s0;
    sh[1][w] = s1;
    sh[2][w] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) final3_finish(A, sh);
  __syncthreads();
}

__global__ void __launch_bounds__(FT) k_final3(FinalArgs A) { final3_body(A); }

// A pending end-of-step force (single-level runs): the fixed-order sum of the
// three planes of partials by the NT threads of one block, into S->force and
// the log at the time S->tlog of its state; every thread calls it.
template <int NT>
__device__ void log_pending_body(const double *part, int n, Scal *S, double *flog) {
  constexpr int NW = NT / 64;
  __shared__ double sh[3][NW];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  if (!S->pending) return;  // the same value for every thread of the block
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  int b = tid;
  for (; b + 7 * NT < n; b += 8 * NT) {
    double x[8][3];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int q = 0; q < 3; ++q) x[u][q] = part[(size_t)q * n + b + u * NT];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s0 += x[u][0];
      s1 += x[u][1];
      s2 += x[u][2];
    }
  }
  for (; b < n; b += NT) {
    s0 += part[b];
    s1 += part[(size_t)n + b];
    s2 += part[2 * (size_t)n + b];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (tid % 64 == 0) {
    sh[0][tid / 64] = s0;
    sh[1][tid / 64] = s1;
    sh[2][tid / 64] = s2;
  }
  __syncthreads();
  if (tid == 0) {
    const unsigned int k = S->nlog;
    double *e = flog + 4 * (size_t)(k % FLOG);
    for (int q = 0; q < 3; ++q) {
      double t = 0.0;
      for (int v = 0; v < NW; ++v) t += sh[q][v];
      t *= S->fmul[q];
      S->force[q] = t;
      e[q] = t;
    }
    e[3] = S->tlog;
    S->nlog = k + 1;
    S->pending = 0;
  }
}

__global__ void __launch_bounds__(FT) k_log_pending(const double *part, int n, Scal *S, double *flog) {
  log_pending_body<FT>(part, n, S, flog);
}

// Signal speed c_s + |v| of an active cell, the largest over its six faces,
// and whether its density and energy are positive and finite.
template <typename T>
__device__ __forceinline__ double cell_signal(const Geo &G, const Phys &P, const RedArgs<T> &A, idx_t c,
                                              int &bad) {
  const double r = P.rho0 + (double)A.rho[c], en = P.e0 + (double)A.e[c];
  if (!(r > 0.0) || !(en > 0.0) || !isfinite(r) || !isfinite(en)) bad = 1;
  const double cs = sqrt(P.gamma * P.gm1 * en / r);
  double vm = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double a = fabs(vback(P, d) + (double)A.v[d][c]);
    const double b = fabs(vback(P, d) + (double)A.v[d][c + dstride(G, d)]);
    vm = fmax(vm, fmax(a, b));
  }
  const double sig = cs + vm;
  if (!isfinite(sig)) bad = 1;
  return sig;
}

// block maximum of the signal speeds into spart[block]; a bad cell raises
// the health flag
__device__ void block_signal(double sig, int bad, double *spart, Scal *S, Blk bk = grid_blk()) {
  sig = wave_max(bad ? 0.0 : sig);
  const bool anybad = __any(bad);
  __shared__ double sh[BX * BY / 64];
  const int t = threadIdx.y * BX + threadIdx.x;
  if ((t % 64) == 0) {
    sh[t / 64] = sig;
    if (anybad) atomicOr(&S->health, 1);
  }
  __syncthreads();
  if (t == 0) {
    double m = sh[0];
    for (int q = 1; q < BX * BY / 64; ++q) m = fmax(m, sh[q]);
    spart[bk.id] = m;
    // the same maximum into this block's slot (m >= 0, so the order of the
    // bits is that of the values)
    if (S)
      __hip_atomic_fetch_max(&S->smax[bk.id & (NSLOT - 1)], (unsigned long long)__double_as_longlong(m),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Largest signal speed over the active cells and their faces (per block,
// reduced by the final kernel), and the health check.
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_signal(Geo G, Phys P, RedArgs<T> A) {
  int i, j, k;
  const bool ok = thread_cell(A.b, i, j, k);
  double sig = 0.0;
  int bad = 0;
  if (ok) sig = cell_signal(G, P, A, lin(G, i, j, k), bad);
  block_signal(sig, bad, A.spart, A.S);
}

// End of a step: the force partials of eq. 18 (as k_force) and the signal
// speed partials of the next step's time step (as k_signal) in one pass over
// the state, which both read.
template <typename T>
__global__ void __launch_bounds__(BX * BY) k_post(Geo G, Phys P, RedArgs<T> A) {
  int i, j, k;
  const bool ok = thread_cell(A.b, i, j, k);
  double fx = 0.0, fy = 0.0, fz = 0.0, sig = 0.0;
  int bad = 0;
  if (ok) {
    const idx_t c = lin(G, i, j, k);
    sig = cell_signal(G, P, A, c, bad);
    if (!is_covered(A, i, j, k)) {
      const double x = xcen<double>(G, 0, i), y = xcen<double>(G, 1, j), z = xcen<double>(G, 2, k);
      const double d2 = x * x + y * y + z * z + P.eps2;
      const double vol = G.dx * G.dx * G.dx;
      const double w = P.GM * (double)A.rho[c] * vol / (d2 * sqrt(d2));
      fx = w * x;
      fy = w * y;
      fz = w * z;
    }
  }
  block_sum3(fx, fy, fz, A.part, A.npart);
  block_signal(sig, bad, A.spart, A.S);
}

// Level-0 form of the kick (rows of even length, as every level-0 mesh has):
// one thread per pair of adjacent active cells (the box's x range counts
// pairs) computes the faces on the low side of both cells and, for the last
// cells along a dimension, also the boundary face n there (the injection face
// at x_max carries the wind), so the grid is exactly the active box.  The
// pair's own fields and its y and z neighbours move as 8- or 16-byte
// accesses; the two low x faces take the cell before the pair and the pair
// itself.  With POST (the last kernel of a single-level step) it also forms
// the end-of-step reductions of k_post: the force partials of its cells, and
// the signal speed c_s + |v| of every pair of an active cell and one of its
// faces, taken at the face's owner (the cell on its high side, or the last
// cell for face n), which holds both adjacent cells' densities and energies.
// A block then covers the cells of up to two blocks of the one-cell-per-thread
// grid whose blocks k_post and the final sums count: it writes its partials to
// slot blockIdx.x and zeros to slot gridDim.x + blockIdx.x (when that is below
// npart).  With COMP (the first kick of a step) it then compresses its cells
// as k_compress2 does, from the kicked velocities of their six faces: the high
// faces that other threads own (x face i+2, y face j+1, z face k+1) it kicks
// again itself with their owners' arithmetic (they are not written); the
// compressed energy goes to A.eo.
// (five waves per SIMD: the FP64 end-of-step form fits 93 registers with no
// spill, against 104 and four waves unconstrained)
template <typename T, int BCM, bool REBUILD, bool KICK, bool POST, bool COMP>
__device__ __forceinline__ void kick0p_body(Geo G, Phys P, KickArgs<T> A, RedArgs<T> R, Blk bk) {
  using V = typename lanes_of<T, 2>::type;
  int p, j, k;
  const bool ok = thread_cell_flat(A.b, p, j, k, bk);
  // with COMP in FP64, a block whose threads all hold pairs (the same for
  // all its threads) hands each pair's low y faces to the pairs below them in
  // the block, which then need not kick their high y faces again (128^3: the
  // FP64 step 0.7 % faster; in FP32, where the kick is cheap, no faster)
  const int tid = threadIdx.y * BX + threadIdx.x;
  const int exb = A.b.hi[0] - A.b.lo[0];
  const long fl = (long)(j - A.b.lo[1]) * exb + (p - A.b.lo[0]);
  const bool full = COMP && sizeof(T) == 8 && fl - tid + BX * BY <= (long)exb * (A.b.hi[1] - A.b.lo[1]);
  const bool yx = full && tid + exb < BX * BY;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  T sig = T(0);
  int bad = 0;
  // the step length: as dt_body (one level), from the slots of the last
  // end-of-step pass; the first thread records it and advances the time
  double dtk = 0.0;
  if (A.slots) {
    __shared__ double shs[BX * BY / 64];
    double m = 0.0;
    for (int q = tid; q < NSLOT; q += BX * BY) m = fmax(m, __longlong_as_double((long long)A.slots->smax[q]));
    m = wave_max(m);
    if (tid % 64 == 0) shs[tid / 64] = m;
    __syncthreads();
    double smax = shs[0];
#pragma unroll
    for (int q = 1; q < BX * BY / 64; ++q) smax = fmax(smax, shs[q]);
    double dtl = G.dx / smax;
    if (P.chi > 0.0) dtl = fmin(dtl, G.dx * G.dx / (6.0 * P.chi));
    dtk = P.cfl * dtl;
    if (bk.id == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
      A.slots->dtl[0] = P.cfl * dtl;
      A.slots->dt[0] = dtk;
      A.slots->t += dtk;
    }
  }
  if (POST && bk.id == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
    R.S->tlog = R.S->t;  // the force partials of this state await the log
    R.S->pending = 1;
  }
  if (ok) {
    const int i = 2 * p;
    const T h = (T)(A.fac * (A.slots ? dtk : A.dtp[0]));
    const T rho0 = (T)P.rho0, gm1 = (T)P.gm1, GM = (T)P.GM, eps2 = (T)P.eps2, dx = (T)G.dx;
    const T *rho = A.q[0], *e = A.q[1];
    const int id[3] = {i, j, k};
    const idx_t c = lin(G, i, j, k);
    const V drc = gldv<V>(rho, c), dec = gldv<V>(e, c);
    V xcx;
    xcx.x = xcen<T>(G, 0, i);
    xcx.y = xcen<T>(G, 0, i + 1);
    const T yc = xcen<T>(G, 1, j), zc = xcen<T>(G, 2, k);
    // squared softened distance of cells at (xv, y, z): every cell's distance
    // is formed by this one expression, whichever thread needs it
    auto r2of = [&](V xv, T y, T z) -> V { return xv * xv + y * y + z * z + eps2; };
    const V r2c = r2of(xcx, yc, zc);
    const V dcen = qsqrtv(r2c);
    const T gg = (T)(P.gamma * P.gm1), e0 = (T)P.e0;
    // pair p-1 is the lane before, unless this is the wave's first lane (BX is
    // the wave width) or p the row's first pair (flat tiles)
    const int lane = threadIdx.x;
    auto sound1 = [&](T dr, T de) -> T {
      const T r = rho0 + dr, en = e0 + de;
      if (!(r > T(0)) || !(en > T(0)) || !isfinite(r) || !isfinite(en)) bad = 1;
      return qsqrt(qdiv(gg * en, r));
    };
    auto sound = [&](V dr, V de) -> V {
      V s;
      s.x = sound1(dr.x, de.x);
      s.y = sound1(dr.y, de.y);
      return s;
    };
    auto vmax = [&](V a) { sig = fmax(sig, fmax(a.x, a.y)); };
    auto vabs = [&](V a) -> V {
      V r;
      r.x = fabs(a.x);
      r.y = fabs(a.y);
      return r;
    };
    V cs_own = V(0);
    if (POST) cs_own = sound(drc, dec);
    const T csprev = POST ? dpp_fill<DPP_WAVE_SHR1>(cs_own.y, T(0)) : T(0);
    // the kick of a face pair: cells below (drm, dem) and above (dcr, der) the
    // faces, the coordinate along d of the cell above (xr; the cell below is
    // at xr - dx) and the distances of the cells below (dm) and above (dr_)
    auto kickv = [&](int d, V vf, V drm, V dem, V dcr, V der, V xr, V dm, V dr_) -> V {
      if (KICK) {
        const V rface = rho0 + T(0.5) * (drm + dcr);
        const V gradp = qdiv(gm1 * (der - dem), dx * rface);
        const V xm = xr - dx;
        const V gradphi = qdiv(GM * (xr + xm), dm * dr_ * (dm + dr_));
        vf = vf - h * (gradp + gradphi);
      }
      return vf;
    };
    // the own cells' distances and sound speeds shifted by one lane: lane l
    // gets pair l-1's second cell, cell i-1 (lane 0 forms it itself)
    const T dprev = dpp_fill<DPP_WAVE_SHR1>(dcen.y, T(0));
    auto rebuild = [&](int d, V ppm, V pmc, V drm, V dcr) -> V {
      const T vb = (T)vback(P, d);
      return qdiv(ppm + pmc - vb * (drm + dcr), T(2) * rho0 + drm + dcr);
    };
    // kicked velocities of the low faces of both cells and, with COMP, of
    // their high faces
    V vlo[3], vhi[3];
    // x: faces i and i+1; below them cell i-1 (the own cell i again at x = 0,
    // the background under bc 2) and cell i
    {
      V drm, dem, ppm;
      drm.y = drc.x;
      dem.y = dec.x;
      const T *pm = A.q[2], *pp = A.q[3];
      if (i > 0) {
        drm.x = gld(rho, c - 1);
        dem.x = gld(e, c - 1);
      } else if (BCM == 2) {
        drm.x = T(0);
        dem.x = T(0);
      } else {
        drm.x = drc.x;
        dem.x = dec.x;
      }
      V vf;
      if (REBUILD) {
        const V ppc = gldv<V>(pp, c);
        ppm.y = ppc.x;
        ppm.x = i > 0 ? gld(pp, c - 1) : (BCM == 2 ? T(0) : ppc.x);
        vf = rebuild(0, ppm, gldv<V>(pm, c), drm, drc);
      } else {
        vf = gldv<V>(A.vin[0], c);
      }
      V dmx;
      dmx.y = dcen.x;
      if (i > 0 && lane > 0) {
        dmx.x = dprev;
      } else {
        V xb;
        xb.x = xcen<T>(G, 0, i - 1);  // cell i-1 (a ghost position at x = 0)
        xb.y = xb.x;
        dmx.x = qsqrtv(r2of(xb, yc, zc)).x;
      }
      vf = kickv(0, vf, drm, dem, drc, dec, xcx, dmx, dcen);
      gstv<V>(A.v[0], c, vf);
      vlo[0] = vf;
      if (POST) {
        const V a = vabs((T)vback(P, 0) + vf);
        vmax(a + cs_own);
        if (i > 0) sig = fmax(sig, a.x + (lane > 0 ? csprev : sound1(drm.x, dem.x)));
        sig = fmax(sig, a.y + cs_own.x);
      }
      if (i + 1 == G.n[0] - 1) {
        A.v[0][c + 2] = T(0);  // injection face at x_max carries the wind
        if (POST) sig = fmax(sig, fabs((T)vback(P, 0)) + cs_own.y);
      }
    }
    // y and z: the low faces of both cells, then face n after the last ones
#pragma unroll
    for (int d = 1; d < 3; ++d) {
      const idx_t sd = dstride(G, d);
      const T xd = d == 1 ? yc : zc;
      const T *pm = A.q[2 + 2 * d], *pp = A.q[3 + 2 * d];
      if (BCM == 2 && id[d] == 0) {
        gstv<V>(A.v[d], c, V(0));  // a wall: no normal velocity
        vlo[d] = V(0);
        if (POST) vmax(cs_own);
      } else {
        const idx_t cm = id[d] > 0 ? c - sd : c;
        const V drm = gldv<V>(rho, cm), dem = gldv<V>(e, cm);
        V vf = REBUILD ? rebuild(d, gldv<V>(pp, cm), gldv<V>(pm, c), drm, drc) : gldv<V>(A.vin[d], c);
        // the cell below id (a ghost position at id = 0)
        const T xb = xcen<T>(G, d, id[d] - 1);
        const V dmb = qsqrtv(d == 1 ? r2of(xcx, xb, zc) : r2of(xcx, yc, xb));
        vf = kickv(d, vf, drm, dem, drc, dec, V(xd), dmb, dcen);
        gstv<V>(A.v[d], c, vf);
        vlo[d] = vf;
        if (POST) {
          const V a = vabs((T)vback(P, d) + vf);
          vmax(a + cs_own);
          if (id[d] > 0) vmax(a + sound(drm, dem));
        }
      }
      if (id[d] == G.n[d] - 1) {
        const idx_t cf = c + sd;
        if (BCM == 2) {
          gstv<V>(A.v[d], cf, V(0));  // a wall
          vhi[d] = V(0);
          if (POST) vmax(cs_own);
        } else {
          // both sides read the last cells (zero-gradient outflow)
          const T xr = xcen<T>(G, d, id[d] + 1);
          const V dr_ = qsqrtv(d == 1 ? r2of(xcx, xr, zc) : r2of(xcx, yc, xr));
          V vf = REBUILD ? rebuild(d, gldv<V>(pp, c), gldv<V>(pm, c), drc, drc) : gldv<V>(A.vin[d], cf);
          vf = kickv(d, vf, drc, dec, drc, dec, V(xr), dcen, dr_);
          gstv<V>(A.v[d], cf, vf);
          vhi[d] = vf;
          if (POST) vmax(vabs((T)vback(P, d) + vf) + cs_own);
        }
      } else if (COMP && !(d == 1 && yx)) {
        // face id+1: the low face of the next cells, kicked as their thread
        // does (the own cells below it)
        const idx_t cn = c + sd;
        const T xn = xcen<T>(G, d, id[d] + 1);
        const V r2n = d == 1 ? r2of(xcx, xn, zc) : r2of(xcx, yc, xn);
        vhi[d] = kickv(d, gldv<V>(A.vin[d], cn), drc, dec, gldv<V>(rho, cn), gldv<V>(e, cn), V(xn), dcen,
                       qsqrtv(r2n));
      }
    }
    if (COMP && full) {
      // the pairs above in the block: their low y faces (every thread of a
      // full block is here)
      __shared__ V ylo[BX * BY];
      ylo[tid] = vlo[1];
      __syncthreads();
      if (yx && id[1] != G.n[1] - 1) vhi[1] = ylo[tid + exb];
    }
    if (COMP) {
      // x face i+2: the injection face (a zero departure) at x_max, else the
      // first face of the next pair: the next lane's (it holds that pair
      // unless this is the wave's last lane; a lane past the box holds none,
      // but then this pair is the row's last), else kicked here as the next
      // pair's thread does
      const T vnext = dpp_fill<DPP_WAVE_SHL1>(vlo[0].x, T(0));
      V vx1;
      vx1.x = vlo[0].y;
      if (i + 2 == G.n[0]) {
        vx1.y = T(0);
      } else if (lane < BX - 1) {
        vx1.y = vnext;
      } else {
        const idx_t cn = c + 2;
        const T xn = xcen<T>(G, 0, i + 2);
        const V xnv = V(xn);
        vx1.y = kickv(0, V(gld(A.vin[0], cn)), V(drc.y), V(dec.y), V(gld(rho, cn)), V(gld(e, cn)), xnv,
                      V(dcen.y), qsqrtv(r2of(xnv, yc, zc))).x;
      }
      // compression over the step (as k_compress2)
      const T dtc = (T)(A.cfac * (A.slots ? dtk : A.dtp[0]));
      const V divv = qdiv((vx1 - vlo[0]) + (vhi[1] - vlo[1]) + (vhi[2] - vlo[2]), V(dx));
      const V a = T(0.5) * gm1 * dtc * divv;
      gstv<V>(A.eo, c, qdiv(dec * (T(1) - a) - T(2) * a * (T)P.e0, T(1) + a));
    }
    if (POST) {
      // force of the gas in these cells on the perturber, eq. 18: each cell's
      // term in the storage type, the sum in FP64
      const V w = qdiv(GM * drc * (dx * dx * dx), r2c * dcen);
      fx = (double)(w.x * xcx.x) + (double)(w.y * xcx.y);
      fy = (double)(w.x * yc) + (double)(w.y * yc);
      fz = (double)(w.x * zc) + (double)(w.y * zc);
      if (!isfinite(sig)) bad = 1;
    }
  }
  if (COMP && A.log && bk.id == 0) log_pending_body<BX * BY>(A.part, A.npart, A.log, A.flog);
  if (POST) {
    block_sum3(fx, fy, fz, R.part, R.npart, bk);
    block_signal((double)sig, bad, R.spart, R.S, bk);
    if (threadIdx.x == 0 && threadIdx.y == 0)
      for (unsigned z = bk.n + bk.id; z < (unsigned)R.npart; z += bk.n) {
        R.part[z] = 0.0;
        R.part[R.npart + z] = 0.0;
        R.part[2 * (size_t)R.npart + z] = 0.0;
        R.spart[z] = 0.0;
      }
  }
}

template <typename T, int BCM, bool REBUILD, bool KICK, bool POST, bool COMP = false>
__global__ void __launch_bounds__(BX * BY) __attribute__((amdgpu_waves_per_eu(5)))
k_kick0p(Geo G, Phys P, KickArgs<T> A, RedArgs<T> R) {
  kick0p_body<T, BCM, REBUILD, KICK, POST, COMP>(G, P, A, R, grid_blk());
}

// ------------------------------------------ z pass fused with the step's end
//
// The z pass of a level-0 step without a finer level (bc 1, rows of at most
// 128 cells), the velocity rebuild, the second half kick S(dt/2) of eq. 15
// and the end-of-step reductions in one launch.  One block per (band of ZF_TY
// rows, z segment), 3 ZF_TY + 1 waves, each lane holding two adjacent cells of
// a row:
//  - per band row two walker waves stream the z pass's column segments
//    (march_column, groups {rho, e, P-x, P+x} and {P-y, P+y, P-z, P+z}), and
//    one more walker takes the row below the band ({rho, e, P+y}: the first
//    row's y faces need that row's new values);
//  - per band row one finisher wave takes each plane's new departures from
//    LDS and does what k_kick0p's end-of-step form does: rebuilds the face
//    velocities of its cells' low faces (and of the boundary faces after the
//    last cells), kicks them, forms the signal speeds and the force partials.
// Walkers write plane k into one of two LDS buffers and a barrier hands it
// over: the finishers work on plane k while the walkers compute plane k+1.
// The walk starts one plane below the segment, so that the segment's first
// z faces have their lower cells.  Only the new density and energy (written
// by the first group's walkers) and the face velocities reach HBM; the eight
// transported fields of the z pass never do.
constexpr int ZF_TY = 2;
constexpr int ZF_WAVES = 3 * ZF_TY + 1;

// LDS planes: [2 buffers][ZF_TY + 1 row slots (slot 0: the row below the
// band)][NQ quantities, then the cells' sound speeds and distances from the
// perturber][2 * 64 cells]
constexpr int ZF_CS = NQ, ZF_DIST = NQ + 1, ZF_NQ = NQ + 2;
template <typename T>
struct ZfLds {
  T *base;
  __device__ __forceinline__ T *at(int buf, int r, int m) const {
    return base + ((buf * (ZF_TY + 1) + r) * ZF_NQ + m) * 128;
  }
};

// A walker's sink: the plane's new departures into its row slot of the
// current buffer, the density and energy of a band row (OUT) also to the
// output set -- for the segment's own planes only: the plane below it
// belongs to the segment below, whose block writes it (its value there may
// differ in the last bit, its first face transfer being formed by the walk's
// first step rather than its loop); done() hands the plane over.
// In FP64 the walkers also take a share of the finisher's work on their
// plane (the finisher's work per plane is about twice a walker's, and every
// plane ends in a barrier): the first group the cells' sound speeds (from the
// new density and energy), the second group (and the walker of the row below)
// the cells' distances from the perturber, and the second group the force
// partials of the segment's planes -- with the finisher's expressions, into
// LDS for the finisher of the row and of the row above.  (In FP32 the extra
// registers this costs the walkers lower the occupancy from four waves per
// SIMD to three, which costs more than the balance gains: the finisher keeps
// that work.)
template <typename T>
constexpr bool zf_share() {
  return sizeof(T) == 8;
}
template <typename T>
struct ZfWork {
  const Geo *G;
  const Phys *P;
  typename lanes_of<T, 2>::type xcx;  // x of the lane's two cells
  T yc;                               // y of the row
  double *fx, *fy, *fz;
  int *bad;
};

template <typename T, int GRP, int NG, bool OUT>
struct ZfSink {
  using V = typename lanes_of<T, 2>::type;
  ZfLds<T> L;
  T *rho_out, *e_out;
  int r, x0, buf, plane, c0;
  bool live;
  ZfWork<T> W;
  V drc;
  __device__ __forceinline__ void put(int u, idx_t ic, V val) {
    if (zf_share<T>() && u == 0 && (GRP == 1 || NG == 3)) {
      // distances of the plane's cells (and, second group, their force terms)
      const T zcen = xcen<T>(*W.G, 2, plane);
      const T eps2 = (T)W.P->eps2;
      const V r2c = W.xcx * W.xcx + W.yc * W.yc + zcen * zcen + eps2;
      const V dcen = qsqrtv(r2c);
      *reinterpret_cast<V *>(L.at(buf, r, ZF_DIST) + x0) = dcen;
      if (GRP == 1 && live && plane >= c0) {
        const T GM = (T)W.P->GM, dx = (T)W.G->dx;
        const V w = qdiv(GM * val * (dx * dx * dx), r2c * dcen);
        *W.fx += (double)(w.x * W.xcx.x) + (double)(w.y * W.xcx.y);
        *W.fy += (double)(w.x * W.yc) + (double)(w.y * W.yc);
        *W.fz += (double)(w.x * zcen) + (double)(w.y * zcen);
      }
    }
    if (u == 0 && GRP != 0) return;  // the first group holds the density
    const int m = u == 0 ? 0 : group_q(NG, GRP, u - 1);
    *reinterpret_cast<V *>(L.at(buf, r, m) + x0) = val;
    if (OUT && m <= 1 && live && plane >= c0) gstv<V>(m == 0 ? rho_out : e_out, ic, val);
    if (zf_share<T>() && GRP == 0 && m == 0) drc = val;
    if (zf_share<T>() && GRP == 0 && m == 1) {
      // sound speeds of the plane's cells (the health check on live lanes)
      const T rho0 = (T)W.P->rho0, e0 = (T)W.P->e0, gg = (T)(W.P->gamma * W.P->gm1);
      V cs;
      {
        const T rr = rho0 + drc.x, en = e0 + val.x;
        if (live && (!(rr > T(0)) || !(en > T(0)) || !isfinite(rr) || !isfinite(en))) *W.bad = 1;
        cs.x = qsqrt(qdiv(gg * en, rr));
      }
      {
        const T rr = rho0 + drc.y, en = e0 + val.y;
        if (live && (!(rr > T(0)) || !(en > T(0)) || !isfinite(rr) || !isfinite(en))) *W.bad = 1;
        cs.y = qsqrt(qdiv(gg * en, rr));
      }
      *reinterpret_cast<V *>(L.at(buf, r, ZF_CS) + x0) = cs;
    }
  }
  __device__ __forceinline__ void done(int) {
    __syncthreads();
    buf ^= 1;
    ++plane;
  }
};

template <typename T, int GRP, int NG, bool OUT>
__device__ __forceinline__ void zf_walk(const Geo &G, const Phys &P, const MarchArgs<T> &M, ZfLds<T> L, int r,
                                        int row, int x0, bool live, int cs, int c0, int c1, ZfWork<T> W) {
  using V = typename lanes_of<T, 2>::type;
  // lanes past the row end read the row's first cells (in bounds, unused)
  const idx_t base = lin(G, live ? x0 : 0, row, 0);
  const T *qi = M.qi[0];
  ColSrc<T, V, 2, 1, GRP, NG> src{qi, {M.qi[group_q(NG, GRP, 0)], M.qi[group_q(NG, GRP, 1)],
                                       M.qi[group_q(NG, GRP, 2)], M.qi[group_q(NG, GRP, 3)]},
                                  base, (idx_t)G.sz, G.n[2]};
  ZfSink<T, GRP, NG, OUT> snk{L, M.qo[0], M.qo[1], r, x0, 0, cs, c0, live, W, V(0)};
  march_column<T, 2, 1, GRP, false, 2, NG>(G, P, M, live ? x0 : 0, row, cs, c1, src, snk, live);
}

template <typename T>
__device__ __forceinline__ void zfinish_body(Geo G, Phys P, MarchArgs<T> M, KickArgs<T> K, RedArgs<T> R, Blk bk) {
  using V = typename lanes_of<T, 2>::type;
  __shared__ __align__(16) T zl[2 * (ZF_TY + 1) * ZF_NQ * 128];
  __shared__ double sh[5][ZF_WAVES];
  const ZfLds<T> L{zl};
  const int lane = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
  // block -> (row band, z segment): each XCD (block h runs on XCD h % 8)
  // takes one contiguous range of bands through all segments
  const int nch = (G.n[2] + M.chunk - 1) / M.chunk;
  const unsigned N = bk.n, h = bk.id;
  const unsigned q8 = N / 8, r8 = N % 8, xcd = h % 8, s8 = h / 8;
  const unsigned Lg = (xcd < r8) ? xcd * (q8 + 1) + s8 : r8 * (q8 + 1) + (xcd - r8) * q8 + s8;
  const int band = (int)(Lg / (unsigned)nch), ch = (int)(Lg % (unsigned)nch);
  const int j0 = band * ZF_TY;
  const int c0 = ch * M.chunk, c1 = min(c0 + M.chunk, G.n[2]);
  const int cs = c0 > 0 ? c0 - 1 : 0;  // first plane walked
  const int x0 = 2 * lane;
  const bool live = x0 < G.n[0];
  double fx = 0.0, fy = 0.0, fz = 0.0;
  T sig = T(0);
  int bad = 0;
  if (bk.id == 0 && lane == 0 && wv == 0) {
    R.S->tlog = R.S->t;  // the force partials of this state await the log
    R.S->pending = 1;
  }
  if (wv <= 2 * ZF_TY) {
    V xw;
    xw.x = xcen<T>(G, 0, x0);
    xw.y = xcen<T>(G, 0, x0 + 1);
    if (wv == 0) {
      // the row below the band (row 0 again for the first band: its sound
      // speeds and distances are not used there)
      const int jb = max(j0 - 1, 0);
      zf_walk<T, 0, 3, false>(G, P, M, L, 0, jb, x0, live, cs, c0, c1,
                              ZfWork<T>{&G, &P, xw, xcen<T>(G, 1, jb), &fx, &fy, &fz, &bad});
    } else {
      const int y = (wv - 1) >> 1;
      const ZfWork<T> W{&G, &P, xw, xcen<T>(G, 1, j0 + y), &fx, &fy, &fz, &bad};
      if ((wv - 1) & 1) zf_walk<T, 1, 2, false>(G, P, M, L, 1 + y, j0 + y, x0, live, cs, c0, c1, W);
      else zf_walk<T, 0, 2, true>(G, P, M, L, 1 + y, j0 + y, x0, live, cs, c0, c1, W);
    }
  } else {
    // finisher of band row y, cells x0, x0 + 1 of row j
    const int y = wv - 1 - 2 * ZF_TY, j = j0 + y, r = 1 + y;
    const int i = x0;
    const T h = (T)(K.fac * K.dtp[0]);
    const T rho0 = (T)P.rho0, gm1 = (T)P.gm1, GM = (T)P.GM, eps2 = (T)P.eps2, dx = (T)G.dx;
    const T gg = (T)(P.gamma * P.gm1), e0 = (T)P.e0;
    V xcx;
    xcx.x = xcen<T>(G, 0, i);
    xcx.y = xcen<T>(G, 0, i + 1);
    const T yc = xcen<T>(G, 1, j);
    auto r2of = [&](V xv, T yy, T zz) -> V { return xv * xv + yy * yy + zz * zz + eps2; };
    auto sound1 = [&](T dr, T de) -> T {
      const T rr = rho0 + dr, en = e0 + de;
      if (!(rr > T(0)) || !(en > T(0)) || !isfinite(rr) || !isfinite(en)) bad = 1;
      return qsqrt(qdiv(gg * en, rr));
    };
    auto sound = [&](V dr, V de) -> V {
      V s;
      s.x = sound1(dr.x, de.x);
      s.y = sound1(dr.y, de.y);
      return s;
    };
    auto vmax = [&](V a) { sig = fmax(sig, fmax(a.x, a.y)); };
    auto vabs = [&](V a) -> V {
      V o;
      o.x = fabs(a.x);
      o.y = fabs(a.y);
      return o;
    };
    auto kickv = [&](V vf, V drm, V dem, V dcr, V der, V xr, V dm, V dr_) -> V {
      const V rface = rho0 + T(0.5) * (drm + dcr);
      const V gradp = qdiv(gm1 * (der - dem), dx * rface);
      const V xm = xr - dx;
      const V gradphi = qdiv(GM * (xr + xm), dm * dr_ * (dm + dr_));
      return vf - h * (gradp + gradphi);
    };
    auto rebuild = [&](int d, V ppm, V pmc, V drm, V dcr) -> V {
      const T vb = (T)vback(P, d);
      return qdiv(ppm + pmc - vb * (drm + dcr), T(2) * rho0 + drm + dcr);
    };
    auto ldv = [&](int buf, int rr, int m) -> V { return *reinterpret_cast<const V *>(L.at(buf, rr, m) + x0); };
    // the cells below the z faces: new departures, sound speeds and
    // distances of the plane before
    V zr = V(0), ze = V(0), zp = V(0), zc = V(0), zd = V(0);
    for (int k = cs; k < c1; ++k) {
      __syncthreads();
      const int buf = (k - cs) & 1;
      if (!live) continue;
      const V drc = ldv(buf, r, 0), dec = ldv(buf, r, 1);
      const T zcen = xcen<T>(G, 2, k);
      V dcen, cs_own, r2c;
      if (zf_share<T>()) {
        dcen = ldv(buf, r, ZF_DIST);  // the walkers' distances and sound speeds
        cs_own = ldv(buf, r, ZF_CS);
      } else {
        r2c = r2of(xcx, yc, zcen);
        dcen = qsqrtv(r2c);
        cs_own = sound(drc, dec);
      }
      const V ppz = ldv(buf, r, 7);
      if (k >= c0) {
        const idx_t c = lin(G, i, j, k);
        const T csprev = dpp_fill<DPP_WAVE_SHR1>(cs_own.y, T(0));
        const T dprev = dpp_fill<DPP_WAVE_SHR1>(dcen.y, T(0));
        // x: faces i and i+1; below them cell i-1 (the cell itself at x = 0) and cell i
        {
          V drm, dem, ppm;
          drm.y = drc.x;
          dem.y = dec.x;
          const V ppc = ldv(buf, r, 3);
          ppm.y = ppc.x;
          if (i > 0) {
            drm.x = L.at(buf, r, 0)[x0 - 1];
            dem.x = L.at(buf, r, 1)[x0 - 1];
            ppm.x = L.at(buf, r, 3)[x0 - 1];
          } else {
            drm.x = drc.x;
            dem.x = dec.x;
            ppm.x = ppc.x;
          }
          V vf = rebuild(0, ppm, ldv(buf, r, 2), drm, drc);
          V dmx;
          dmx.y = dcen.x;
          if (i > 0 && lane > 0) {
            dmx.x = dprev;
          } else {
            V xb;
            xb.x = xcen<T>(G, 0, i - 1);  // cell i-1 (a ghost position at x = 0)
            xb.y = xb.x;
            dmx.x = qsqrtv(r2of(xb, yc, zcen)).x;
          }
          vf = kickv(vf, drm, dem, drc, dec, xcx, dmx, dcen);
          gstv<V>(K.v[0], c, vf);
          const V a = vabs((T)vback(P, 0) + vf);
          vmax(a + cs_own);
          if (i > 0) sig = fmax(sig, a.x + (lane > 0 ? csprev : sound1(drm.x, dem.x)));
          sig = fmax(sig, a.y + cs_own.x);
          if (i + 1 == G.n[0] - 1) {
            K.v[0][c + 2] = T(0);  // injection face at x_max carries the wind
            sig = fmax(sig, fabs((T)vback(P, 0)) + cs_own.y);
          }
        }
        // y: face j (the row below from slot r-1; the row itself at y = 0),
        // and face n after the last row
        {
          const V pmy = ldv(buf, r, 4), ppy = ldv(buf, r, 5);
          const bool lo = j > 0;
          const V drm = lo ? ldv(buf, r - 1, 0) : drc, dem = lo ? ldv(buf, r - 1, 1) : dec;
          V vf = rebuild(1, lo ? ldv(buf, r - 1, 5) : ppy, pmy, drm, drc);
          // the row below: its walkers' distances and sound speeds (the ghost
          // row's distance at y = 0)
          const V dmb = zf_share<T>() && lo ? ldv(buf, r - 1, ZF_DIST)
                                            : qsqrtv(r2of(xcx, xcen<T>(G, 1, j - 1), zcen));
          vf = kickv(vf, drm, dem, drc, dec, V(yc), dmb, dcen);
          gstv<V>(K.v[1], c, vf);
          const V a = vabs(vf);
          vmax(a + cs_own);
          if (lo) vmax(a + (zf_share<T>() ? ldv(buf, r - 1, ZF_CS) : sound(drm, dem)));
          if (j == G.n[1] - 1) {
            const T xr = xcen<T>(G, 1, j + 1);
            const V dr_ = qsqrtv(r2of(xcx, xr, zcen));
            V vh = rebuild(1, ppy, pmy, drc, drc);
            vh = kickv(vh, drc, dec, drc, dec, V(xr), dcen, dr_);
            gstv<V>(K.v[1], c + (idx_t)G.sy, vh);
            vmax(vabs(vh) + cs_own);
          }
        }
        // z: face k (the plane before from the walk's previous plane; the
        // plane itself at z = 0), and face n after the last plane
        {
          const V pmz = ldv(buf, r, 6);
          const bool lo = k > 0;
          const V drm = lo ? zr : drc, dem = lo ? ze : dec;
          V vf = rebuild(2, lo ? zp : ppz, pmz, drm, drc);
          const V dmb = lo ? zd : qsqrtv(r2of(xcx, yc, xcen<T>(G, 2, k - 1)));
          vf = kickv(vf, drm, dem, drc, dec, V(zcen), dmb, dcen);
          gstv<V>(K.v[2], c, vf);
          const V a = vabs(vf);
          vmax(a + cs_own);
          if (lo) vmax(a + zc);
          if (k == G.n[2] - 1) {
            const T xr = xcen<T>(G, 2, k + 1);
            const V dr_ = qsqrtv(r2of(xcx, yc, xr));
            V vh = rebuild(2, ppz, pmz, drc, drc);
            vh = kickv(vh, drc, dec, drc, dec, V(xr), dcen, dr_);
            gstv<V>(K.v[2], c + (idx_t)G.sz, vh);
            vmax(vabs(vh) + cs_own);
          }
        }
        // force of the gas in these cells on the perturber, eq. 18: each
        // cell's term in the storage type, the sum in FP64 (in FP64 formed by
        // the second group's walker)
        if (!zf_share<T>()) {
          const V w = qdiv(GM * drc * (dx * dx * dx), r2c * dcen);
          fx += (double)(w.x * xcx.x) + (double)(w.y * xcx.y);
          fy += (double)(w.x * yc) + (double)(w.y * yc);
          fz += (double)(w.x * zcen) + (double)(w.y * zcen);
        }
      }
      zr = drc;
      ze = dec;
      zp = ppz;
      zc = cs_own;
      zd = dcen;
    }
    if (!isfinite(sig)) bad = 1;
  }
  // block sums of the force partials and maximum of the signal speeds (every
  // wave takes part; walkers contribute zeros), written to the block's slot;
  // the slots of the one-cell-per-thread grid past the launch are zeroed
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  double sg = wave_max(bad ? 0.0 : (double)sig);
  const bool anybad = __any(bad);
  if (lane == 0) {
    sh[0][wv] = fx;
    sh[1][wv] = fy;
    sh[2][wv] = fz;
    sh[3][wv] = sg;
    if (anybad) atomicOr(&R.S->health, 1);
  }
  __syncthreads();
  if (lane == 0 && wv == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, m = 0.0;
    for (int w = 0; w < ZF_WAVES; ++w) {
      s0 += sh[0][w];
      s1 += sh[1][w];
      s2 += sh[2][w];
      m = fmax(m, sh[3][w]);
    }
    const long nb = R.npart;
    R.part[bk.id] = s0;
    R.part[nb + bk.id] = s1;
    R.part[2 * nb + bk.id] = s2;
    R.spart[bk.id] = m;
    __hip_atomic_fetch_max(&R.S->smax[bk.id & (NSLOT - 1)], (unsigned long long)__double_as_longlong(m),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (unsigned z = bk.n + bk.id + (unsigned)(wv * 64 + lane) * bk.n; z < (unsigned)R.npart;
       z += bk.n * 64u * ZF_WAVES) {
    R.part[z] = 0.0;
    R.part[R.npart + z] = 0.0;
    R.part[2 * (size_t)R.npart + z] = 0.0;
    R.spart[z] = 0.0;
  }
}

template <typename T>
__global__ void __launch_bounds__(64 * ZF_WAVES) k_zfinish(Geo G, Phys P, MarchArgs<T> M, KickArgs<T> K,
                                                            RedArgs<T> R) {
  zfinish_body<T>(G, P, M, K, R, grid_blk());
}

struct DtArgs {
  // advance: 0 set dt, 1 set dt and advance the time, 2 per-level limits only
  double dx[MAXLEV];
  const double *part[MAXLEV];  // per-block maximum signal speeds of each level
  int npart[MAXLEV];
  int nl;
  int advance;
};

// coarse step cfl * min_l 2^l min(dx_l / smax_l, dx_l^2 / (6 chi)) (eq. 55, xi = 2)
// thread 0: the step lengths from each level's largest signal speed smax
__device__ void dt_finish(const Phys &P, const DtArgs &A, Scal *S, const double *smax) {
  double best = INFINITY;
  for (int l = 0; l < A.nl; ++l) {
    double dtl = A.dx[l] / smax[l];
    if (P.chi > 0.0) dtl = fmin(dtl, A.dx[l] * A.dx[l] / (6.0 * P.chi));
    S->dtl[l] = P.cfl * dtl;  // the level's own limit (for the sub-cycling criterion)
    dtl = ldexp(dtl, l);
    best = fmin(best, dtl);
  }
  if (A.advance == 2) return;  // limits only: the host sets the schedule
  const double dt0 = P.cfl * best;
  for (int l = 0; l < A.nl; ++l) S->dt[l] = ldexp(dt0, -l);
  if (A.advance) S->t += dt0;
}

__device__ void dt_body(const Phys &P, const DtArgs &A, Scal *S) {
  __shared__ double sh[FW];
  __shared__ double smax[MAXLEV];
  for (int l = 0; l < A.nl; ++l) {
    const double *p = A.part[l];
    const int n = A.npart[l];
    double m = 0.0;
    int b = threadIdx.x;
    for (; b + 7 * FT < n; b += 8 * FT) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = p[b + u * FT];
#pragma unroll
      for (int u = 0; u < 8; ++u) m = fmax(m, x[u]);
    }
    for (; b < n; b += FT) m = fmax(m, p[b]);
    m = wave_max(m);
    if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = sh[0];
      for (int v = 1; v < FW; ++v) t = fmax(t, sh[v]);
      smax[l] = t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) dt_finish(P, A, S, smax);
}

__global__ void __launch_bounds__(FT) k_dt_final(Phys P, DtArgs A, Scal *S) { dt_body(P, A, S); }

// Between two steps: the force of the state just reached (logged at its
// time), then the next step's time step from the same state's signal speeds.
// One pass reads the partials of both (the force planes and the signal
// speeds of a block side by side, all in flight together); the sums keep the
// order of final3_body and the maxima are those of dt_body.
template <bool do_force, bool do_dt>
__global__ void __launch_bounds__(FT) k_step_final(Phys P, FinalArgs F, DtArgs D, Scal *S) {
  __shared__ double sh[3][FW];
  __shared__ double shm[MAXLEV][FW];
  __shared__ double smax[MAXLEV];
  const int t = threadIdx.x, w = t / 64;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int l = 0; l < D.nl; ++l) {
    const double *p = F.part[l], *q = D.part[l];
    const int n = D.npart[l];
    double m = 0.0;
    int b = t;
    for (; b + 7 * FT < n; b += 8 * FT) {
      double x[8][3], y[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (do_force)
#pragma unroll
          for (int c = 0; c < 3; ++c) x[u][c] = p[(size_t)c * n + b + u * FT];
        if (do_dt) y[u] = q[b + u * FT];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (do_force) {
          s0 += x[u][0];
          s1 += x[u][1];
          s2 += x[u][2];
        }
        if (do_dt) m = fmax(m, y[u]);
      }
    }
    for (; b < n; b += FT) {
      if (do_force) {
        s0 += p[b];
        s1 += p[(size_t)n + b];
        s2 += p[2 * (size_t)n + b];
      }
      if (do_dt) m = fmax(m, q[b]);
    }
    m = wave_max(m);
    if (t % 64 == 0) shm[l][w] = m;
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (t % 64 == 0) {
    sh[0][w] = s0;
    sh[1][w] = s1;
    sh[2][w] = s2;
  }
  __syncthreads();
  if (t != 0) return;
  if (do_force) final3_finish(F, sh);
  if (do_dt) {
    for (int l = 0; l < D.nl; ++l) {
      double v = shm[l][0];
      for (int u = 1; u < FW; ++u) v = fmax(v, shm[l][u]);
      smax[l] = v;
    }
    dt_finish(P, D, S, smax);
  }
}

__global__ void k_zero(unsigned int *p, size_t n) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) p[t] = 0u;
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

// A finer level's launch computes only the entries within its stage's margin
// G.mg of the active range (the entries later stages and the level's
// observers need); the range [lo, hi) along d, of cells or (face) of faces
// normal to d, is cut to it.
inline void clip_margin(const Geo &G, int d, bool face, int &lo, int &hi) {
  lo = max(lo, -G.mg[d]);
  hi = min(hi, G.n[d] + G.mg[d] + (face ? 1 : 0));
}
inline Box clip_cells(const Geo &G, Box b) {
  for (int d = 0; d < 3; ++d) clip_margin(G, d, false, b.lo[d], b.hi[d]);
  return b;
}

template <typename T>
inline T *tp(void *p) {
  return reinterpret_cast<T *>(p);
}

}  // namespace

// launch only non-empty grids
// While a recorder is set (the engine's dry run of a step), every launch that
// is not one of the batched stages marks the recording failed and is not made.
#define DFK_LAUNCH(K, GR, BL, ST, ...)                                      \
  do {                                                                      \
    if (g_rec) {                                                            \
      g_rec->failed = true;                                                 \
      break;                                                                \
    }                                                                       \
    dim3 g_ = (GR);                                                         \
    if (!empty_grid(g_)) hipLaunchKernelGGL(K, g_, BL, 0, ST, __VA_ARGS__); \
  } while (0)

thread_local Recorder *g_rec = nullptr;

// in a recording: add the launch of stage kind `kind` with its arguments
template <typename E>
bool record(int kind, const E &e) {
  if (!g_rec) return false;
  if (e.nblk == 0) return true;  // an empty launch is no launch
  JobRec r;
  r.kind = kind;
  r.nblk = e.nblk;
  r.bytes.resize(sizeof(E));
  std::memcpy(r.bytes.data(), &e, sizeof(E));
  g_rec->recs.push_back(std::move(r));
  return true;
}

// ============================================================ batched jobs
// One launch for one stage of several single-level runs (the engine's batched
// step): run r owns the blocks [start[r], start[r+1]) of the launch, each
// run's count padded to a multiple of 8 so that its blocks keep their XCD
// placement (block h on XCD h % 8), and its launch arguments are entry r of
// the table; block b runs as block b - start[r] of the run's own launch.  The
// bodies are those of the single-run kernels, so a run's results do not
// depend on the other runs in the launch.
template <typename T>
struct KcJob {
  Geo G;
  Phys P;
  KickArgs<T> A;
  RedArgs<T> R;
  unsigned nblk;
};
template <typename T>
struct DiffJob {
  Geo G;
  Phys P;
  DiffArgs<T> A;
  unsigned nblk;
};
template <typename T>
struct XyJob {
  Geo G;
  Phys P;
  PassArgs<T> A;
  MarchArgs<T> M;
  unsigned nblk;
};
template <typename T>
struct ZfJob {
  Geo G;
  Phys P;
  MarchArgs<T> M;
  KickArgs<T> K;
  RedArgs<T> R;
  unsigned nblk;
};
struct LogJob {
  const double *part;
  int npart;
  Scal *S;
  double *flog;
  unsigned nblk;
};

// stage kinds of the batched launches (dfk.h), per storage type and form
template <typename T>
constexpr int jk_kc(int bc) {
  return (sizeof(T) == 4 ? JK_KC_F1 : JK_KC_D1) + (bc == 2 ? 1 : 0);
}
template <typename T>
constexpr int jk_df(int bc) {
  return (sizeof(T) == 4 ? JK_DF_F1 : JK_DF_D1) + (bc == 2 ? 1 : 0);
}
template <typename T>
constexpr int jk_xy(int n) {  // the k_xyshared form transport_xy_t takes for rows of n cells
  return (sizeof(T) == 4 ? JK_XY_F1P : JK_XY_D1P) + (n > BX ? 2 : 0) + ((n == BX || n == 2 * BX) ? 1 : 0);
}
template <typename T>
constexpr int jk_zf() {
  return sizeof(T) == 4 ? JK_ZF_F : JK_ZF_D;
}

template <typename E>
struct JobTab {
  const E *__restrict__ e;
  const unsigned *__restrict__ start;  // n + 1 block offsets
  int n;
};

// the run of block b and the block's place in the run's launch; false for a
// padding block
template <typename E>
__device__ __forceinline__ bool job_of(const JobTab<E> &t, unsigned b, int &r, Blk &bk) {
  int lo = 0, hi = t.n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (t.start[mid] <= b) lo = mid;
    else hi = mid;
  }
  r = lo;
  bk.id = b - t.start[lo];
  bk.n = t.e[lo].nblk;
  return bk.id < bk.n;
}

template <typename T, int BCM>
__global__ void __launch_bounds__(BX * BY) __attribute__((amdgpu_waves_per_eu(5)))
k_kick_compress_jobs(JobTab<KcJob<T>> t) {
  int r;
  Blk bk;
  if (!job_of(t, blockIdx.x, r, bk)) return;
  const KcJob<T> &J = t.e[r];
  kick0p_body<T, BCM, false, true, false, true>(J.G, J.P, J.A, J.R, bk);
}

template <typename T, int BC>
__global__ void __launch_bounds__(BX * BY) k_diffuse_heat2_jobs(JobTab<DiffJob<T>> t) {
  int r;
  Blk bk;
  if (!job_of(t, blockIdx.x, r, bk)) return;
  const DiffJob<T> &J = t.e[r];
  diffuse_heat2_body<T, BC>(J.G, J.P, J.A, bk);
}

template <typename T, int W, bool FULL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_xyshared_jobs(JobTab<XyJob<T>> t) {
  int r;
  Blk bk;
  if (!job_of(t, blockIdx.x, r, bk)) return;
  const XyJob<T> &J = t.e[r];
  xyshared_body<T, W, FULL, false>(J.G, J.P, J.A, J.M, bk);
}

template <typename T>
__global__ void __launch_bounds__(64 * ZF_WAVES) k_zfinish_jobs(JobTab<ZfJob<T>> t) {
  int r;
  Blk bk;
  if (!job_of(t, blockIdx.x, r, bk)) return;
  const ZfJob<T> &J = t.e[r];
  zfinish_body<T>(J.G, J.P, J.M, J.K, J.R, bk);
}

__global__ void __launch_bounds__(FT) k_log_pending_jobs(JobTab<LogJob> t) {
  const LogJob &J = t.e[blockIdx.x];
  log_pending_body<FT>(J.part, J.npart, J.S, J.flog);
}

// ======================================================================
// launchers (templated on the storage type, dispatched on P.fp32)

template <typename T>
static void init_state_t(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, uint64_t seed,
                         double amp) {
  InitArgs<T> A;
  A.b = full_box(G);
  A.rho = tp<T>(B.q[cur][0]);
  A.e = tp<T>(B.q[cur][1]);
  A.vx = tp<T>(B.v[0]);
  A.vy = tp<T>(B.v[1]);
  A.vz = tp<T>(B.v[2]);
  A.seed = seed;
  A.amp = amp;
  DFK_LAUNCH(k_init<T>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
}
void init_state(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, uint64_t seed, double amp) {
  if (P.fp32) init_state_t<float>(st, G, P, B, cur, seed, amp);
  else init_state_t<double>(st, G, P, B, cur, seed, amp);
}

template <typename T>
static RedArgs<T> red_args(const Geo &G, LevBufs &B, int cur, Scal *S);

template <typename T>
static void kick_t(hipStream_t st, const Geo &G, const Phys &P, void *const *q, void *const *v, const double *dtp,
                   double fac, bool rebuild, bool do_kick, LevBufs *post = nullptr, Scal *S = nullptr,
                   Scal *slots = nullptr) {
  KickArgs<T> A{};
  A.slots = nullptr;
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
      if (!G.bc) clip_margin(G, e, d == e, A.flo[d][e], A.fhi[d][e]);
    }
  for (int e = 0; e < 3; ++e) {
    A.b.lo[e] = min(A.flo[0][e], min(A.flo[1][e], A.flo[2][e]));
    A.b.hi[e] = max(A.fhi[0][e], max(A.fhi[1][e], A.fhi[2][e]));
  }
  for (int m = 0; m < NQ; ++m) A.q[m] = tp<T>(q[m]);
  for (int d = 0; d < 3; ++d) {
    A.v[d] = tp<T>(v[d]);
    A.vin[d] = A.v[d];
  }
  A.dtp = dtp;
  A.fac = fac;
  const dim3 bl(BX, BY);
  if (G.bc) {
    // level 0: one thread per pair of active cells (boundary faces by the
    // last cells)
    A.b = active_box(G);
    RedArgs<T> R{};
    if (post) R = red_args<T>(G, *post, 0, S);
    A.b.hi[0] = G.n[0] / 2;  // level-0 rows have an even length
    A.slots = slots;
    const dim3 gr = grid_of_flat(A.b);
    if (G.bc == 2) {
      if (rebuild && do_kick && post) DFK_LAUNCH((k_kick0p<T, 2, true, true, true>), gr, bl, st, G, P, A, R);
      else if (rebuild && do_kick) DFK_LAUNCH((k_kick0p<T, 2, true, true, false>), gr, bl, st, G, P, A, R);
      else if (rebuild) DFK_LAUNCH((k_kick0p<T, 2, true, false, false>), gr, bl, st, G, P, A, R);
      else DFK_LAUNCH((k_kick0p<T, 2, false, true, false>), gr, bl, st, G, P, A, R);
    } else {
      if (rebuild && do_kick && post) DFK_LAUNCH((k_kick0p<T, 1, true, true, true>), gr, bl, st, G, P, A, R);
      else if (rebuild && do_kick) DFK_LAUNCH((k_kick0p<T, 1, true, true, false>), gr, bl, st, G, P, A, R);
      else if (rebuild) DFK_LAUNCH((k_kick0p<T, 1, true, false, false>), gr, bl, st, G, P, A, R);
      else DFK_LAUNCH((k_kick0p<T, 1, false, true, false>), gr, bl, st, G, P, A, R);
    }
    return;
  }
  const dim3 gr = grid_of_flat(A.b);
  {
    if (rebuild && do_kick) DFK_LAUNCH((k_kick<T, true, true>), gr, bl, st, G, P, A);
    else if (rebuild) DFK_LAUNCH((k_kick<T, true, false>), gr, bl, st, G, P, A);
    else DFK_LAUNCH((k_kick<T, false, true>), gr, bl, st, G, P, A);
  }
}

void kick(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp, double fac,
          Scal *slots) {
  if (!G.bc) slots = nullptr;  // the slots belong to level 0
  if (P.fp32) kick_t<float>(st, G, P, B.q[cur], B.v, dtp, fac, false, true, nullptr, nullptr, slots);
  else kick_t<double>(st, G, P, B.q[cur], B.v, dtp, fac, false, true, nullptr, nullptr, slots);
}

template <typename T>
static void kick_compress_t(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
                            double kfac, double cfac, Scal *slots, double *flog) {
  KickArgs<T> A{};
  A.b = active_box(G);
  A.b.hi[0] = G.n[0] / 2;  // cell pairs: level-0 rows have an even length
  for (int m = 0; m < NQ; ++m) A.q[m] = tp<T>(B.q[cur][m]);
  for (int d = 0; d < 3; ++d) {
    A.v[d] = tp<T>(B.vk[d]);
    A.vin[d] = tp<T>(B.v[d]);
  }
  A.dtp = dtp;
  A.fac = kfac;
  A.slots = slots;
  A.eo = tp<T>(B.etmp);
  A.cfac = cfac;
  A.log = slots;
  A.part = B.part;
  A.npart = (int)part_count(G);
  A.flog = flog;
  RedArgs<T> R{};
  const dim3 gr = grid_of_flat(A.b), bl(BX, BY);
  if (record(jk_kc<T>(G.bc), KcJob<T>{G, P, A, R, gr.x})) return;
  if (G.bc == 2) DFK_LAUNCH((k_kick0p<T, 2, false, true, false, true>), gr, bl, st, G, P, A, R);
  else DFK_LAUNCH((k_kick0p<T, 1, false, true, false, true>), gr, bl, st, G, P, A, R);
}
template <typename T>
static void kick_compress_fine_t(hipStream_t st, const Geo &Gk, const Geo &Gc, const Phys &P, LevBufs &B, int cur,
                                 const double *dtp, double kfac, double cfac) {
  KickArgs<T> A{};
  // the kick's face ranges within Gk's margins (as kick_t), the compression's
  // cells within Gc's (as compress_t)
  for (int d = 0; d < 3; ++d)
    for (int e = 0; e < 3; ++e) {
      A.flo[d][e] = -Gk.g + (d == e ? 1 : 0);
      A.fhi[d][e] = Gk.n[e] + Gk.g;
      clip_margin(Gk, e, d == e, A.flo[d][e], A.fhi[d][e]);
    }
  Box ub;
  for (int e = 0; e < 3; ++e) {
    ub.lo[e] = min(A.flo[0][e], min(A.flo[1][e], A.flo[2][e]));
    ub.hi[e] = max(A.fhi[0][e], max(A.fhi[1][e], A.fhi[2][e]));
  }
  const Box cb = clip_cells(Gc, uniform_box(Gc, 0, 1));
  for (int e = 0; e < 3; ++e) {
    ub.lo[e] = min(ub.lo[e], cb.lo[e]);
    ub.hi[e] = max(ub.hi[e], cb.hi[e]);
  }
  for (int m = 0; m < NQ; ++m) A.q[m] = tp<T>(B.q[cur][m]);
  for (int d = 0; d < 3; ++d) {
    A.v[d] = tp<T>(B.vk[d]);
    A.vin[d] = tp<T>(B.v[d]);
  }
  A.dtp = dtp;
  A.fac = kfac;
  A.eo = tp<T>(B.etmp);
  A.cfac = cfac;
  DFK_LAUNCH(k_kick_compress_fine<T>, grid_of_flat<BX - 1>(ub), dim3(BX, BY), st, Gk, P, A, cb, ub);
}
void kick_compress_fine(hipStream_t st, const Geo &Gk, const Geo &Gc, const Phys &P, LevBufs &B, int cur,
                        const double *dtp, double kfac, double cfac) {
  if (P.fp32) kick_compress_fine_t<float>(st, Gk, Gc, P, B, cur, dtp, kfac, cfac);
  else kick_compress_fine_t<double>(st, Gk, Gc, P, B, cur, dtp, kfac, cfac);
}

void kick_compress(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp, double kfac,
                   double cfac, Scal *slots, double *flog) {
  if (P.fp32) kick_compress_t<float>(st, G, P, B, cur, dtp, kfac, cfac, slots, flog);
  else kick_compress_t<double>(st, G, P, B, cur, dtp, kfac, cfac, slots, flog);
}

void rebuild_kick(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src, const double *dtp,
                  double fac, bool do_kick, Scal *post) {
  LevBufs *pb = (post && G.bc && do_kick) ? &B : nullptr;
  if (P.fp32) kick_t<float>(st, G, P, B.q[src], B.v, dtp, fac, true, do_kick, pb, post);
  else kick_t<double>(st, G, P, B.q[src], B.v, dtp, fac, true, do_kick, pb, post);
}

template <typename T>
static void compress_t(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
                       double fac, Scal *log, double *flog) {
  CellArgs<T> A;
  A.b = G.bc ? active_box(G) : clip_cells(G, uniform_box(G, 0, 1));
  A.e = tp<T>(B.q[cur][1]);
  for (int d = 0; d < 3; ++d) A.v[d] = tp<T>(B.v[d]);
  A.dtp = dtp;
  A.fac = fac;
  A.log = log;
  A.part = B.part;
  A.npart = (int)part_count(G);
  A.flog = flog;
  if (G.bc) {
    A.b.hi[0] = G.n[0] / 2;  // cell pairs: level-0 rows have an even length
    DFK_LAUNCH(k_compress2<T>, grid_of_flat(A.b), dim3(BX, BY), st, G, P, A);
    return;
  }
  DFK_LAUNCH(k_compress<T>, grid_of_flat(A.b), dim3(BX, BY), st, G, P, A);
}
void compress(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp, double fac,
              Scal *log, double *flog) {
  if (!G.bc) log = nullptr;  // the slots and the log belong to level 0
  if (P.fp32) compress_t<float>(st, G, P, B, cur, dtp, fac, log, flog);
  else compress_t<double>(st, G, P, B, cur, dtp, fac, log, flog);
}

template <typename T>
static void viscosity_t(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
                        double fac) {
  ViscArgs<T> A;
  for (int e = 0; e < 3; ++e) {
    A.elo[e] = G.bc ? 0 : -G.g;
    A.ehi[e] = G.bc ? G.n[e] : G.n[e] + G.g - 1;
    if (!G.bc) clip_margin(G, e, false, A.elo[e], A.ehi[e]);
  }
  for (int d = 0; d < 3; ++d)
    for (int e = 0; e < 3; ++e) {
      if (G.bc) {
        A.flo[d][e] = 0;
        A.fhi[d][e] = G.n[e] + (d == e ? 1 : 0);
      } else {
        A.flo[d][e] = -G.g + (d == e ? 1 : 0);
        A.fhi[d][e] = G.n[e] + G.g - 1;
        clip_margin(G, e, d == e, A.flo[d][e], A.fhi[d][e]);
      }
    }
  for (int e = 0; e < 3; ++e) {
    A.lo[e] = min(A.elo[e], min(A.flo[0][e], min(A.flo[1][e], A.flo[2][e])));
    A.hi[e] = max(A.ehi[e], max(A.fhi[0][e], max(A.fhi[1][e], A.fhi[2][e])));
  }
  A.rho = tp<T>(B.q[cur][0]);
  A.e = tp<T>(B.q[cur][1]);
  for (int d = 0; d < 3; ++d) {
    A.v[d] = tp<T>(B.v[d]);
    A.vn[d] = tp<T>(B.q[1 - cur][2 + d]);
  }
  A.dtp = dtp;
  A.fac = fac;
  Box ub;
  for (int e = 0; e < 3; ++e) {
    ub.lo[e] = A.lo[e];
    ub.hi[e] = A.hi[e];
  }
  if (G.bc == 2) DFK_LAUNCH((k_visc<T, 2>), grid_of_flat(ub), dim3(BX, BY), st, G, P, A);
  else if (G.bc) DFK_LAUNCH((k_visc<T, 1>), grid_of_flat(ub), dim3(BX, BY), st, G, P, A);
  else DFK_LAUNCH((k_visc<T, 0>), grid_of_flat(ub), dim3(BX, BY), st, G, P, A);
  for (int d = 0; d < 3; ++d) {
    Box fb;
    for (int e = 0; e < 3; ++e) {
      fb.lo[e] = A.flo[d][e];
      fb.hi[e] = A.fhi[d][e];
    }
    DFK_LAUNCH((k_copy_faces<T>), grid_of_flat(fb), dim3(BX, BY), st, G, fb, tp<T>(B.v[d]), A.vn[d]);
  }
}

void viscosity(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp, double fac) {
  if (!(P.visc > 0.0)) return;
  if (P.fp32) viscosity_t<float>(st, G, P, B, cur, dtp, fac);
  else viscosity_t<double>(st, G, P, B, cur, dtp, fac);
}

template <typename T>
static void diffuse_heat_t(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
                           double fac, bool do_diff, bool do_heat, Scal *clear) {
  DiffArgs<T> A;
  A.clear = G.bc ? clear : nullptr;
  A.b = G.bc ? active_box(G) : clip_cells(G, uniform_box(G, 1, 1));
  A.rho = tp<T>(B.q[cur][0]);
  A.e = tp<T>(B.q[cur][1]);
  A.eo = tp<T>(B.etmp);
  A.hw = B.hw;
  for (int d = 0; d < 3; ++d) {
    A.hw_n[d] = B.hw_n[d];
    A.hw_lo[d] = G.anch[d] ? 0 : G.n[d] / 2 - B.hw_n[d] / 2;
  }
  A.dtp = dtp;
  A.fac = fac;
  A.do_diff = do_diff && P.chi > 0.0;
  A.do_heat = do_heat && P.L != 0.0;
  if (G.bc) {
    A.b.hi[0] = G.n[0] / 2;  // cell pairs: level-0 rows have an even length
    if (record(jk_df<T>(G.bc), DiffJob<T>{G, P, A, grid_of_flat(A.b).x})) return;
    if (G.bc == 2) DFK_LAUNCH((k_diffuse_heat2<T, 2>), grid_of_flat(A.b), dim3(BX, BY), st, G, P, A);
    else DFK_LAUNCH((k_diffuse_heat2<T, 1>), grid_of_flat(A.b), dim3(BX, BY), st, G, P, A);
  } else {
    DFK_LAUNCH(k_diffuse_heat<T>, grid_of_flat(A.b), dim3(BX, BY), st, G, P, A);
  }
}
void diffuse_heat(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, const double *dtp,
                  double fac, bool do_diff, bool do_heat, Scal *clear) {
  if (P.fp32) diffuse_heat_t<float>(st, G, P, B, cur, dtp, fac, do_diff, do_heat, clear);
  else diffuse_heat_t<double>(st, G, P, B, cur, dtp, fac, do_diff, do_heat, clear);
}

template <typename T, int BC, bool FRONT, int W>
static void march_launch(hipStream_t st, int dir, const Geo &G, const Phys &P, const MarchArgs<T> &M, dim3 gr,
                         dim3 bl) {
  if (dir == 1) DFK_LAUNCH((k_march<T, 1, BC, FRONT, W>), gr, bl, st, G, P, M);
  else DFK_LAUNCH((k_march<T, 2, BC, FRONT, W>), gr, bl, st, G, P, M);
}

template <typename T>
static void transport_pass_t(hipStream_t st, int dir, const Geo &G, const Phys &P, LevBufs &B, int src,
                             const double *dtp, double fac, const Geo *Gf, const void *fine_acc, int chunk) {
  PassArgs<T> A;
  if (G.bc) {
    A.b = active_box(G);
  } else {
    // in-bounds ranges that cover every entry the active cells depend on
    for (int d = 0; d < 3; ++d) {
      if (d == dir || (dir != 0 && d < dir)) {
        A.b.lo[d] = -G.g + 2;
        A.b.hi[d] = G.n[d] + G.g - 3;
      } else {
        A.b.lo[d] = -G.g;
        A.b.hi[d] = G.n[d] + G.g - 1;
      }
    }
    A.b = clip_cells(G, A.b);
  }
  for (int m = 0; m < NQ; ++m) {
    A.qi[m] = tp<T>(B.q[src][m]);
    A.qo[m] = tp<T>(B.q[1 - src][m]);
  }
  for (int d = 0; d < 3; ++d) A.v[d] = tp<T>(B.v[d]);
  A.dtp = dtp;
  A.fac = fac;
  A.acc = G.level > 0 ? tp<T>(B.acc) : nullptr;
  A.facc = (G.has_fine && fine_acc) ? reinterpret_cast<const T *>(fine_acc) : nullptr;
  for (int d = 0; d < 3; ++d) A.fn[d] = Gf ? Gf->n[d] : 0;
  if (dir == 0) {
    const dim3 bl(BX, BY);
    const int n = G.n[0];
    if (G.bc == 2) DFK_LAUNCH((k_xpass<T, 2>), grid_of(xtile_box(A.b)), bl, st, G, P, A);
    else if (G.bc && n <= BX) DFK_LAUNCH((k_xrow<T, 1>), grid_of(xrow_box(A.b)), bl, st, G, P, A);
    else if (G.bc && n <= 2 * BX && n % 2 == 0) DFK_LAUNCH((k_xrow<T, 2>), grid_of(xrow_box(A.b)), bl, st, G, P, A);
    else if (G.bc && n <= 4 * BX && n % 4 == 0) DFK_LAUNCH((k_xrow<T, 4>), grid_of(xrow_box(A.b)), bl, st, G, P, A);
    else if (G.bc) DFK_LAUNCH((k_xpass<T, 1>), grid_of(xtile_box(A.b)), bl, st, G, P, A);
    else {
      // finer levels: a row per wave when the cells the update reads, from an
      // aligned start, fit 64 R of them (in FP64 R <= 2: four cells per lane
      // take 138 registers, and the overlapping tiles were faster); else the
      // overlapping tiles
      const int x1 = A.b.hi[0] + 2;
      auto start = [&](int R) { return A.b.lo[0] - 2 - (((A.b.lo[0] - 2) % R) + R) % R; };
      if (x1 - start(1) <= BX) DFK_LAUNCH((k_xrow_fine<T, 1>), grid_of_flat(xrow_box(A.b)), bl, st, G, P, A, start(1));
      else if (x1 - start(2) <= 2 * BX)
        DFK_LAUNCH((k_xrow_fine<T, 2>), grid_of_flat(xrow_box(A.b)), bl, st, G, P, A, start(2));
      else if (sizeof(T) == 4 && x1 - start(4) <= 4 * BX)
        DFK_LAUNCH((k_xrow_fine<T, 4>), grid_of_flat(xrow_box(A.b)), bl, st, G, P, A, start(4));
      else DFK_LAUNCH((k_xpass<T, 0>), grid_of(xtile_box(A.b)), bl, st, G, P, A);
    }
    return;
  }
  MarchArgs<T> M;
  for (int d = 0; d < 3; ++d) {
    M.lo[d] = A.b.lo[d];
    M.hi[d] = A.b.hi[d];
    M.fn[d] = A.fn[d];
  }
  const int ext = M.hi[dir] - M.lo[dir];
  if (ext <= 0) return;
  M.chunk = ext <= chunk ? ext : chunk;
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
  const long ntb = (M.hi[td] - M.lo[td] + 1) / 2;
  const long nch = (ext + M.chunk - 1) / M.chunk;
  const long ncol = (long)(M.hi[0] - M.lo[0]) * (M.hi[td] - M.lo[td]);
  const bool front = M.acc || M.facc;
  // level 0 without frontier transfers: two adjacent columns per lane (its
  // rows start 128-byte aligned and the x extent is even) in FP32, and in FP64
  // for the z pass (its 16-byte accesses halve the address and load work per
  // byte; the FP64 y pass is fused with the x pass or keeps one column)
  const int w = ((sizeof(T) == 4 || dir == 2) && G.bc && !front && (M.hi[0] - M.lo[0]) % 2 == 0 &&
                 M.lo[0] % 2 == 0)
                    ? 2
                    : 1;
  const long nbx = (M.hi[0] - M.lo[0] + 64 * w - 1) / (64 * w);
  // one column per lane: blocks of 128 consecutive columns (k_march)
  const dim3 gr((unsigned)(w == 1 ? (ncol + 127) / 128 * nch : nbx * ntb * nch)), bl(64, 4);
  if (!G.bc) {
    march_launch<T, 0, true, 1>(st, dir, G, P, M, gr, bl);  // finer levels always carry frontier transfers
  } else if (G.bc == 2) {
    if (front) march_launch<T, 2, true, 1>(st, dir, G, P, M, gr, bl);
    else if (w == 2) march_launch<T, 2, false, 2>(st, dir, G, P, M, gr, bl);
    else march_launch<T, 2, false, 1>(st, dir, G, P, M, gr, bl);
  } else {
    if (front) march_launch<T, 1, true, 1>(st, dir, G, P, M, gr, bl);
    else if (w == 2) march_launch<T, 1, false, 2>(st, dir, G, P, M, gr, bl);
    else march_launch<T, 1, false, 1>(st, dir, G, P, M, gr, bl);
  }
}
bool transport_xy_fits(const Geo &G) {
  const int n = G.n[0];
  return G.bc == 1 && n <= 2 * BX && (n <= BX || n % 2 == 0);
}

template <typename T>
static bool transport_xy_t(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src, const double *dtp,
                           double fac, int chunk, const Geo *Gf, const void *fine_acc) {
  const int n = G.n[0];
  if (!transport_xy_fits(G)) return false;
  PassArgs<T> A;
  A.b = active_box(G);
  for (int m = 0; m < NQ; ++m) {
    A.qi[m] = tp<T>(B.q[src][m]);
    A.qo[m] = tp<T>(B.q[1 - src][m]);
  }
  for (int d = 0; d < 3; ++d) A.v[d] = tp<T>(B.v[d]);
  A.dtp = dtp;
  A.fac = fac;
  // under a finer level: flux matching on its frontier (level 0 accumulates
  // nothing)
  A.acc = nullptr;
  A.facc = (G.has_fine && fine_acc) ? reinterpret_cast<const T *>(fine_acc) : nullptr;
  for (int d = 0; d < 3; ++d) A.fn[d] = A.facc ? Gf->n[d] : 0;
  MarchArgs<T> M;
  for (int d = 0; d < 3; ++d) {
    M.lo[d] = A.b.lo[d];
    M.hi[d] = A.b.hi[d];
    M.fn[d] = A.fn[d];
  }
  M.chunk = G.n[1] <= chunk ? G.n[1] : chunk;
  for (int m = 0; m < NQ; ++m) {
    M.qi[m] = A.qo[m];
    M.qo[m] = A.qo[m];
  }
  M.v = A.v[1];
  M.dtp = dtp;
  M.fac = fac;
  M.acc = nullptr;
  M.facc = A.facc;
  // one block of four waves per (plane, y segment)
  const long nch = (G.n[1] + M.chunk - 1) / M.chunk;
  const dim3 gr((unsigned)(G.n[2] * nch)), bl(64, 4);
  if (A.facc) {
    if (n == BX) DFK_LAUNCH((k_xyshared<T, 1, true, true>), gr, bl, st, G, P, A, M);
    else if (n < BX) DFK_LAUNCH((k_xyshared<T, 1, false, true>), gr, bl, st, G, P, A, M);
    else if (n == 2 * BX) DFK_LAUNCH((k_xyshared<T, 2, true, true>), gr, bl, st, G, P, A, M);
    else DFK_LAUNCH((k_xyshared<T, 2, false, true>), gr, bl, st, G, P, A, M);
    return true;
  }
  if (record(jk_xy<T>(n), XyJob<T>{G, P, A, M, gr.x})) return true;
  if (n == BX) DFK_LAUNCH((k_xyshared<T, 1, true>), gr, bl, st, G, P, A, M);
  else if (n < BX) DFK_LAUNCH((k_xyshared<T, 1, false>), gr, bl, st, G, P, A, M);
  else if (n == 2 * BX) DFK_LAUNCH((k_xyshared<T, 2, true>), gr, bl, st, G, P, A, M);
  else DFK_LAUNCH((k_xyshared<T, 2, false>), gr, bl, st, G, P, A, M);
  return true;
}
bool transport_xy(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src, const double *dtp, double fac,
                  int chunk, const Geo *Gf, const void *fine_acc) {
  if (P.fp32) return transport_xy_t<float>(st, G, P, B, src, dtp, fac, chunk, Gf, fine_acc);
  return transport_xy_t<double>(st, G, P, B, src, dtp, fac, chunk, Gf, fine_acc);
}

template <typename T>
static void transport_xy_fine_t(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src,
                                const double *dtp, double fac, const Geo *Gf, const void *fine_acc, int chunk) {
  PassArgs<T> A;
  // the y pass's box (x, y two cells inside the stored box, z all of it),
  // within G's margins
  for (int d = 0; d < 3; ++d) {
    A.b.lo[d] = d < 2 ? -G.g + 2 : -G.g;
    A.b.hi[d] = d < 2 ? G.n[d] + G.g - 3 : G.n[d] + G.g - 1;
  }
  A.b = clip_cells(G, A.b);
  for (int m = 0; m < NQ; ++m) {
    A.qi[m] = tp<T>(B.q[src][m]);
    A.qo[m] = tp<T>(B.q[1 - src][m]);
  }
  for (int d = 0; d < 3; ++d) A.v[d] = tp<T>(B.v[d]);
  A.dtp = dtp;
  A.fac = fac;
  A.acc = tp<T>(B.acc);
  A.facc = (G.has_fine && fine_acc) ? reinterpret_cast<const T *>(fine_acc) : nullptr;
  for (int d = 0; d < 3; ++d) A.fn[d] = Gf ? Gf->n[d] : 0;
  MarchArgs<T> M;
  for (int d = 0; d < 3; ++d) {
    M.lo[d] = A.b.lo[d];
    M.hi[d] = A.b.hi[d];
    M.fn[d] = A.fn[d];
  }
  const int ext = M.hi[1] - M.lo[1];
  if (ext <= 0 || M.hi[0] <= M.lo[0] || M.hi[2] <= M.lo[2]) return;
  // each segment x-updates two rows past either end of its own: at least 16
  // rows per segment (on 4 levels of 128^3, 16 ran 2 % faster than 32 and 8
  // suits the other walks)
  chunk = chunk < 16 ? 16 : chunk;
  M.chunk = ext <= chunk ? ext : chunk;
  for (int m = 0; m < NQ; ++m) {
    M.qi[m] = A.qi[m];
    M.qo[m] = A.qo[m];
  }
  M.v = A.v[1];
  M.dtp = dtp;
  M.fac = fac;
  M.acc = A.acc;
  M.facc = A.facc;
  // whole tiles, then (FP64) the row's last cells in half-wave tiles of two planes
  const int ex = M.hi[0] - M.lo[0], np = M.hi[2] - M.lo[2];
  int ntiles = ex / XF_TILE, tail = ex - ntiles * XF_TILE;
  if (tail > XF_HALF || sizeof(T) == 4) {
    ++ntiles;
    tail = 0;
  }
  const int nseg = (ext + M.chunk - 1) / M.chunk;
  const long nblk = (long)ntiles * nseg * np + (tail ? (long)nseg * ((np + 1) / 2) : 0);
  const dim3 gr((unsigned)nblk), bl(64, 2);
  // FP64: four quantity groups (127 registers, four waves per SIMD; the
  // density is walked four times), 2.5 % faster on 4 levels of 128^3 than
  // two groups at 168 registers; FP32: two groups (1 % faster than four)
  if constexpr (sizeof(T) == 8) DFK_LAUNCH((k_xyfine<T, 4>), gr, dim3(64, 4), st, G, P, A, M, ntiles, nseg, tail);
  else DFK_LAUNCH((k_xyfine<T, 2>), gr, bl, st, G, P, A, M, ntiles, nseg, tail);
}
void transport_xy_fine(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int src, const double *dtp,
                       double fac, const Geo *Gf, const void *fine_acc, int chunk) {
  if (P.fp32) transport_xy_fine_t<float>(st, G, P, B, src, dtp, fac, Gf, fine_acc, chunk);
  else transport_xy_fine_t<double>(st, G, P, B, src, dtp, fac, Gf, fine_acc, chunk);
}

bool transport_z_finish_fits(const Geo &G) {
  return G.bc == 1 && !G.has_fine && G.n[0] <= 2 * BX && G.n[0] % 2 == 0 && G.n[1] % ZF_TY == 0;
}

template <typename T>
static bool transport_z_finish_t(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, void *const *vin, int src,
                                 const double *dtp, double fac, double kfac, Scal *S, int chunk) {
  // the walk reads the z-face velocities the finish rewrites: they must be
  // another set (the first kick's, when it was fused with the compression)
  if (!transport_z_finish_fits(G) || !S || vin[2] == B.v[2]) return false;
  MarchArgs<T> M{};
  const Box b = active_box(G);
  for (int d = 0; d < 3; ++d) {
    M.lo[d] = b.lo[d];
    M.hi[d] = b.hi[d];
    M.fn[d] = 0;
  }
  M.chunk = G.n[2] <= chunk ? G.n[2] : chunk;
  for (int m = 0; m < NQ; ++m) {
    M.qi[m] = tp<T>(B.q[src][m]);
    M.qo[m] = tp<T>(B.q[1 - src][m]);
  }
  M.v = tp<T>(vin[2]);
  M.dtp = dtp;
  M.fac = fac;
  M.acc = nullptr;
  M.facc = nullptr;
  KickArgs<T> K{};
  for (int d = 0; d < 3; ++d) {
    K.v[d] = tp<T>(B.v[d]);
    K.vin[d] = K.v[d];
  }
  K.dtp = dtp;
  K.fac = kfac;
  const RedArgs<T> R = red_args<T>(G, B, 1 - src, S);
  const long nch = (G.n[2] + M.chunk - 1) / M.chunk;
  const long nblk = (long)(G.n[1] / ZF_TY) * nch;
  if (nblk > R.npart) return false;  // every block needs a partial slot (never the case for a fitting mesh)
  if (record(jk_zf<T>(), ZfJob<T>{G, P, M, K, R, (unsigned)nblk})) return true;
  DFK_LAUNCH(k_zfinish<T>, dim3((unsigned)nblk), dim3(64, ZF_WAVES), st, G, P, M, K, R);
  return true;
}
bool transport_z_finish(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, void *const *vin, int src,
                        const double *dtp, double fac, double kfac, Scal *S, int chunk) {
  if (P.fp32) return transport_z_finish_t<float>(st, G, P, B, vin, src, dtp, fac, kfac, S, chunk);
  return transport_z_finish_t<double>(st, G, P, B, vin, src, dtp, fac, kfac, S, chunk);
}

void transport_pass(hipStream_t st, int dir, const Geo &G, const Phys &P, LevBufs &B, int src, const double *dtp,
                    double fac, const Geo *Gf, const void *fine_acc, int chunk) {
  if (P.fp32) transport_pass_t<float>(st, dir, G, P, B, src, dtp, fac, Gf, fine_acc, chunk);
  else transport_pass_t<double>(st, dir, G, P, B, src, dtp, fac, Gf, fine_acc, chunk);
}

// each thread moves four 16-byte words (loads first), block b the words
// [1024 b, 1024 b + 1024)
__global__ void __launch_bounds__(256) k_copy16(uint4 *dst, const uint4 *src, size_t n) {
  const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x;
  uint4 w[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (base + 256 * u < n) w[u] = src[base + 256 * u];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (base + 256 * u < n) dst[base + 256 * u] = w[u];
}

void log_pending(hipStream_t st, const Geo &G, LevBufs &B, Scal *S, double *flog) {
  const LogJob J{(const double *)B.part, (int)part_count(G), S, flog, 1u};
  if (record(JK_LOG, J)) return;
  DFK_LAUNCH(k_log_pending, dim3(1), dim3(FT), st, J.part, J.npart, S, flog);
}

void set_recorder(Recorder *r) { g_rec = r; }

size_t job_entry_size(int kind) {
  switch (kind) {
    case JK_KC_D1: case JK_KC_D2: return sizeof(KcJob<double>);
    case JK_KC_F1: case JK_KC_F2: return sizeof(KcJob<float>);
    case JK_DF_D1: case JK_DF_D2: return sizeof(DiffJob<double>);
    case JK_DF_F1: case JK_DF_F2: return sizeof(DiffJob<float>);
    case JK_XY_D1P: case JK_XY_D1F: case JK_XY_D2P: case JK_XY_D2F: return sizeof(XyJob<double>);
    case JK_XY_F1P: case JK_XY_F1F: case JK_XY_F2P: case JK_XY_F2F: return sizeof(XyJob<float>);
    case JK_ZF_D: return sizeof(ZfJob<double>);
    case JK_ZF_F: return sizeof(ZfJob<float>);
    case JK_LOG: return sizeof(LogJob);
    default: return 0;
  }
}

template <typename E>
static JobTab<E> tab_of(const void *entries, const unsigned *start, int n) {
  return JobTab<E>{reinterpret_cast<const E *>(entries), start, n};
}

void launch_jobs(hipStream_t st, int kind, const void *entries, const unsigned *start, int n, unsigned nblocks) {
  const dim3 gr(nblocks), bl(BX, BY), xb(64, 4), zb(64, ZF_WAVES);
  switch (kind) {
    case JK_KC_D1: DFK_LAUNCH((k_kick_compress_jobs<double, 1>), gr, bl, st, tab_of<KcJob<double>>(entries, start, n)); break;
    case JK_KC_D2: DFK_LAUNCH((k_kick_compress_jobs<double, 2>), gr, bl, st, tab_of<KcJob<double>>(entries, start, n)); break;
    case JK_KC_F1: DFK_LAUNCH((k_kick_compress_jobs<float, 1>), gr, bl, st, tab_of<KcJob<float>>(entries, start, n)); break;
    case JK_KC_F2: DFK_LAUNCH((k_kick_compress_jobs<float, 2>), gr, bl, st, tab_of<KcJob<float>>(entries, start, n)); break;
    case JK_DF_D1: DFK_LAUNCH((k_diffuse_heat2_jobs<double, 1>), gr, bl, st, tab_of<DiffJob<double>>(entries, start, n)); break;
    case JK_DF_D2: DFK_LAUNCH((k_diffuse_heat2_jobs<double, 2>), gr, bl, st, tab_of<DiffJob<double>>(entries, start, n)); break;
    case JK_DF_F1: DFK_LAUNCH((k_diffuse_heat2_jobs<float, 1>), gr, bl, st, tab_of<DiffJob<float>>(entries, start, n)); break;
    case JK_DF_F2: DFK_LAUNCH((k_diffuse_heat2_jobs<float, 2>), gr, bl, st, tab_of<DiffJob<float>>(entries, start, n)); break;
    case JK_XY_D1P: DFK_LAUNCH((k_xyshared_jobs<double, 1, false>), gr, xb, st, tab_of<XyJob<double>>(entries, start, n)); break;
    case JK_XY_D1F: DFK_LAUNCH((k_xyshared_jobs<double, 1, true>), gr, xb, st, tab_of<XyJob<double>>(entries, start, n)); break;
    case JK_XY_D2P: DFK_LAUNCH((k_xyshared_jobs<double, 2, false>), gr, xb, st, tab_of<XyJob<double>>(entries, start, n)); break;
    case JK_XY_D2F: DFK_LAUNCH((k_xyshared_jobs<double, 2, true>), gr, xb, st, tab_of<XyJob<double>>(entries, start, n)); break;
    case JK_XY_F1P: DFK_LAUNCH((k_xyshared_jobs<float, 1, false>), gr, xb, st, tab_of<XyJob<float>>(entries, start, n)); break;
    case JK_XY_F1F: DFK_LAUNCH((k_xyshared_jobs<float, 1, true>), gr, xb, st, tab_of<XyJob<float>>(entries, start, n)); break;
    case JK_XY_F2P: DFK_LAUNCH((k_xyshared_jobs<float, 2, false>), gr, xb, st, tab_of<XyJob<float>>(entries, start, n)); break;
    case JK_XY_F2F: DFK_LAUNCH((k_xyshared_jobs<float, 2, true>), gr, xb, st, tab_of<XyJob<float>>(entries, start, n)); break;
    case JK_ZF_D: DFK_LAUNCH(k_zfinish_jobs<double>, gr, zb, st, tab_of<ZfJob<double>>(entries, start, n)); break;
    case JK_ZF_F: DFK_LAUNCH(k_zfinish_jobs<float>, gr, zb, st, tab_of<ZfJob<float>>(entries, start, n)); break;
    case JK_LOG: DFK_LAUNCH(k_log_pending_jobs, gr, dim3(FT), st, tab_of<LogJob>(entries, start, n)); break;
    default: break;
  }
}

void stream_copy(hipStream_t st, void *dst, const void *src, size_t n16) {
  if (n16 == 0) return;
  const size_t blocks = (n16 + 1023) / 1024;
  DFK_LAUNCH(k_copy16, dim3((unsigned)blocks), dim3(256), st, reinterpret_cast<uint4 *>(dst),
                     reinterpret_cast<const uint4 *>(src), n16);
}

void zero(hipStream_t st, void *p, size_t bytes) {
  const size_t n = bytes / 4;
  if (n == 0 || !p) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  DFK_LAUNCH(k_zero, dim3((unsigned)blocks), dim3(256), st, reinterpret_cast<unsigned int *>(p), n);
}

// floor(i / 2)
static int fdiv2_host(int i) { return (i >= 0) ? i / 2 : -((1 - i) / 2); }

template <typename T>
static void commup_t(hipStream_t st, const Geo &Gc, LevBufs &Bc, int curc, const Geo &Gf, LevBufs &Bf, int curf) {
  UpArgs<T> A;
  for (int f = 0; f < NSTATE; ++f) {
    A.Q[f] = tp<T>(f == 0 ? Bc.q[curc][0] : (f == 1 ? Bc.q[curc][1] : Bc.v[f - 2]));
    A.out[f] = tp<T>(f == 0 ? Bf.q[curf][0] : (f == 1 ? Bf.q[curf][1] : Bf.v[f - 2]));
  }
  // hosts of the stored fine entries [-g, n+g) along each axis (from the
  // mirror plane along an anchored one: the entries beyond it are the fine
  // level's own images, set after the fill)
  for (int d = 0; d < 3; ++d) {
    A.b.lo[d] = Gf.anch[d] ? 0 : fdiv2_host(-Gf.g);
    A.b.hi[d] = fdiv2_host(Gf.s[d] - Gf.g - 1) + 1;
  }
  // the inner hosts, relative to b.lo (every fine child an active cell)
  unsigned ext[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = (unsigned)(A.b.hi[d] - A.b.lo[d]);
    const int lo = std::max(0, -A.b.lo[d]), hi = std::min((int)ext[d], Gf.n[d] / 2 - A.b.lo[d]);
    A.in_lo[d] = lo;
    A.in_n[d] = std::max(0, hi - lo);
  }
  if (A.in_n[0] == 0 || A.in_n[1] == 0 || A.in_n[2] == 0) A.in_n[0] = A.in_n[1] = A.in_n[2] = 0;
  A.c1 = (ext[2] - A.in_n[2]) * ext[0] * ext[1];
  A.c2 = A.c1 + A.in_n[2] * (ext[1] - A.in_n[1]) * ext[0];
  A.nshell = A.c2 + A.in_n[2] * A.in_n[1] * (ext[0] - A.in_n[0]);
  A.nb = (A.nshell + BX * BY - 1) / (BX * BY);
  const dim3 gr(A.nb * NSTATE);
  if (Gc.bc == 2) DFK_LAUNCH((k_commup<T, 2>), gr, dim3(BX, BY), st, Gc, Gf, A);
  else if (Gc.bc) DFK_LAUNCH((k_commup<T, 1>), gr, dim3(BX, BY), st, Gc, Gf, A);
  else DFK_LAUNCH((k_commup<T, 0>), gr, dim3(BX, BY), st, Gc, Gf, A);
}
void commup(hipStream_t st, const Geo &Gc, const Phys &P, LevBufs &Bc, int curc, const Geo &Gf, LevBufs &Bf,
            int curf) {
  if (P.fp32) commup_t<float>(st, Gc, Bc, curc, Gf, Bf, curf);
  else commup_t<double>(st, Gc, Bc, curc, Gf, Bf, curf);
}

template <typename T>
static void mirror_state_t(hipStream_t st, const Geo &G, LevBufs &B, int cur) {
  for (int d = 1; d < 3; ++d) {
    if (!G.anch[d]) continue;
    MirArgs<T> A{};
    A.nf = 5;
    for (int f = 0; f < 5; ++f) {
      T *a = tp<T>(f < 2 ? B.q[cur][f] : B.v[f - 2]);
      A.dst[f] = a;
      A.src[f] = a;
      A.sgn[f] = (f == 2 + d) ? T(-1) : T(1);  // the velocity normal to the plane is odd
      A.face[f] = 0;
    }
    A.face[2 + d] = 1;
    A.d = d;
    for (int e = 0; e < 3; ++e) {
      A.b.lo[e] = -G.g;
      A.b.hi[e] = e == d ? 0 : G.s[e] - G.g;
    }
    DFK_LAUNCH(k_mirror<T>, grid_of_flat(A.b), dim3(BX, BY), st, G, A);
  }
}

template <typename T>
static void mirror_q_t(hipStream_t st, const Geo &G, LevBufs &B, int set) {
  for (int d = 1; d < 3; ++d) {
    if (!G.anch[d]) continue;
    MirArgs<T> A{};
    A.nf = NQ;
    for (int m = 0; m < NQ; ++m) {
      // the momenta normal to the plane swap and change sign: P-_d of an
      // image is -P+_d of its cell
      const int pair = (m == 2 + 2 * d) ? m + 1 : ((m == 3 + 2 * d) ? m - 1 : m);
      A.dst[m] = tp<T>(B.q[set][m]);
      A.src[m] = tp<T>(B.q[set][pair]);
      A.sgn[m] = pair != m ? T(-1) : T(1);
      A.face[m] = 0;
    }
    A.d = d;
    for (int e = 0; e < 3; ++e) {
      A.b.lo[e] = -G.g;
      A.b.hi[e] = e == d ? 0 : G.s[e] - G.g;
    }
    DFK_LAUNCH(k_mirror<T>, grid_of_flat(A.b), dim3(BX, BY), st, G, A);
  }
}

void mirror_state(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur) {
  if (G.bc || !(G.anch[1] || G.anch[2])) return;
  if (P.fp32) mirror_state_t<float>(st, G, B, cur);
  else mirror_state_t<double>(st, G, B, cur);
}

void mirror_q(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int set) {
  if (G.bc || !(G.anch[1] || G.anch[2])) return;
  if (P.fp32) mirror_q_t<float>(st, G, B, set);
  else mirror_q_t<double>(st, G, B, set);
}

template <typename T>
static void commmean_t(hipStream_t st, const Geo &Gf, LevBufs &Bf, int curf, const Geo &Gc, LevBufs &Bc,
                       int curc) {
  MeanArgs<T> A;
  A.start[0] = 0;
  for (int f = 0; f < NSTATE; ++f) {
    const int stag = f >= 2 ? f - 2 : -1;
    A.Q[f] = tp<T>(f == 0 ? Bf.q[curf][0] : (f == 1 ? Bf.q[curf][1] : Bf.v[f - 2]));
    A.out[f] = tp<T>(f == 0 ? Bc.q[curc][0] : (f == 1 ? Bc.q[curc][1] : Bc.v[f - 2]));
    Box b;
    for (int d = 0; d < 3; ++d) {
      A.b.lo[d] = b.lo[d] = 0;
      A.b.hi[d] = Gc.cn[d];
      b.hi[d] = Gc.cn[d] + (d == stag ? 1 : 0);
    }
    A.start[f + 1] = A.start[f] + grid_of_flat(b).x;
  }
  DFK_LAUNCH(k_commmean<T>, dim3(A.start[NSTATE]), dim3(BX, BY), st, Gf, Gc, A);
}
void commmean(hipStream_t st, const Geo &Gf, const Phys &P, LevBufs &Bf, int curf, const Geo &Gc, LevBufs &Bc,
              int curc) {
  if (P.fp32) commmean_t<float>(st, Gf, Bf, curf, Gc, Bc, curc);
  else commmean_t<double>(st, Gf, Bf, curf, Gc, Bc, curc);
}

size_t part_count(const Geo &G) {
  const Box b = active_box(G);
  return (size_t)grid_of(b).x;
}

template <typename T>
static RedArgs<T> red_args(const Geo &G, LevBufs &B, int cur, Scal *S) {
  RedArgs<T> A;
  A.b = active_box(G);
  A.rho = tp<T>(B.q[cur][0]);
  A.e = tp<T>(B.q[cur][1]);
  for (int d = 0; d < 3; ++d) A.v[d] = tp<T>(B.v[d]);
  A.part = B.part;
  A.npart = (int)part_count(G);
  A.spart = B.part + 3 * (size_t)A.npart;
  A.S = S;
  for (int d = 0; d < 3; ++d) {
    A.cov_lo[d] = G.has_fine ? G.co[d] : 0;
    A.cov_hi[d] = G.has_fine ? G.co[d] + G.cn[d] : 0;
  }
  return A;
}

void signal_speed(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, Scal *S) {
  if (P.fp32) {
    RedArgs<float> A = red_args<float>(G, B, cur, S);
    DFK_LAUNCH(k_signal<float>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  } else {
    RedArgs<double> A = red_args<double>(G, B, cur, S);
    DFK_LAUNCH(k_signal<double>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  }
}

static DtArgs dt_args(const Geo *G, const LevBufs *B, int nl, int advance) {
  DtArgs A;
  for (int l = 0; l < MAXLEV; ++l) {
    A.dx[l] = l < nl ? G[l].dx : 0.0;
    A.part[l] = l < nl ? B[l].part + 3 * part_count(G[l]) : nullptr;
    A.npart[l] = l < nl ? (int)part_count(G[l]) : 0;
  }
  A.nl = nl;
  A.advance = advance;
  return A;
}

void dt_final(hipStream_t st, const Geo *G, const LevBufs *B, int nl, const Phys &P, Scal *S, int advance) {
  DFK_LAUNCH(k_dt_final, dim3(1), dim3(FT), st, P, dt_args(G, B, nl, advance), S);
}

void post_partials(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur, Scal *S) {
  if (P.fp32) {
    RedArgs<float> A = red_args<float>(G, B, cur, S);
    DFK_LAUNCH(k_post<float>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  } else {
    RedArgs<double> A = red_args<double>(G, B, cur, S);
    DFK_LAUNCH(k_post<double>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  }
}

static FinalArgs final_args(double *const *parts, const int *nparts, int nl, Scal *S, int slot, double *flog) {
  FinalArgs A;
  for (int l = 0; l < MAXLEV; ++l) {
    A.part[l] = l < nl ? parts[l] : nullptr;
    A.npart[l] = l < nl ? nparts[l] : 0;
  }
  A.nl = nl;
  A.out = slot == 1 ? S->totals : S->force;
  A.S = S;
  A.flog = slot == 2 ? flog : nullptr;
  return A;
}

void step_final(hipStream_t st, const Geo *G, LevBufs *B, int nl, const Phys &P, Scal *S, double *flog,
                int do_force, int do_dt) {
  double *parts[MAXLEV];
  int np[MAXLEV];
  for (int l = 0; l < nl; ++l) {
    parts[l] = B[l].part;
    np[l] = (int)part_count(G[l]);
  }
  const FinalArgs F = final_args(parts, np, nl, S, 2, flog);
  const DtArgs D = dt_args(G, B, nl, do_dt == 2 ? 2 : 1);
  if (do_force && do_dt) DFK_LAUNCH((k_step_final<true, true>), dim3(1), dim3(FT), st, P, F, D, S);
  else if (do_force) DFK_LAUNCH((k_step_final<true, false>), dim3(1), dim3(FT), st, P, F, D, S);
  else if (do_dt) DFK_LAUNCH((k_step_final<false, true>), dim3(1), dim3(FT), st, P, F, D, S);
}

int force_partials(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur) {
  if (P.fp32) {
    RedArgs<float> A = red_args<float>(G, B, cur, nullptr);
    DFK_LAUNCH(k_force<float>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  } else {
    RedArgs<double> A = red_args<double>(G, B, cur, nullptr);
    DFK_LAUNCH(k_force<double>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  }
  return (int)part_count(G);
}

int totals_partials(hipStream_t st, const Geo &G, const Phys &P, LevBufs &B, int cur) {
  if (P.fp32) {
    RedArgs<float> A = red_args<float>(G, B, cur, nullptr);
    DFK_LAUNCH(k_totals<float>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  } else {
    RedArgs<double> A = red_args<double>(G, B, cur, nullptr);
    DFK_LAUNCH(k_totals<double>, grid_of(A.b), dim3(BX, BY), st, G, P, A);
  }
  return (int)part_count(G);
}

void force_final(hipStream_t st, double *const *parts, const int *nparts, int nl, Scal *S, int slot,
                 double *flog) {
  DFK_LAUNCH(k_final3, dim3(1), dim3(FT), st, final_args(parts, nparts, nl, S, slot, flog));
}

}  // namespace dfk
