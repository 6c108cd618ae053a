// gks.hip -- kernels and C-ABI host library of the compact third-order
// gas-kinetic scheme (Pan & Xu, arXiv:1412.4489) for MI355X (gfx950).
//
// A handle holds any number of independent grids ("problems").  Problems of
// the same dimension and precision form a group; one time step of a group is
// a fixed sequence of launches, each covering every problem of the group
// (a block-owner table maps each block to its problem and tile):
//   2D: k_ghost_2d               boundary images (cells: two layers incl.
//                                corners; interface values of edge ghosts)
//                                and, in one thread per problem, the CFL
//                                time step or the fixed step
//       k_recon_2d               compact reconstruction (Sec. 3.2)
//       k_iface_2d               every interface: prologue (U0, equilibrium
//                                quadratic, tau, time integrals, leading terms;
//                                double), eq. dis1 (g0), eq. dis2 of side 0
//                                (g_l on u > 0) and side 1 (g_r on u < 0), in
//                                sections passing the frame record through LDS
//       k_update_2d              domain-edge walls (no-slip impermeable, slip a
//                                symmetry line), conservative update (eq.
//                                finite), nonphysical flag, CFL bound of the
//                                new state
//   1D: k_ghost_1d (+ time step), k_recon_1d, k_face_1d (fused interface), k_update_1d
// The step of all groups is captured once in a hipGraph and replayed.
//
// Memory per 2D problem (structure of arrays, x fastest):
//   W   double [4][ny+4][nx+4]      cell averages with two ghost layers
//   FX  TS     [2][4][ny+2][nx+3]   x-interface Gauss values, interfaces -1..nx+1, rows -1..ny
//   FY  TS     [2][4][ny+3][nx+2]   y-interface Gauss values, interfaces -1..ny+1, cols -1..nx
//   PC  TP     [4][5][ny+2][nx+2]   reconstruction coefficients, cells -1..nx
//   FLX double [4][ny][nx+1], FLY double [4][ny+1][nx]   integrated fluxes
// per 1D problem: W double [3][nx+4], FX TS [3][nx+3] (interfaces -1..nx+1),
//   PC TP [3][2][nx+2], FLX double [3][nx+1].
// TS = TP = TC = double (GKS_FP64) or float (GKS_FP32_MIXED).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "gks.h"
#include "gks_device.h"

using namespace gks;

namespace {

// ---------------------------------------------------------------------------
// indexing
// ---------------------------------------------------------------------------
struct Idx {
  int nx, ny;
  // computed interfaces: fxr x interfaces per row, fyr rows of y interfaces.
  // On a periodic axis the last interface is the first one and is not
  // computed again (fxr = nx, fyr = ny; else nx + 1, ny + 1).
  int fxr, fyr;
  // Every index is (plane number) x (plane size) + (offset in the plane): the
  // plane part is uniform over a wave, the in-plane part is one 32-bit
  // multiply-add per lane shared by all planes (a plane holds fewer than 2^32
  // entries: the grid size is bounded at initialisation).
  __device__ __host__ unsigned off(int row, int col, int pitch) const {
    return (unsigned)row * (unsigned)pitch + (unsigned)col;
  }
  __device__ __host__ size_t w(int v, int j, int i) const {
    return (size_t)v * ((size_t)(ny + 4) * (nx + 4)) + off(j + 2, i + 2, nx + 4);
  }
  __device__ __host__ size_t fx(int g, int v, int j, int fi) const {
    return (size_t)(g * 4 + v) * ((size_t)(ny + 2) * (nx + 3)) + off(j + 1, fi + 1, nx + 3);
  }
  __device__ __host__ size_t fy(int g, int v, int fj, int i) const {
    return (size_t)(g * 4 + v) * ((size_t)(ny + 3) * (nx + 2)) + off(fj + 1, i + 1, nx + 2);
  }
  __device__ __host__ size_t pc(int v, int m, int j, int i) const {
    return (size_t)(v * 5 + m) * ((size_t)(ny + 2) * (nx + 2)) + off(j + 1, i + 1, nx + 2);
  }
  __device__ __host__ size_t flx(int v, int j, int fi) const {
    return (size_t)v * ((size_t)ny * (nx + 1)) + off(j, fi, nx + 1);
  }
  __device__ __host__ size_t fly(int v, int fj, int i) const {
    return (size_t)v * ((size_t)(ny + 1) * nx) + off(fj, i, nx);
  }
  // the same x / y interface indices in nested form, for the final
  // read-modify-write of the correction phases: there the address is formed
  // late, which keeps it out of the phases' register peak
  __device__ __host__ size_t fx_late(int g, int v, int j, int fi) const {
    return (((size_t)g * 4 + v) * (ny + 2) + (size_t)(j + 1)) * (nx + 3) + (size_t)(fi + 1);
  }
  __device__ __host__ size_t fy_late(int g, int v, int fj, int i) const {
    return (((size_t)g * 4 + v) * (ny + 3) + (size_t)(fj + 1)) * (nx + 2) + (size_t)(i + 1);
  }
  __device__ __host__ size_t flx_late(int v, int j, int fi) const { return ((size_t)v * ny + j) * (nx + 1) + fi; }
  __device__ __host__ size_t fly_late(int v, int fj, int i) const { return ((size_t)v * (ny + 1) + fj) * nx + i; }
  // 1D layouts (ny = 1)
  __device__ __host__ size_t w1(int v, int i) const { return (size_t)v * (nx + 4) + (size_t)(i + 2); }
  __device__ __host__ size_t f1(int v, int fi) const { return (size_t)v * (nx + 3) + (size_t)(fi + 1); }
  __device__ __host__ size_t pc1(int v, int m, int i) const { return ((size_t)v * 2 + m) * (nx + 2) + (size_t)(i + 1); }
  __device__ __host__ size_t fl1(int v, int fi) const { return (size_t)v * (nx + 1) + fi; }
};

struct BCDev {
  int kind;
  double state[4];  // conservative
  double alt[4];    // conservative
  double wu, wv, wT;
  double wo;        // curvilinear grids: angular velocity of a turning no-slip wall
};

struct Geo {
  double x0, y0, h, k;  // curvilinear grids: h = k = 1 (logical coordinates)
};

// Geometry of a curvilinear grid (all null for the uniform grid):
//   fx   x interfaces (logical direction i), 7 planes of [ny][nx+1]: unit
//        normal (2), unit tangent (2), length L, metric G_nn, G_ns
//        (d/dn = G_nn d/dxi + G_ns d/deta, d/dt = d/deta / L)
//   fy   y interfaces, 7 planes of [ny+1][nx], the same with xi <-> eta
//   area cell areas [ny+2][nx+2] over cells -1..nx x -1..ny (an edge ghost
//        cell has its image's)
//   wid  2 planes of [ny][nx]: widths across the i and the j direction
//   bnd  boundary vertices (x, y): west [ny+1], east [ny+1], south [nx+1], north [nx+1]
struct CurvDev {
  const double* fx;
  const double* fy;
  const double* area;
  const double* wid;
  const double* bnd;
};
constexpr int kFaceGeo = 7;

template <typename TS, typename TP>
struct Grid {
  Idx ix;
  Geo geo;
  CurvDev cv;
  double* W;
  TS* FX;
  TS* FY;
  TP* PC;
  double* FLX;
  double* FLY;
  double* t;                  // time
  double* dt;                 // step of the current step
  long long* steps;
  unsigned long long* err;    // 0, or the location of the first nonphysical state (see gks_fetch)
  unsigned long long* nfall;  // interior cells whose reconstruction fell back to the average (summed over steps)
  unsigned long long* dtmin;  // dtmask + 1 running minima of the CFL bound (bits of positive doubles)
  unsigned dtmask;            // slots of the problem - 1 (a power of two minus one)
};

// The CFL bound is reduced into slots per problem (one atomic per wave of
// cells, into slot (wave within the problem) & dtmask), which keeps the atomics
// on one address few.  A problem has one slot per wave of its cells, rounded
// up to a power of two within [64, kDtSlots]: up to kDtSlots waves no two
// share a slot.  The slots lie kDtStride words apart, each in a 256-byte
// block of its own: atomics on one address are serialised in the memory
// system, so many distinct addresses keep the reduction off the update's
// critical path.
constexpr int kDtSlots = 512;
constexpr int kDtStride = 32;
constexpr size_t kScalHead = 64;  // t, dt, steps, err, fallbacks (+ padding); the slots follow
inline unsigned dt_slots(size_t cells) {
  unsigned n = 64;
  while (n < kDtSlots && (size_t)n * 64 < cells) n *= 2;
  return n;
}
inline size_t scal_bytes(size_t cells) { return kScalHead + (size_t)dt_slots(cells) * kDtStride * 8; }

// work decomposition of one launch kind over the problems of a group
enum Kind { KK_GA = 0, KK_RECON, KK_FACE, KK_CELL, KK_OBST, KK_COUNT };  // boundary, cells+ring, interfaces, cells, step images

// device descriptor of one problem, read by every kernel
template <typename TS, typename TP, typename TC>
struct Prob {
  Grid<TS, TP> g;
  Phys P;
  BCDev bc[4];
  int recon_vars;            // 0 conservative, 1 characteristic variables
  int admissibility;         // 0: rho, p > 0 at the interface centres; 1: also the factor-two range
  int obst_i0, obst_nj;      // solid step: cells i >= obst_i0, j < obst_nj (none: obst_nj = 0)
  unsigned first[KK_COUNT];  // first logical block of the problem in each kind's launch
  // cell (i, j) inside the solid step (ghost indices included)
  __device__ __forceinline__ bool solid(int i, int j) const { return obst_nj > 0 && i >= obst_i0 && j < obst_nj; }
};

// kernel argument: the group's descriptors and the block-owner table of one kind
template <class PR>
struct KA {
  const PR* __restrict__ probs;
  const uint32_t* __restrict__ owner;
  unsigned nblk;
  int single;  // one problem in the group: every block is its, no table lookup
};

// Blocks are dispatched round robin over the eight XCDs (each with its own
// L2); logical blocks are assigned so that every XCD works on a contiguous
// range of tiles (neighbouring rows share stencil data in its L2).  The map
// is a bijection of [0, nblk).
// A persistent launch (a grid of a multiple of eight blocks, each taking
// blocks b, b + gridDim.x, ...) keeps every block on its XCD's range.
__device__ __forceinline__ unsigned logical_of(unsigned b, unsigned nblk) {
  const unsigned per = nblk >> 3, rem = nblk & 7u, xcd = b & 7u, idx = b >> 3;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}
__device__ __forceinline__ unsigned logical_block(unsigned nblk) { return logical_of(blockIdx.x, nblk); }

// the problem and the item index (local) of thread threadIdx.x of logical block L
template <class PR>
__device__ __forceinline__ const PR& locate_at(const KA<PR>& a, unsigned L, int kind, int& local, int* problem = nullptr) {
  const int p = a.single ? 0 : (int)a.owner[L];
  const PR& Q = a.probs[p];
  local = (int)((L - Q.first[kind]) * blockDim.x + threadIdx.x);
  if (problem) *problem = p;
  return Q;
}

template <class PR>
__device__ __forceinline__ const PR& locate(const KA<PR>& a, int kind, int& local, int* problem = nullptr) {
  const unsigned L = logical_block(a.nblk);
  const int p = a.single ? 0 : (int)a.owner[L];
  const PR& Q = a.probs[p];
  local = (int)((L - Q.first[kind]) * blockDim.x + threadIdx.x);
  if (problem) *problem = p;
  return Q;
}

// ---------------------------------------------------------------------------
// boundary images
// ---------------------------------------------------------------------------

// fixed state at location (x, y) at time t; false where the boundary mirrors
__device__ bool bc_fixed(const BCDev& b, int nv, double x, double y, double t, double* out) {
  if (b.kind == GKS_BC_INFLOW) {
    for (int v = 0; v < nv; ++v) out[v] = b.state[v];
    return true;
  }
  if (b.kind == GKS_BC_DMR_BOTTOM) {
    if (!(x < 1.0 / 6.0)) return false;
    for (int v = 0; v < nv; ++v) out[v] = b.state[v];
    return true;
  }
  if (b.kind == GKS_BC_DMR_TOP) {
    const double xs = 1.0 / 6.0 + (y + 20.0 * t) * 0.57735026918962576451;
    const double* src = x < xs ? b.state : b.alt;
    for (int v = 0; v < nv; ++v) out[v] = src[v];
    return true;
  }
  return false;
}

// wall velocity of boundary `side` at logical position sp along it: a
// turning wall of a curvilinear grid moves at its wall point (linear along
// the boundary's edges, continued linearly past its ends)
template <typename TS, typename TP>
__device__ void wall_velocity(const Grid<TS, TP>& g, const BCDev& b, int side, double sp, double& wu, double& wv) {
  wu = b.wu;
  wv = b.wv;
  if (b.wo == 0.0) return;
  const int nx = g.ix.nx, ny = g.ix.ny, n = side < 2 ? ny : nx;
  const double* v = g.cv.bnd + (side == 0 ? 0 : side == 1 ? 2 * (ny + 1) : side == 2 ? 4 * (ny + 1) : 4 * (ny + 1) + 2 * (nx + 1));
  int e = (int)floor(sp);
  e = e < 0 ? 0 : (e > n - 1 ? n - 1 : e);
  const double f = sp - e;
  const double x = v[2 * e] + f * (v[2 * e + 2] - v[2 * e]), y = v[2 * e + 1] + f * (v[2 * e + 3] - v[2 * e + 1]);
  wu -= b.wo * y;
  wv += b.wo * x;
}

// mirror image of a 2D state across a boundary with normal `axis` (wu, wv:
// the wall velocity of a no-slip wall)
__device__ void bc_mirror(const BCDev& b, int axis, double gamma, const double* s, double* o, double wu,
                          double wv) {
  for (int v = 0; v < 4; ++v) o[v] = s[v];
  const int kind = b.kind;
  if (kind == GKS_BC_REFLECT || kind == GKS_BC_DMR_BOTTOM) {
    o[1 + axis] = -s[1 + axis];
  } else if (kind == GKS_BC_NOSLIP_ISOTHERMAL || kind == GKS_BC_NOSLIP_ADIABATIC) {
    const double rho = s[0], u = s[1] / rho, v = s[2] / rho;
    const double p = (gamma - 1.0) * (s[3] - 0.5 * rho * (u * u + v * v));
    const double T = p / rho;
    const double Tg = kind == GKS_BC_NOSLIP_ISOTHERMAL ? 2.0 * b.wT - T : T;
    const double ug = 2.0 * wu - u, vg = 2.0 * wv - v;
    o[0] = rho;
    o[1] = rho * ug;
    o[2] = rho * vg;
    o[3] = rho * Tg / (gamma - 1.0) + 0.5 * rho * (ug * ug + vg * vg);
  }
}

// mirror image of a 1D state (rho, rho u, rho E)
__device__ void bc_mirror_1d(const BCDev& b, double gamma, const double* s, double* o) {
  for (int v = 0; v < 3; ++v) o[v] = s[v];
  const int kind = b.kind;
  if (kind == GKS_BC_REFLECT) {
    o[1] = -s[1];
  } else if (kind == GKS_BC_NOSLIP_ISOTHERMAL || kind == GKS_BC_NOSLIP_ADIABATIC) {
    const double rho = s[0], u = s[1] / rho;
    const double T = (gamma - 1.0) * (s[2] - 0.5 * rho * u * u) / rho;
    const double Tg = kind == GKS_BC_NOSLIP_ISOTHERMAL ? 2.0 * b.wT - T : T;
    const double ug = 2.0 * b.wu - u;
    o[0] = rho;
    o[1] = rho * ug;
    o[2] = rho * Tg / (gamma - 1.0) + 0.5 * rho * ug * ug;
  }
}

// image of ghost cell (j, ig), ig < 0 or ig >= nx, of an interior row j under
// the west (ig < 0) or east boundary
template <typename TS, typename TP, typename TC>
__device__ void ghost_x_cell(const Prob<TS, TP, TC>& Q, const Grid<TS, TP>& g, double t, int j, int ig, double* out) {
  const int nx = g.ix.nx, side = ig < 0 ? 0 : 1;
  const BCDev& b = Q.bc[side];
  const double xc = g.geo.x0 + (ig + 0.5) * g.geo.h, yc = g.geo.y0 + (j + 0.5) * g.geo.k;
  if (bc_fixed(b, 4, xc, yc, t, out)) return;
  double src[4];
  const int is = b.kind == GKS_BC_PERIODIC ? (side == 0 ? ig + nx : ig - nx) : (side == 0 ? -1 - ig : 2 * nx - 1 - ig);
  for (int v = 0; v < 4; ++v) src[v] = g.W[g.ix.w(v, j, is)];
  if (b.kind == GKS_BC_PERIODIC) {
    for (int v = 0; v < 4; ++v) out[v] = src[v];
  } else {
    double wu, wv;
    wall_velocity(g, b, side, j + 0.5, wu, wv);
    bc_mirror(b, 0, Q.P.gamma, src, out, wu, wv);
  }
}

// West (side 0) / east (side 1): ghost cells of rows 0..ny-1, ghost x
// interfaces -1 / nx+1, and the y interfaces of the ghost columns -1 / nx.
template <typename TS, typename TP, typename TC>
__device__ void ghost_we_item(const Prob<TS, TP, TC>& Q, int id) {
  const Grid<TS, TP> g = Q.g;
  const double gamma = Q.P.gamma;
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int ncell = 2 * ny * 2, nfx = 2 * ny * 2, nfy = 2 * (ny + 1) * 2;
  if (id >= ncell + nfx + nfy) return;
  const double t = *g.t, h = g.geo.h, k = g.geo.k;
  double src[4], out[4];
  if (id < ncell) {
    const int side = id / (2 * ny), r = id % (2 * ny), j = r / 2, m = r % 2;
    const int ig = side == 0 ? -1 - m : nx + m;
    ghost_x_cell(Q, g, t, j, ig, out);
    for (int v = 0; v < 4; ++v) g.W[g.ix.w(v, j, ig)] = out[v];
    return;
  }
  id -= ncell;
  if (id < nfx) {
    const int side = id / (2 * ny), r = id % (2 * ny), j = r / 2, gp = r % 2;
    const BCDev& b = Q.bc[side];
    const int fg = side == 0 ? -1 : nx + 1;
    const double xg = g.geo.x0 + fg * h, yg = g.geo.y0 + (j + 0.5 + (gp ? kGaussOffset : -kGaussOffset)) * k;
    if (!bc_fixed(b, 4, xg, yg, t, out)) {
      const int fs = b.kind == GKS_BC_PERIODIC ? (side == 0 ? nx - 1 : 1) : (side == 0 ? 1 : nx - 1);
      for (int v = 0; v < 4; ++v) src[v] = (double)g.FX[g.ix.fx(gp, v, j, fs)];
      if (b.kind == GKS_BC_PERIODIC) {
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      } else {
        double wu, wv;
        wall_velocity(g, b, side, j + 0.5 + (gp ? kGaussOffset : -kGaussOffset), wu, wv);
        bc_mirror(b, 0, gamma, src, out, wu, wv);
      }
    }
    for (int v = 0; v < 4; ++v) g.FX[g.ix.fx(gp, v, j, fg)] = (TS)out[v];
    return;
  }
  id -= nfx;
  {
    const int side = id / (2 * (ny + 1)), r = id % (2 * (ny + 1)), fj = r / 2, gp = r % 2;
    const BCDev& b = Q.bc[side];
    const int ig = side == 0 ? -1 : nx;
    const double xg = g.geo.x0 + (ig + 0.5 + (gp ? kGaussOffset : -kGaussOffset)) * h, yg = g.geo.y0 + fj * k;
    if (!bc_fixed(b, 4, xg, yg, t, out)) {
      const bool per = b.kind == GKS_BC_PERIODIC;
      const int is = per ? (side == 0 ? nx - 1 : 0) : (side == 0 ? 0 : nx - 1);
      const int gs = per ? gp : 1 - gp;  // a mirror swaps the tangential Gauss points
      for (int v = 0; v < 4; ++v) src[v] = (double)g.FY[g.ix.fy(gs, v, fj, is)];
      if (per) {
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      } else {
        double wu, wv;
        wall_velocity(g, b, side, (double)fj, wu, wv);
        bc_mirror(b, 0, gamma, src, out, wu, wv);
      }
    }
    for (int v = 0; v < 4; ++v) g.FY[g.ix.fy(gp, v, fj, ig)] = (TS)out[v];
  }
}

// South (side 2) / north (side 3): ghost cells of columns -2..nx+1 (the
// corners are the south/north images of the west/east images, composed here
// so that this part does not wait for the west/east part), ghost y interfaces
// -1 / ny+1, and the x interfaces of the ghost rows -1 / ny.
template <typename TS, typename TP, typename TC>
__device__ void ghost_sn_item(const Prob<TS, TP, TC>& Q, int id) {
  const Grid<TS, TP> g = Q.g;
  const double gamma = Q.P.gamma;
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int ncell = 2 * (nx + 4) * 2, nfy = 2 * nx * 2, nfx = 2 * (nx + 1) * 2;
  if (id >= ncell + nfy + nfx) return;
  const double t = *g.t, h = g.geo.h, k = g.geo.k;
  double src[4], out[4];
  if (id < ncell) {
    const int side = id / (2 * (nx + 4)), r = id % (2 * (nx + 4)), i = r / 2 - 2, m = r % 2;
    const BCDev& b = Q.bc[2 + side];
    const int jg = side == 0 ? -1 - m : ny + m;
    const double xc = g.geo.x0 + (i + 0.5) * h, yc = g.geo.y0 + (jg + 0.5) * k;
    if (!bc_fixed(b, 4, xc, yc, t, out)) {
      int js;
      if (b.kind == GKS_BC_PERIODIC)
        js = side == 0 ? jg + ny : jg - ny;
      else
        js = side == 0 ? -1 - jg : 2 * ny - 1 - jg;
      if (i < 0 || i >= nx)
        ghost_x_cell(Q, g, t, js, i, src);
      else
        for (int v = 0; v < 4; ++v) src[v] = g.W[g.ix.w(v, js, i)];
      if (b.kind == GKS_BC_PERIODIC) {
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      } else {
        double wu, wv;
        wall_velocity(g, b, 2 + side, i + 0.5, wu, wv);
        bc_mirror(b, 1, gamma, src, out, wu, wv);
      }
    }
    for (int v = 0; v < 4; ++v) g.W[g.ix.w(v, jg, i)] = out[v];
    return;
  }
  id -= ncell;
  if (id < nfy) {
    const int side = id / (2 * nx), r = id % (2 * nx), i = r / 2, gp = r % 2;
    const BCDev& b = Q.bc[2 + side];
    const int fg = side == 0 ? -1 : ny + 1;
    const double xg = g.geo.x0 + (i + 0.5 + (gp ? kGaussOffset : -kGaussOffset)) * h, yg = g.geo.y0 + fg * k;
    if (!bc_fixed(b, 4, xg, yg, t, out)) {
      const int fs = b.kind == GKS_BC_PERIODIC ? (side == 0 ? ny - 1 : 1) : (side == 0 ? 1 : ny - 1);
      for (int v = 0; v < 4; ++v) src[v] = (double)g.FY[g.ix.fy(gp, v, fs, i)];
      if (b.kind == GKS_BC_PERIODIC) {
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      } else {
        double wu, wv;
        wall_velocity(g, b, 2 + side, i + 0.5 + (gp ? kGaussOffset : -kGaussOffset), wu, wv);
        bc_mirror(b, 1, gamma, src, out, wu, wv);
      }
    }
    for (int v = 0; v < 4; ++v) g.FY[g.ix.fy(gp, v, fg, i)] = (TS)out[v];
    return;
  }
  id -= nfy;
  {
    const int side = id / (2 * (nx + 1)), r = id % (2 * (nx + 1)), fi = r / 2, gp = r % 2;
    const BCDev& b = Q.bc[2 + side];
    const int jg = side == 0 ? -1 : ny;
    const double xg = g.geo.x0 + fi * h, yg = g.geo.y0 + (jg + 0.5 + (gp ? kGaussOffset : -kGaussOffset)) * k;
    if (!bc_fixed(b, 4, xg, yg, t, out)) {
      const bool per = b.kind == GKS_BC_PERIODIC;
      const int js = per ? (side == 0 ? ny - 1 : 0) : (side == 0 ? 0 : ny - 1);
      const int gs = per ? gp : 1 - gp;
      for (int v = 0; v < 4; ++v) src[v] = (double)g.FX[g.ix.fx(gs, v, js, fi)];
      if (per) {
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      } else {
        double wu, wv;
        wall_velocity(g, b, 2 + side, (double)fi, wu, wv);
        bc_mirror(b, 1, gamma, src, out, wu, wv);
      }
    }
    for (int v = 0; v < 4; ++v) g.FX[g.ix.fx(gp, v, jg, fi)] = (TS)out[v];
  }
}

// the step of problem p, by one thread of the boundary kernel (which reads
// neither the step nor the CFL slots): ctl[2p] = fixed step (0: CFL),
// ctl[2p+1] = end time (0: none; the step is shortened to reach it, later
// steps are empty); the slots are reset for the update of this step
// The time step of a problem, taken by the first wave of its boundary launch
// (all 64 lanes active): lane q reads the problem's CFL slots q, q + 64, ...
// and resets them, a shuffle minimum gives the bound, lane 0 writes the step (the fixed
// step if one is set, clipped to the end time if one is set; zero once the
// problem has a nonphysical state).
static_assert(kDtSlots % 64 == 0, "the slots split evenly over the lanes of a wave");
template <typename TS, typename TP, typename TC>
__device__ void step_dt(const Prob<TS, TP, TC>& Q, const double* __restrict__ ctl, int p, int lane) {
  const Grid<TS, TP> g = Q.g;
  const double fixed = ctl[2 * p], t_end = ctl[2 * p + 1], t = *g.t;
  unsigned long long m = ~0ull;
#pragma unroll
  for (int r = 0; r < kDtSlots / 64; ++r) {  // all loads in flight at once
    const unsigned q = lane + 64 * r;
    const unsigned long long o = q <= g.dtmask ? g.dtmin[q * kDtStride] : ~0ull;
    m = o < m ? o : m;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(m, off, 64);
    m = o < m ? o : m;
  }
#pragma unroll
  for (int r = 0; r < kDtSlots / 64; ++r)
    if (lane + 64 * r <= g.dtmask) g.dtmin[(lane + 64 * r) * kDtStride] = (unsigned long long)__double_as_longlong(1e300);
  if (lane == 0) {
    double dt = fixed > 0.0 ? fixed : Q.P.cfl * __longlong_as_double((long long)m);
    if (t_end > 0.0) dt = fmin(dt, fmax(t_end - t, 0.0));
    // after a nonphysical state the problem's steps are empty: its state stays
    // the one the failing step produced
    if (*g.err) dt = 0.0;
    *g.dt = dt;
  }
}

// all 2D boundary images of a problem in one launch, and its time step
template <typename TS, typename TP, typename TC>
__global__ void __launch_bounds__(256) k_ghost_2d(KA<Prob<TS, TP, TC>> a, const double* __restrict__ ctl) {
  int id, p;
  const Prob<TS, TP, TC>& Q = locate(a, KK_GA, id, &p);
  if (id < 64) step_dt(Q, ctl, p, id);
  const int nx = Q.g.ix.nx, ny = Q.g.ix.ny;
  const int nwe = 4 * ny + 4 * ny + 4 * (ny + 1), nsn = 4 * (nx + 4) + 4 * nx + 4 * (nx + 1);
  if (id < nwe)
    ghost_we_item(Q, id);
  else if (id < nwe + nsn)
    ghost_sn_item(Q, id - nwe);
}

// ---------------------------------------------------------------------------
// The solid step (Sec. 4.6): images in the two layers of solid cells along
// its faces, filled after the domain-edge images.  Below the top face the
// slip-wall image across it (v negated), beside the vertical face below
// those two rows the image across that face (u negated); the 2 x 2 block at
// the corner thus takes the top face's image (the paper defers the corner to
// an external reference).  The Gauss-point values between those solid cells
// are imaged alike (a mirror swaps the Gauss points along it), and so are
// the domain-edge images that the first solid layer reads: the south images
// below the vertical face's solid columns and the east images of the top
// face's solid rows, each the edge's own image of the solid cell's image.
// Every item reads gas data only and writes solid data only.
// ---------------------------------------------------------------------------
__host__ __device__ inline int step_items(int nx, int i0, int nj) {
  const int w = nx - i0;
  return 2 * w + 2 * (nj - 2) + 4 + 4 + 4 * w + 2 * (nj - 2) + 2 * w + 2 * (nj - 1);
}

__device__ __forceinline__ void flip_uv(const double* s, bool fu, bool fv, double* o) {
#pragma unroll
  for (int v = 0; v < 4; ++v) o[v] = s[v];
  if (fu) o[1] = -s[1];
  if (fv) o[2] = -s[2];
}

template <typename TS, typename TP, typename TC>
__global__ void __launch_bounds__(256) k_step_images_2d(KA<Prob<TS, TP, TC>> a) {
  int id;
  const Prob<TS, TP, TC>& Q = locate(a, KK_OBST, id);
  const Grid<TS, TP> g = Q.g;
  const Idx& x = g.ix;
  const int nx = x.nx, i0 = Q.obst_i0, nj = Q.obst_nj, w = nx - i0;
  if (nj <= 0 || id >= step_items(nx, i0, nj)) return;
  const double gamma = Q.P.gamma;
  double src[4], out[4], mid[4];
  // cells: the two rows below the top face
  if (id < 2 * w) {
    const int dy = id / w, i = i0 + id % w;
    for (int v = 0; v < 4; ++v) src[v] = g.W[x.w(v, nj + dy, i)];
    flip_uv(src, false, true, out);
    for (int v = 0; v < 4; ++v) g.W[x.w(v, nj - 1 - dy, i)] = out[v];
    return;
  }
  id -= 2 * w;
  // cells: the two columns beside the vertical face below them
  if (id < 2 * (nj - 2)) {
    const int dx = id / (nj - 2), j = id % (nj - 2);
    for (int v = 0; v < 4; ++v) src[v] = g.W[x.w(v, j, i0 - 1 - dx)];
    flip_uv(src, true, false, out);
    for (int v = 0; v < 4; ++v) g.W[x.w(v, j, i0 + dx)] = out[v];
    return;
  }
  id -= 2 * (nj - 2);
  // the south edge's images of the vertical face's solid columns
  if (id < 4) {
    const int dx = id / 2, m = id % 2;
    for (int v = 0; v < 4; ++v) src[v] = g.W[x.w(v, m, i0 - 1 - dx)];
    flip_uv(src, true, false, mid);
    bc_mirror(Q.bc[2], 1, gamma, mid, out, Q.bc[2].wu, Q.bc[2].wv);
    for (int v = 0; v < 4; ++v) g.W[x.w(v, -1 - m, i0 + dx)] = out[v];
    return;
  }
  id -= 4;
  // the east edge's images of the top face's solid rows
  if (id < 4) {
    const int m = id / 2, dy = id % 2;
    for (int v = 0; v < 4; ++v) src[v] = g.W[x.w(v, nj + dy, nx - 1 - m)];
    flip_uv(src, false, true, mid);
    bc_mirror(Q.bc[1], 0, gamma, mid, out, Q.bc[1].wu, Q.bc[1].wv);
    for (int v = 0; v < 4; ++v) g.W[x.w(v, nj - 1 - dy, nx + m)] = out[v];
    return;
  }
  id -= 4;
  // x interfaces i0+1..nx of the two rows below the top face
  if (id < 4 * w) {
    const int dy = id / (2 * w), r = id % (2 * w), fi = i0 + 1 + r / 2, gp = r % 2;
    for (int v = 0; v < 4; ++v) src[v] = (double)g.FX[x.fx(1 - gp, v, nj + dy, fi)];
    flip_uv(src, false, true, out);
    for (int v = 0; v < 4; ++v) g.FX[x.fx(gp, v, nj - 1 - dy, fi)] = (TS)out[v];
    return;
  }
  id -= 4 * w;
  // x interface i0+1 beside the vertical face below them
  if (id < 2 * (nj - 2)) {
    const int j = id / 2, gp = id % 2;
    for (int v = 0; v < 4; ++v) src[v] = (double)g.FX[x.fx(gp, v, j, i0 - 1)];
    flip_uv(src, true, false, out);
    for (int v = 0; v < 4; ++v) g.FX[x.fx(gp, v, j, i0 + 1)] = (TS)out[v];
    return;
  }
  id -= 2 * (nj - 2);
  // y interface nj-1 of the columns i0..nx-1
  if (id < 2 * w) {
    const int i = i0 + id / 2, gp = id % 2;
    for (int v = 0; v < 4; ++v) src[v] = (double)g.FY[x.fy(gp, v, nj + 1, i)];
    flip_uv(src, false, true, out);
    for (int v = 0; v < 4; ++v) g.FY[x.fy(gp, v, nj - 1, i)] = (TS)out[v];
    return;
  }
  id -= 2 * w;
  // y interfaces 0..nj-2 of column i0
  {
    const int fj = id / 2, gp = id % 2;
    for (int v = 0; v < 4; ++v) src[v] = (double)g.FY[x.fy(1 - gp, v, fj, i0 - 1)];
    flip_uv(src, true, false, out);
    for (int v = 0; v < 4; ++v) g.FY[x.fy(gp, v, fj, i0)] = (TS)out[v];
  }
}

// 1D: tasks (side, m), m = 0, 1 ghost cells -1-m / nx+m, m = 2 the ghost
// interface -1 / nx+1
template <typename TS, typename TP, typename TC>
__global__ void __launch_bounds__(256) k_ghost_1d(KA<Prob<TS, TP, TC>> a, const double* __restrict__ ctl) {
  int id, p;
  const Prob<TS, TP, TC>& Q = locate(a, KK_GA, id, &p);
  if (id < 64) step_dt(Q, ctl, p, id);
  if (id >= 6) return;
  const Grid<TS, TP> g = Q.g;
  const double gamma = Q.P.gamma;
  const int nx = g.ix.nx, side = id / 3, m = id % 3;
  const BCDev& b = Q.bc[side];
  const bool per = b.kind == GKS_BC_PERIODIC;
  const double t = *g.t;
  double src[4], out[4];
  if (m < 2) {
    const int ig = side == 0 ? -1 - m : nx + m;
    if (!bc_fixed(b, 3, 0.0, 0.0, t, out)) {
      const int is = per ? (side == 0 ? ig + nx : ig - nx) : (side == 0 ? -1 - ig : 2 * nx - 1 - ig);
      for (int v = 0; v < 3; ++v) src[v] = g.W[g.ix.w1(v, is)];
      if (per)
        for (int v = 0; v < 3; ++v) out[v] = src[v];
      else
        bc_mirror_1d(b, gamma, src, out);
    }
    for (int v = 0; v < 3; ++v) g.W[g.ix.w1(v, ig)] = out[v];
  } else {
    const int fg = side == 0 ? -1 : nx + 1;
    if (!bc_fixed(b, 3, 0.0, 0.0, t, out)) {
      const int fs = per ? (side == 0 ? nx - 1 : 1) : (side == 0 ? 1 : nx - 1);
      for (int v = 0; v < 3; ++v) src[v] = (double)g.FX[g.ix.f1(v, fs)];
      if (per)
        for (int v = 0; v < 3; ++v) out[v] = src[v];
      else
        bc_mirror_1d(b, gamma, src, out);
    }
    for (int v = 0; v < 3; ++v) g.FX[g.ix.f1(v, fg)] = (TS)out[v];
  }
}

// ---------------------------------------------------------------------------
// time step: dt = cfl * min over cells of min(h/(|u|+c+2nu/h), k/(|v|+c+2nu/k))
// The per-cell bound is reduced into the slots g.dtmin (bits of positive
// doubles, ordered like unsigned integers) by the update kernel for the next
// step (and by its scan form for the initial state); step_dt takes the minimum
// of the slots, turns it into the step and resets them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cell_dt_bound(const double* W, const Phys& P, double h, double k) {
  const double rho = W[0], u = W[1] / rho, v = W[2] / rho;
  const double p = (P.gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v));
  const double cs = sqrt(P.gamma * p / rho);
  const double nu = P.viscous ? P.mu / rho : 0.0;
  return fmin(h / (fabs(u) + cs + 2.0 * nu / h), k / (fabs(v) + cs + 2.0 * nu / k));
}

// curvilinear grids: the widths w1, w2 across the two logical directions and
// the speed
__device__ __forceinline__ double cell_dt_bound_curv(const double* W, const Phys& P, double w1, double w2) {
  const double rho = W[0], u = W[1] / rho, v = W[2] / rho;
  const double p = (P.gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v));
  const double cs = sqrt(P.gamma * p / rho), sp = sqrt(u * u + v * v);
  const double nu = P.viscous ? P.mu / rho : 0.0;
  return fmin(w1 / (sp + cs + 2.0 * nu / w1), w2 / (sp + cs + 2.0 * nu / w2));
}

__device__ __forceinline__ double cell_dt_bound_1d(const double* W, const Phys& P, double h) {
  const double rho = W[0], u = W[1] / rho;
  const double p = (P.gamma - 1.0) * (W[2] - 0.5 * rho * u * u);
  const double cs = sqrt(P.gamma * p / rho);
  const double nu = P.viscous ? P.mu / rho : 0.0;
  return h / (fabs(u) + cs + 2.0 * nu / h);
}

// wave minimum of a positive bound, one atomic per wave into slot
// (wave within the problem) & mask (NaN bounds of a nonphysical cell are
// skipped; the update flags that cell).  Every lane of the wave takes part.
__device__ __forceinline__ void reduce_dt_bound(double b, unsigned long long* slots, unsigned wave, unsigned mask) {
  if (!(b > 0.0) || !isfinite(b)) b = 1e300;
  for (int off = 32; off > 0; off >>= 1) b = fmin(b, __shfl_down(b, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMin(slots + (wave & mask) * kDtStride, (unsigned long long)__double_as_longlong(b));
}

// ---------------------------------------------------------------------------
// reconstruction
// ---------------------------------------------------------------------------

// 2D: cells -1..nx x -1..ny except the four corners; kChar: the limiter of
// each direction in that direction's characteristic variables.  Wn: the
// averages of the cell and its east, west, north, south neighbours.
template <typename TS, typename TP, typename TC, bool kChar>
__device__ __forceinline__ void recon_cell_2d(const Prob<TS, TP, TC>& Q, const Grid<TS, TP>& g, int i, int j,
                                              const double (&Wn)[5][4]) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  // a curvilinear grid reconstructs in logical coordinates (h = k = 1) with
  // I(U1) = C |K|, the cell's area
  const double h = g.geo.h, k = g.geo.k, eps = Q.P.weno_eps, gamma = Q.P.gamma;
  const double Cw = Q.P.weno_c * (g.cv.area ? g.cv.area[(size_t)(j + 1) * (nx + 2) + (i + 1)] : 1.0);
  const Idx& x = g.ix;
  // ties of the cross-derivative candidates: the rounding noise of the stored
  // point values -- in double the accumulated rounding of the arithmetic that
  // made them (128 units, 2^-46); in single precision their storage rounding
  // (one unit, 2^-24), which exceeds that arithmetic noise
  constexpr double kTieRel = sizeof(TS) == 4 ? 5.9604644775390625e-08 : 1.4210854715202004e-14;
  double p[4][5], Wc[4];
  const ReconDiv D(h, k);
  if constexpr (!kChar) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wc[v] = Wn[0][v];
      recon_2d(Wc[v], Wn[1][v], Wn[2][v], Wn[3][v], Wn[4][v], (double)g.FX[x.fx(1, v, j, i + 1)],
               (double)g.FX[x.fx(0, v, j, i + 1)], (double)g.FX[x.fx(1, v, j, i)], (double)g.FX[x.fx(0, v, j, i)],
               (double)g.FY[x.fy(1, v, j + 1, i)], (double)g.FY[x.fy(0, v, j + 1, i)],
               (double)g.FY[x.fy(1, v, j, i)], (double)g.FY[x.fy(0, v, j, i)], h, k, eps, Cw, D, kTieRel, p[v]);
    }
  } else {
    double S[13][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wc[v] = Wn[0][v];
#pragma unroll
      for (int q = 0; q < 5; ++q) S[q][v] = Wn[q][v];
      S[5][v] = (double)g.FX[x.fx(1, v, j, i + 1)];
      S[6][v] = (double)g.FX[x.fx(0, v, j, i + 1)];
      S[7][v] = (double)g.FX[x.fx(1, v, j, i)];
      S[8][v] = (double)g.FX[x.fx(0, v, j, i)];
      S[9][v] = (double)g.FY[x.fy(1, v, j + 1, i)];
      S[10][v] = (double)g.FY[x.fy(0, v, j + 1, i)];
      S[11][v] = (double)g.FY[x.fy(1, v, j, i)];
      S[12][v] = (double)g.FY[x.fy(0, v, j, i)];
    }
    double lim[4][4];
    if (recon_pair_characteristic<true>(gamma, S, h, D.h, D.hh, D.six, lim) &&
        recon_pair_characteristic<false>(gamma, S, k, D.k, D.kk, D.six, lim)) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        recon_finish(S[0][v], S[1][v], S[2][v], S[3][v], S[4][v], S[5][v], S[6][v], S[7][v], S[8][v], S[9][v],
                     S[10][v], S[11][v], S[12][v], h, k, eps, Cw, D, lim[v][0], lim[v][1], lim[v][2], lim[v][3],
                     kTieRel, p[v]);
    } else {
      // a nonphysical average: the constant polynomial (the interfaces and
      // the update report the state)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int m = 0; m < 5; ++m) p[v][m] = 0.0;
    }
  }
  // an inadmissible polynomial is replaced by the constant cell average for
  // this step
  Range rg;
#pragma unroll
  for (int q = 0; q < 5; ++q) rg.add(Wn[q][0], pressure_2d(gamma, Wn[q]));
  const bool ok = recon_admissible_2d(Wc, p, h, k, gamma, rg, Q.admissibility);
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int m = 0; m < 5; ++m) g.PC[x.pc(v, m, j, i)] = ok ? (TP)p[v][m] : TP(0);
  // count of interior gas cells that fell back (rare: one atomic per such cell)
  if (!ok && i >= 0 && i < nx && j >= 0 && j < ny && !Q.solid(i, j) && *g.dt > 0.0) atomicAdd(g.nfall, 1ull);
}

// one thread per cell of the range, in row order
template <typename TS, typename TP, typename TC, bool kChar>
__global__ void __launch_bounds__(256) k_recon_2d(KA<Prob<TS, TP, TC>> a) {
  int id;
  const Prob<TS, TP, TC>& Q = locate(a, KK_RECON, id);
  const Grid<TS, TP> g = Q.g;
  const int nx = g.ix.nx, ny = g.ix.ny;
  if (id >= (nx + 2) * (ny + 2)) return;
  const int j = id / (nx + 2) - 1, i = id % (nx + 2) - 1;
  if ((i < 0 || i >= nx) && (j < 0 || j >= ny)) return;
  const Idx& x = g.ix;
  double Wn[5][4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    Wn[0][v] = g.W[x.w(v, j, i)];
    Wn[1][v] = g.W[x.w(v, j, i + 1)];
    Wn[2][v] = g.W[x.w(v, j, i - 1)];
    Wn[3][v] = g.W[x.w(v, j + 1, i)];
    Wn[4][v] = g.W[x.w(v, j - 1, i)];
  }
  recon_cell_2d<TS, TP, TC, kChar>(Q, g, i, j, Wn);
}

// Tiled form: a block takes a tile of tx x rows cells of the range (rows =
// blockDim.x / tx) and first stages the averages of the tile and its
// one-cell ring in LDS (the compact stencil's five averages per cell then
// come from LDS; each average is read from memory once per tile); the
// arithmetic is the row-order form's.  Every thread of the block takes part
// in the staging and the barrier before it leaves.
template <typename TS, typename TP, typename TC, bool kChar>
__global__ void __launch_bounds__(256) k_recon_2d_tile(KA<Prob<TS, TP, TC>> a, int rows) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* sw = (double*)lds_raw;  // [4][rows + 2][tx + 2]
  const unsigned L = logical_block(a.nblk);
  const int p = a.single ? 0 : (int)a.owner[L];
  const Prob<TS, TP, TC>& Q = a.probs[p];
  const Grid<TS, TP> g = Q.g;
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int tx = (int)blockDim.x / rows, ntx = (nx + 2 + tx - 1) / tx;
  const int lb = (int)(L - Q.first[KK_RECON]);
  const int i0 = (lb % ntx) * tx - 1, j0 = (lb / ntx) * rows - 1;  // first cell of the tile
  const int sx = tx + 2, sy = rows + 2;
  const Idx& x = g.ix;
  // stage cells i0-1..i0+tx, j0-1..j0+rows (inside the ghosted array)
  for (int q = threadIdx.x; q < 4 * sx * sy; q += blockDim.x) {
    const int v = q / (sx * sy), r = q % (sx * sy), ci = i0 - 1 + r % sx, cj = j0 - 1 + r / sx;
    if (ci >= -2 && ci <= nx + 1 && cj >= -2 && cj <= ny + 1) sw[q] = g.W[x.w(v, cj, ci)];
  }
  __syncthreads();
  const int ti = (int)threadIdx.x % tx, tj = (int)threadIdx.x / tx, i = i0 + ti, j = j0 + tj;
  if (i > nx || j > ny) return;
  if ((i < 0 || i >= nx) && (j < 0 || j >= ny)) return;
  double Wn[5][4];
  const int c = (tj + 1) * sx + (ti + 1);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double* s = sw + v * sx * sy;
    Wn[0][v] = s[c];
    Wn[1][v] = s[c + 1];
    Wn[2][v] = s[c - 1];
    Wn[3][v] = s[c + sx];
    Wn[4][v] = s[c - sx];
  }
  recon_cell_2d<TS, TP, TC, kChar>(Q, g, i, j, Wn);
}

// 1D: cells -1..nx, in conservative or characteristic variables (Sec. 4:
// characteristic variables of the cell's own state)
template <typename TS, typename TP, typename TC>
__global__ void __launch_bounds__(256) k_recon_1d(KA<Prob<TS, TP, TC>> a) {
  int id;
  const Prob<TS, TP, TC>& Q = locate(a, KK_RECON, id);
  const Grid<TS, TP> g = Q.g;
  const int nx = g.ix.nx;
  if (id >= nx + 2) return;
  const int i = id - 1;
  const double h = g.geo.h, eps = Q.P.weno_eps, Cw = Q.P.weno_c;
  const Idx& x = g.ix;
  double s[5][3];  // cell, east, west averages; right and left interface values
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    s[0][v] = g.W[x.w1(v, i)];
    s[1][v] = g.W[x.w1(v, i + 1)];
    s[2][v] = g.W[x.w1(v, i - 1)];
    s[3][v] = (double)g.FX[x.f1(v, i + 1)];
    s[4][v] = (double)g.FX[x.f1(v, i)];
  }
  double p[3][2];
  if (Q.recon_vars == 1) {
    double R[3][3], L[3][3];
    if (!euler_eigen_1d(Q.P.gamma, s[0], R, L)) {
      // a nonphysical average is reported by the interfaces and the update
#pragma unroll
      for (int v = 0; v < 3; ++v) p[v][0] = p[v][1] = 0.0;
    } else {
      double c[5][3];
#pragma unroll
      for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma clang fp contract(off)
          double acc = 0.0;
#pragma unroll
          for (int v = 0; v < 3; ++v) acc += L[r][v] * s[q][v];
          c[q][r] = acc;
        }
      double pc[3][2];
#pragma unroll
      for (int r = 0; r < 3; ++r) recon_1d(c[0][r], c[1][r], c[2][r], c[3][r], c[4][r], h, eps, Cw, pc[r]);
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          double acc = 0.0;
#pragma unroll
          for (int r = 0; r < 3; ++r) acc += R[v][r] * pc[r][m];
          p[v][m] = acc;
        }
    }
  } else {
#pragma unroll
    for (int v = 0; v < 3; ++v) recon_1d(s[0][v], s[1][v], s[2][v], s[3][v], s[4][v], h, eps, Cw, p[v]);
  }
  // an inadmissible polynomial is replaced by the constant cell average
  Range rg;
#pragma unroll
  for (int q = 0; q < 3; ++q) rg.add(s[q][0], pressure_1d(Q.P.gamma, s[q]));
  const double Wc[3] = {s[0][0], s[0][1], s[0][2]};
  const bool ok = recon_admissible_1d(Wc, p, h, Q.P.gamma, rg, Q.admissibility);
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < 2; ++m) g.PC[x.pc1(v, m, i)] = ok ? (TP)p[v][m] : TP(0);
  if (!ok && i >= 0 && i < nx && *g.dt > 0.0) atomicAdd(g.nfall, 1ull);
}

// ---------------------------------------------------------------------------
// 2D interfaces: one thread per interface, x interfaces first, then y
// interfaces; one kernel whose sections (prologue, hydrodynamic part, kinetic
// part of each side) hand the frame record of g0 on through LDS.
// ---------------------------------------------------------------------------
struct Face {
  bool isx;   // x interface (else y)
  int a, b;   // x: (j, fi); y: (fj, i)
};

// both cells of interface F inside the solid step of Q (no flux, no point
// values: the interface is skipped by every phase)
template <class PR>
__device__ __forceinline__ bool inside_step(const PR& Q, const Face& F) {
  return F.isx ? Q.solid(F.b - 1, F.a) && Q.solid(F.b, F.a) : Q.solid(F.b, F.a - 1) && Q.solid(F.b, F.a);
}

__device__ __forceinline__ Face face_of(const Idx& x, int id) {
  const int nfx = x.fxr * x.ny;
  Face F;
  F.isx = id < nfx;
  if (F.isx) {
    F.a = id / x.fxr;
    F.b = id % x.fxr;
  } else {
    const int r = id - nfx;
    F.a = r / x.nx;
    F.b = r % x.nx;
  }
  return F;
}

// interface-frame component of global component v: y interfaces swap the
// two momentum components
__device__ __forceinline__ int loc(bool isx, int v) { return isx ? v : (v == 1 ? 2 : v == 2 ? 1 : v); }

__device__ __forceinline__ int n_faces(const Idx& x) { return x.fxr * x.ny + x.nx * x.fyr; }

// average and reconstruction of side s's cell of interface F in the interface
// frame (y interfaces swap the momentum components and the two directions)
template <typename TS, typename TP>
__device__ __forceinline__ void load_face_cell(const Grid<TS, TP>& g, const Face& F, int s, double (&Wc)[4],
                                               double (&pc)[4][5]) {
  const Idx& x = g.ix;
  if (F.isx) {
    const int j = F.a, ic = F.b - 1 + s;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wc[v] = g.W[x.w(v, j, ic)];
      pc[v][0] = (double)g.PC[x.pc(v, 0, j, ic)];  // p_n  = p2
      pc[v][1] = (double)g.PC[x.pc(v, 1, j, ic)];  // p_s  = p3
      pc[v][2] = (double)g.PC[x.pc(v, 2, j, ic)];  // p_nn = p4
      pc[v][3] = (double)g.PC[x.pc(v, 3, j, ic)];  // p_ss = p5
      pc[v][4] = (double)g.PC[x.pc(v, 4, j, ic)];  // p_ns = p6
    }
  } else {
    const int jc = F.a - 1 + s, i = F.b;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int vl = loc(false, v);
      Wc[vl] = g.W[x.w(v, jc, i)];
      pc[vl][0] = (double)g.PC[x.pc(v, 1, jc, i)];  // p_n  = p3
      pc[vl][1] = (double)g.PC[x.pc(v, 0, jc, i)];  // p_s  = p2
      pc[vl][2] = (double)g.PC[x.pc(v, 3, jc, i)];  // p_nn = p5
      pc[vl][3] = (double)g.PC[x.pc(v, 2, jc, i)];  // p_ss = p4
      pc[vl][4] = (double)g.PC[x.pc(v, 4, jc, i)];  // p_ns = p6
    }
  }
}

// Reflective walls of the solid step (Sec. 4.6): on an interface between a
// gas cell and a solid cell the solid side is the mirror image of the gas
// side across that interface, so the wall passes no mass.  (The solid image
// layers serve the gas cells' reconstruction; at the corner one solid cell
// cannot be the image across both faces.)  wall_side: the solid side (0 or
// 1) of interface F, -1 if it is no wall.
template <class PR>
__device__ __forceinline__ int wall_side(const PR& Q, const Face& F) {
  if (Q.obst_nj <= 0) return -1;
  const bool s0 = F.isx ? Q.solid(F.b - 1, F.a) : Q.solid(F.b, F.a - 1);
  const bool s1 = Q.solid(F.b, F.a);
  return s0 == s1 ? -1 : (s0 ? 0 : 1);
}

// the image of a side across the interface, in the interface frame: the
// normal momentum (component 1) and the odd orders in the normal
// coordinate (p_n, p_ns) negated
__device__ __forceinline__ void mirror_side(double (&Wc)[4], double (&pc)[4][5]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double sg = v == 1 ? -1.0 : 1.0;
    Wc[v] *= sg;
    pc[v][0] *= -sg;
    pc[v][1] *= sg;
    pc[v][2] *= sg;
    pc[v][3] *= sg;
    pc[v][4] *= -sg;
  }
}

// Curvilinear grids: the frame of interface F, fr = (unit normal, unit
// tangent, length L, metric G_nn, G_ns)
template <typename TS, typename TP>
__device__ __forceinline__ void face_geo(const Grid<TS, TP>& g, const Face& F, double (&fr)[kFaceGeo]) {
  const Idx& x = g.ix;
  const double* base = F.isx ? g.cv.fx : g.cv.fy;
  const size_t plane = F.isx ? (size_t)x.ny * (x.nx + 1) : (size_t)(x.ny + 1) * x.nx;
  const size_t o = F.isx ? (size_t)F.a * (x.nx + 1) + F.b : (size_t)F.a * x.nx + F.b;
#pragma unroll
  for (int q = 0; q < kFaceGeo; ++q) fr[q] = base[q * plane + o];
}

// momentum components (x, y) -> (normal, tangential) of frame fr
__device__ __forceinline__ void to_face(const double (&fr)[kFaceGeo], double& m1, double& m2) {
  const double a = fr[0] * m1 + fr[1] * m2, b = fr[2] * m1 + fr[3] * m2;
  m1 = a;
  m2 = b;
}

// Side s of interface F of a curvilinear grid in the interface frame: the
// value and logical derivatives of the side cell's polynomial (logical
// coordinates, unit spacing) at the interface centre, turned into frame
// derivatives by the metric (d/dn = G_nn d/dxi + G_ns d/deta, d/dt =
// d/deta / L; second derivatives likewise) and frame momentum, then written
// as the average and coefficients that side_state_2d and side_targets_2d
// read with hn = 1 and hs = L.
template <typename TS, typename TP>
__device__ __forceinline__ void load_face_cell_curv(const Grid<TS, TP>& g, const Face& F, int s,
                                                    const double (&fr)[kFaceGeo], double (&Wc)[4],
                                                    double (&pc)[4][5]) {
  const Idx& x = g.ix;
  const double xn = s == 0 ? 0.5 : -0.5, L = fr[4], g00 = fr[5], g01 = fr[6], g11 = 1.0 / L;
  double U[4], D[5][4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double w, pn, ps, pnn, pss, pns;
    if (F.isx) {
      const int j = F.a, ic = F.b - 1 + s;
      w = g.W[x.w(v, j, ic)];
      pn = (double)g.PC[x.pc(v, 0, j, ic)];
      ps = (double)g.PC[x.pc(v, 1, j, ic)];
      pnn = (double)g.PC[x.pc(v, 2, j, ic)];
      pss = (double)g.PC[x.pc(v, 3, j, ic)];
      pns = (double)g.PC[x.pc(v, 4, j, ic)];
    } else {
      const int jc = F.a - 1 + s, i = F.b;
      w = g.W[x.w(v, jc, i)];
      pn = (double)g.PC[x.pc(v, 1, jc, i)];
      ps = (double)g.PC[x.pc(v, 0, jc, i)];
      pnn = (double)g.PC[x.pc(v, 3, jc, i)];
      pss = (double)g.PC[x.pc(v, 2, jc, i)];
      pns = (double)g.PC[x.pc(v, 4, jc, i)];
    }
    U[v] = w + pn * xn + pnn * (1.0 / 12.0) - pss * (1.0 / 24.0);
    const double ln = pn + pnn * xn, ls = ps + pns * xn;
    D[0][v] = g00 * ln + g01 * ls;
    D[1][v] = g11 * ls;
    D[2][v] = g00 * g00 * pnn + 2.0 * g00 * g01 * pns + g01 * g01 * pss;
    D[3][v] = g11 * g11 * pss;
    D[4][v] = g11 * (g00 * pns + g01 * pss);
  }
  to_face(fr, U[1], U[2]);
#pragma unroll
  for (int k = 0; k < 5; ++k) to_face(fr, D[k][1], D[k][2]);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    pc[v][2] = D[2][v];
    pc[v][3] = D[3][v];
    pc[v][4] = D[4][v];
    pc[v][0] = D[0][v] - D[2][v] * xn;
    pc[v][1] = D[1][v] - D[4][v] * xn;
    Wc[v] = U[v] - pc[v][0] * xn - D[2][v] * (1.0 / 12.0) + D[3][v] * (L * L * (1.0 / 24.0));
  }
}

// LDS bytes per thread of k_iface_2d: the frame record of g0 and the
// accumulated flux and point values (interface frame)
template <typename TC>
constexpr unsigned iface_lds_per_thread() {
  return ND_REC * 8 + nt_rec<TC>() * sizeof(TC) + 12 * 8;
}

// Section boundary of k_iface_2d: values pass between sections only through
// the thread's LDS slots (the memory clobber), and the scheduler moves no
// instruction across, so that each section holds only its own working set.
__device__ __forceinline__ void section_boundary() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// One thread per 2D interface (x interfaces first, then y interfaces): the
// prologue, the hydrodynamic part and the kinetic parts of the two sides in
// sequence, the frame record and the running sums in the thread's slots of
// LDS, the flux and the point values stored once at the end.  No thread
// reads another's slots (no barrier), so a block may take several logical
// blocks in turn.
// kCurv: the problems of the launch are curvilinear grids (each interface
// in the frame of its edge; no solid step)
template <typename TS, typename TP, typename TC, bool kCurv, unsigned NB>
__device__ __forceinline__ void iface_2d_block(const KA<Prob<TS, TP, TC>>& a, unsigned L, unsigned char* lds) {
  int id;
  const Prob<TS, TP, TC>& Q = locate_at(a, L, KK_FACE, id);
  const Grid<TS, TP> g = Q.g;
  if (id >= n_faces(g.ix)) return;
  const double dt = *g.dt;  // tested after the loads below, which do not wait for it
  const Phys P = Q.P;
  const Idx& x = g.ix;
  const Face F = face_of(x, id);
  if (!kCurv && inside_step(Q, F)) return;
  const int ws = kCurv ? -1 : wall_side(Q, F);
  // the block size as a constant: the record's addresses are immediate
  // offsets, and neighbouring entries pair into one LDS access
  const unsigned nb = NB, me = threadIdx.x;
  const Rec<TC> R{(double*)lds, (TC*)(lds + (size_t)ND_REC * 8 * nb), nb};
  double* acc = (double*)(lds + (size_t)(ND_REC * 8 + nt_rec<TC>() * sizeof(TC)) * nb);  // [12][nb]
  double hn = F.isx ? g.geo.h : g.geo.k, hs = F.isx ? g.geo.k : g.geo.h;
  if constexpr (kCurv) {
    double fr[kFaceGeo];
    face_geo(g, F, fr);
    hn = 1.0;
    hs = fr[4];
  }
  // prologue
  {
    double Wc[2][4], pc[2][4][5], Ueq[2][3][4], flux[4], pv[4];
    double fr[kFaceGeo];
    if constexpr (kCurv) {
      face_geo(g, F, fr);
      load_face_cell_curv(g, F, 0, fr, Wc[0], pc[0]);
      load_face_cell_curv(g, F, 1, fr, Wc[1], pc[1]);
    } else {
      load_face_cell(g, F, 0, Wc[0], pc[0]);
      load_face_cell(g, F, 1, Wc[1], pc[1]);
    }
    if (kCurv && !F.isx) {
      // logical orientation, frame momentum below
      const int fj = F.a, i = F.b;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 3; ++n)
#pragma unroll
          for (int v = 0; v < 4; ++v) Ueq[m][n][v] = g.W[x.w(v, fj - 1 + m, i - 1 + n)];
    } else if (F.isx) {
      const int j = F.a, fi = F.b;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 3; ++n)
#pragma unroll
          for (int v = 0; v < 4; ++v) Ueq[m][n][v] = g.W[x.w(v, j - 1 + n, fi - 1 + m)];
    } else {
      const int fj = F.a, i = F.b;
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 3; ++n)
#pragma unroll
          for (int v = 0; v < 4; ++v) Ueq[m][n][loc(false, v)] = g.W[x.w(v, fj - 1 + m, i - 1 + n)];
    }
    // a wall of the step: the solid side and its stencil row are the gas
    // side's image (constant indices only: the arrays stay in registers)
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (ws == s) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Wc[s][v] = Wc[1 - s][v];
#pragma unroll
          for (int m = 0; m < 5; ++m) pc[s][v][m] = pc[1 - s][v][m];
#pragma unroll
          for (int n = 0; n < 3; ++n) Ueq[s][n][v] = (v == 1 ? -1.0 : 1.0) * Ueq[1 - s][n][v];
        }
        mirror_side(Wc[s], pc[s]);
      }
    double Gm[3] = {0.0, 0.0, 0.0};
    if constexpr (kCurv) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 3; ++n) to_face(fr, Ueq[m][n][1], Ueq[m][n][2]);
      Gm[0] = fr[5];
      Gm[1] = fr[6];
      Gm[2] = 1.0 / fr[4];
    }
    if (!(dt > 0.0)) return;  // an empty step (end time reached, or after a nonphysical state)
    const bool ok = iface_prologue_2d<TC, kCurv>(P, dt, hn, hs, Wc, pc, Ueq, R, me, flux, pv, Gm);
    if (!ok) {
      R.D(D_RHO0, me) = 0.0;  // the later sections add nothing
      atomicCAS(g.err, 0ull,
                1ull + ((unsigned long long)(F.a + 1) << 32) + (unsigned long long)(F.b + 1) + (F.isx ? 0ull : 1ull << 62));
#pragma unroll
      for (int v = 0; v < 4; ++v) flux[v] = pv[v] = 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc[v * nb + me] = flux[v];
      acc[(4 + v) * nb + me] = pv[v];
      acc[(8 + v) * nb + me] = pv[v];
    }
  }
  section_boundary();
  // hydrodynamic part (eq. dis1)
  {
    const bool valid = R.D(D_RHO0, me) > 0.0;
    double flux[4], pvm[4], pvp[4], E[4];
    iface_hydro_2d<TC>(P, dt, hs, R, me, flux, pvm, pvp, E);
    if (valid) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[v * nb + me] += flux[v];
        acc[(4 + v) * nb + me] += pvm[v];
        acc[(8 + v) * nb + me] += pvp[v];
        if (P.viscous) R.D(D_E0 + v, me) += E[v];
      }
    }
  }
  // kinetic parts (eq. dis2) of side 0 (g_l on u > 0), then side 1 (g_r on u < 0)
#pragma unroll 1
  for (int side = 0; side < 2; ++side) {
    section_boundary();
    const bool valid = R.D(D_RHO0, me) > 0.0;
    double Wc[4], pc[4][5];
    if constexpr (sides_in_record<TC>()) {
      // the side's state and targets come from the record
    } else if constexpr (kCurv) {
      double fr[kFaceGeo];
      face_geo(g, F, fr);
      load_face_cell_curv(g, F, side, fr, Wc, pc);
    } else {
      load_face_cell(g, F, side == ws ? 1 - side : side, Wc, pc);
      if (side == ws) mirror_side(Wc, pc);
    }
    double flux[4], pvm[4], pvp[4], E[4];
    iface_kinetic_2d<TC>(P, dt, hn, hs, side, Wc, pc, R, me, flux, pvm, pvp, E);
    if (valid) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[v * nb + me] += flux[v];
        acc[(4 + v) * nb + me] += pvm[v];
        acc[(8 + v) * nb + me] += pvp[v];
        if (P.viscous) R.D(D_E0 + v, me) += E[v];
      }
    }
  }
  section_boundary();
  // Prandtl-number fix on the complete flux: energy flux += (1/Pr - 1) q, q
  // the heat flux relative to the velocity of g0 (interface frame), from the
  // complete <psi f>; then the stores (global components)
  double Fl[4], Pm[4], Pp[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    Fl[v] = acc[v * nb + me];
    Pm[v] = acc[(4 + v) * nb + me];
    Pp[v] = acc[(8 + v) * nb + me];
  }
  if (P.viscous && R.D(D_RHO0, me) > 0.0) {
    const double U0 = R.D(D_U0, me), V0 = R.D(D_V0, me), k2 = 0.5 * (U0 * U0 + V0 * V0);
    double Ed[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Ed[v] = R.D(D_E0 + v, me);
    const double qh = Fl[3] - U0 * Fl[1] - V0 * Fl[2] + k2 * Fl[0] - U0 * (Ed[3] - U0 * Ed[1] - V0 * Ed[2] + k2 * Ed[0]);
    Fl[3] += P.prfix * qh;
  }
  if constexpr (kCurv) {
    // frame momentum back to (x, y); the grid's own interface layouts
    double fr[kFaceGeo];
    face_geo(g, F, fr);
    const double f1 = Fl[1], f2 = Fl[2], m1 = Pm[1], m2 = Pm[2], q1 = Pp[1], q2 = Pp[2];
    Fl[1] = fr[0] * f1 + fr[2] * f2;
    Fl[2] = fr[1] * f1 + fr[3] * f2;
    Pm[1] = fr[0] * m1 + fr[2] * m2;
    Pm[2] = fr[1] * m1 + fr[3] * m2;
    Pp[1] = fr[0] * q1 + fr[2] * q2;
    Pp[2] = fr[1] * q1 + fr[3] * q2;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (F.isx) {
        g.FLX[x.flx(v, F.a, F.b)] = Fl[v];
        g.FX[x.fx(0, v, F.a, F.b)] = (TS)Pm[v];
        g.FX[x.fx(1, v, F.a, F.b)] = (TS)Pp[v];
      } else {
        g.FLY[x.fly(v, F.a, F.b)] = Fl[v];
        g.FY[x.fy(0, v, F.a, F.b)] = (TS)Pm[v];
        g.FY[x.fy(1, v, F.a, F.b)] = (TS)Pp[v];
      }
    }
    return;
  }
  if (F.isx) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int vl = loc(true, v);
      g.FLX[x.flx(v, F.a, F.b)] = Fl[vl];
      g.FX[x.fx(0, v, F.a, F.b)] = (TS)Pm[vl];
      g.FX[x.fx(1, v, F.a, F.b)] = (TS)Pp[vl];
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int vl = loc(false, v);
      g.FLY[x.fly(v, F.a, F.b)] = Fl[vl];
      g.FY[x.fy(0, v, F.a, F.b)] = (TS)Pm[vl];
      g.FY[x.fy(1, v, F.a, F.b)] = (TS)Pp[vl];
    }
  }
}

// one logical block per block (NB threads)
template <typename TS, typename TP, typename TC, bool kCurv, unsigned NB>
__global__ void __launch_bounds__(256) k_iface_2d(KA<Prob<TS, TP, TC>> a) {
  extern __shared__ __align__(16) unsigned char lds[];
  iface_2d_block<TS, TP, TC, kCurv, NB>(a, logical_block(a.nblk), lds);
}

// persistent form: gridDim.x (a multiple of 8) blocks take the logical
// blocks in turn
template <typename TS, typename TP, typename TC, bool kCurv, unsigned NB>
__global__ void __launch_bounds__(256) k_iface_2d_loop(KA<Prob<TS, TP, TC>> a) {
  extern __shared__ __align__(16) unsigned char lds[];
  for (unsigned b = blockIdx.x; b < a.nblk; b += gridDim.x)
    iface_2d_block<TS, TP, TC, kCurv, NB>(a, logical_of(b, a.nblk), lds);
}

// the interface launch of a 2D group with blocks of NB threads
template <typename TS, typename TP, typename TC, bool kCurv, unsigned NB>
void launch_iface_2d(const KA<Prob<TS, TP, TC>>& A, unsigned face_grid, hipStream_t st) {
  const size_t lds = NB * iface_lds_per_thread<TC>();
  if (face_grid)
    k_iface_2d_loop<TS, TP, TC, kCurv, NB><<<face_grid, NB, lds, st>>>(A);
  else
    k_iface_2d<TS, TP, TC, kCurv, NB><<<A.nblk, NB, lds, st>>>(A);
}

// block sizes 64, 128, 256 (gks_set_launch and the tuner allow no others)
template <typename TS, typename TP, typename TC, bool kCurv>
void launch_iface_2d(const KA<Prob<TS, TP, TC>>& A, int bs, unsigned face_grid, hipStream_t st) {
  if (bs == 64)
    launch_iface_2d<TS, TP, TC, kCurv, 64>(A, face_grid, st);
  else if (bs == 128)
    launch_iface_2d<TS, TP, TC, kCurv, 128>(A, face_grid, st);
  else
    launch_iface_2d<TS, TP, TC, kCurv, 256>(A, face_grid, st);
}

// 1D interfaces 0..nx, fused
template <typename TS, typename TP, typename TC>
__global__ void __launch_bounds__(256) k_face_1d(KA<Prob<TS, TP, TC>> a) {
  int id;
  const Prob<TS, TP, TC>& Q = locate(a, KK_FACE, id);
  const Grid<TS, TP> g = Q.g;
  const int nx = g.ix.nx;
  if (id > nx) return;
  const double dt = *g.dt;
  if (!(dt > 0.0)) return;
  const Phys P = Q.P;
  const Idx& x = g.ix;
  const int fi = id;
  double Wc[2][3], pc[2][3][2], flux[3], pv[3];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      Wc[s][v] = g.W[x.w1(v, fi - 1 + s)];
      pc[s][v][0] = (double)g.PC[x.pc1(v, 0, fi - 1 + s)];
      pc[s][v][1] = (double)g.PC[x.pc1(v, 1, fi - 1 + s)];
    }
  if (!iface_1d<TC>(P, dt, g.geo.h, Wc, pc, flux, pv)) {
    atomicCAS(g.err, 0ull, 1ull + (1ull << 32) + (unsigned long long)(fi + 1));
#pragma unroll
    for (int v = 0; v < 3; ++v) flux[v] = pv[v] = 0.0;
  }
  // a slip wall at the domain's end: the symmetry line of its image pair
  // (momentum flux only, a new point value at rest)
  if ((fi == 0 || fi == nx) && Q.bc[fi == 0 ? 0 : 1].kind == GKS_BC_REFLECT) {
    flux[0] = flux[2] = 0.0;
    pv[1] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    g.FLX[x.fl1(v, fi)] = flux[v];
    g.FX[x.f1(v, fi)] = (TS)pv[v];
  }
}

// ---------------------------------------------------------------------------
// conservative update (kScan: only the CFL bound of the present state)
// ---------------------------------------------------------------------------

// Domain-edge walls, applied here to the wall interfaces' fluxes and point
// values (each such interface has one gas cell, whose update alone reads
// it).  A no-slip wall is impermeable: its interface passes no mass, and the
// mass flux F_rho of the ghost-image evaluation takes with it the momentum
// and energy it would carry at the velocity and total enthalpy of the cell
// beside the wall (its average at the start of the step); pressure, viscous
// stress and heat flux stay.  A slip wall is the symmetry line of its image
// pair: normal momentum flux only, and new point values without normal
// momentum (the ghost cell's own reconstruction holds the wall's point
// values unmirrored, so an odd part left there by rounding would not cancel
// and can grow from step to step).
//
// wall_kind: 1 slip, 2 no-slip, 0 neither for side `side` at column or row
// `pos` (the south edge of the double Mach reflection is a slip wall from
// the cell whose centre lies at x = 1/6 on)
template <class PR>
__device__ __forceinline__ int wall_kind(const PR& Q, int side, int pos) {
  const int k = Q.bc[side].kind;
  if (k == GKS_BC_NOSLIP_ISOTHERMAL || k == GKS_BC_NOSLIP_ADIABATIC) return 2;
  if (k == GKS_BC_REFLECT) return 1;
  if (k == GKS_BC_DMR_BOTTOM) return Q.g.geo.x0 + (pos + 0.5) * Q.g.geo.h < 1.0 / 6.0 ? 0 : 1;
  return 0;
}

// the wall treatment of interface flux F (grid components, in place) beside
// the cell of average W; axis: the interface's normal
__device__ __forceinline__ void wall_flux(int kind, int axis, const double* W, double gamma, double* F) {
  if (kind == 2) {
    const double rho = W[0], u = W[1] / rho, v = W[2] / rho;
    const double p = (gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / rho);
    const double h = (W[3] + p) / rho, m = F[0];
    F[1] -= m * u;
    F[2] -= m * v;
    F[3] -= m * h;
    F[0] = 0.0;
  } else {
    F[0] = 0.0;
    F[2 - axis] = 0.0;
    F[3] = 0.0;
  }
}

template <typename TS, typename TP, typename TC, bool kScan>
__global__ void __launch_bounds__(256) k_update_2d(KA<Prob<TS, TP, TC>> a) {
  int id;
  const Prob<TS, TP, TC>& Q = locate(a, KK_CELL, id);
  const Grid<TS, TP> g = Q.g;
  const int nx = g.ix.nx, ny = g.ix.ny;
  double bound = 1e300;
  if (id < nx * ny && !Q.solid(id % nx, id / nx)) {
    const int j = id / nx, i = id % nx;
    const Idx& x = g.ix;
    double W[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) W[v] = g.W[x.w(v, j, i)];
    const double dt = kScan ? 0.0 : *g.dt;
    if (!kScan) {
      // every load is issued before the step is tested: none waits for it
      // periodic seams: the last interface is the first one
      const int ie = (i + 1 == nx && x.fxr == nx) ? 0 : i + 1;
      const int je = (j + 1 == ny && x.fyr == ny) ? 0 : j + 1;
      double f[4][4];  // west, east, south, north interface fluxes
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        f[0][v] = g.FLX[x.flx(v, j, i)];
        f[1][v] = g.FLX[x.flx(v, j, ie)];
        f[2][v] = g.FLY[x.fly(v, j, i)];
        f[3][v] = g.FLY[x.fly(v, je, i)];
      }
      // the seam gets the first interface's new point values (read by the
      // next reconstruction)
      const bool sx = i == 0 && x.fxr == nx, sy = j == 0 && x.fyr == ny;
      TS px[8], py[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        px[q] = sx ? g.FX[x.fx(q >> 2, q & 3, j, 0)] : TS(0);
        py[q] = sy ? g.FY[x.fy(q >> 2, q & 3, 0, i)] : TS(0);
      }
      const double t0 = id == 0 ? *g.t : 0.0;
      const long long n0 = id == 0 ? *g.steps : 0;
      if (dt > 0.0 && (i == 0 || i + 1 == nx || j == 0 || j + 1 == ny)) {
        // the walls among the cell's interfaces
#pragma unroll
        for (int side = 0; side < 4; ++side) {
          const bool on = side == 0 ? i == 0 : side == 1 ? i + 1 == nx : side == 2 ? j == 0 : j + 1 == ny;
          const int kind = on ? wall_kind(Q, side, side < 2 ? j : i) : 0;
          if (!kind) continue;
          wall_flux(kind, side >> 1, W, Q.P.gamma, f[side]);
          if (kind == 1) {
#pragma unroll
            for (int gp = 0; gp < 2; ++gp) {
              if (side < 2)
                g.FX[x.fx(gp, 1, j, side == 0 ? 0 : nx)] = TS(0);
              else
                g.FY[x.fy(gp, 2, side == 2 ? 0 : ny, i)] = TS(0);
            }
          }
        }
      }
      double d[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) d[v] = f[0][v] - f[1][v] + f[2][v] - f[3][v];
      if (dt > 0.0) {
        const double ia = 1.0 / (g.cv.area ? g.cv.area[(size_t)(j + 1) * (nx + 2) + (i + 1)] : g.geo.h * g.geo.k);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          W[v] += d[v] * ia;
          g.W[x.w(v, j, i)] = W[v];
        }
        if (sx)
#pragma unroll
          for (int q = 0; q < 8; ++q) g.FX[x.fx(q >> 2, q & 3, j, nx)] = px[q];
        if (sy)
#pragma unroll
          for (int q = 0; q < 8; ++q) g.FY[x.fy(q >> 2, q & 3, ny, i)] = py[q];
        if (id == 0) {
          *g.t = t0 + dt;
          *g.steps = n0 + 1;
        }
      }
    }
    // (the scan checks the state it is given: a caller's initial state)
    if (kScan || dt > 0.0) {
      const double p = (Q.P.gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0]);
      if (!(W[0] > 0.0) || !(p > 0.0) || !isfinite(p))
        atomicCAS(g.err, 0ull,
                  1ull + ((unsigned long long)(j + 1) << 32) + (unsigned long long)(i + 1) + (1ull << 63));
    }
    bound = g.cv.wid ? cell_dt_bound_curv(W, Q.P, g.cv.wid[id], g.cv.wid[(size_t)nx * ny + id])
                     : cell_dt_bound(W, Q.P, g.geo.h, g.geo.k);
  }
  reduce_dt_bound(bound, g.dtmin, (unsigned)id >> 6, g.dtmask);
}

template <typename TS, typename TP, typename TC, bool kScan>
__global__ void __launch_bounds__(256) k_update_1d(KA<Prob<TS, TP, TC>> a) {
  int id;
  const Prob<TS, TP, TC>& Q = locate(a, KK_CELL, id);
  const Grid<TS, TP> g = Q.g;
  const int nx = g.ix.nx;
  double bound = 1e300;
  if (id < nx) {
    const int i = id;
    const Idx& x = g.ix;
    double W[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) W[v] = g.W[x.w1(v, i)];
    const double dt = kScan ? 0.0 : *g.dt;
    if (dt > 0.0) {
      const double ih = 1.0 / g.geo.h;
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        W[v] += (g.FLX[x.fl1(v, i)] - g.FLX[x.fl1(v, i + 1)]) * ih;
        g.W[x.w1(v, i)] = W[v];
      }
      if (id == 0) {
        *g.t += dt;
        *g.steps += 1;
      }
    }
    if (kScan || dt > 0.0) {
      const double p = (Q.P.gamma - 1.0) * (W[2] - 0.5 * W[1] * W[1] / W[0]);
      if (!(W[0] > 0.0) || !(p > 0.0) || !isfinite(p))
        atomicCAS(g.err, 0ull, 1ull + (1ull << 32) + (unsigned long long)(i + 1) + (1ull << 63));
    }
    bound = cell_dt_bound_1d(W, Q.P, g.geo.h);
  }
  reduce_dt_bound(bound, g.dtmin, (unsigned)id >> 6, g.dtmask);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct Problem;
size_t cells_of(const Problem& p);

struct Problem {
  gks_problem spec;
  Phys phys;
  BCDev bc[4];
  Idx ix;
  Geo geo;
  bool mixed;
  void* W = nullptr;
  void* FX = nullptr;
  void* FY = nullptr;
  void* PC = nullptr;
  void* FLX = nullptr;
  void* FLY = nullptr;
  void* scal = nullptr;  // t, dt, steps, err, fallbacks, CFL slots (scal_bytes of the cells)
  bool borrowed = false;  // W, FX, FY belong to the caller (gks_init_device)
  void* geom = nullptr;   // curvilinear grids: CurvDev arrays (one allocation)
};

// problems of one dimension and precision, advanced by one launch sequence
struct Group {
  int dim = 2;
  bool mixed = false;
  bool chr = false;   // 2D reconstruction in characteristic variables
  bool curv = false;  // curvilinear grids
  std::vector<int> members;
  void* dprobs = nullptr;                  // device Prob<...>[members]
  uint32_t* owner[KK_COUNT] = {};          // device block-owner tables
  unsigned nblk[KK_COUNT] = {};
  unsigned cap[KK_COUNT] = {};             // allocated owner entries
  int bs[KK_COUNT] = {256, 256, 256, 256, 64};  // block size of each kind
  unsigned face_grid = 0;  // 2D interfaces: 0 one block per logical block, else a persistent grid of this many
  int recon_rows = 0;      // 2D reconstruction: 0 row order, else LDS tiles of (block / rows) x rows cells
  double* ctl = nullptr;                   // device [members][2]: fixed step, end time
  std::vector<double> ctl_host;            // values last uploaded
};

}  // namespace

struct gks_handle {
  std::vector<Problem> probs;
  std::vector<Group> groups;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int sticky = GKS_OK;
  std::string msg;
  int profiling = 0;
  double ktime[GKS_K_COUNT] = {0};
  long long klaunch[GKS_K_COUNT] = {0};
  std::vector<hipEvent_t> pend_a, pend_b;
  std::vector<int> pend_k;
};

namespace {

constexpr int kMaxProblems = 65535;  // block-owner tables hold 16-bit problem indices

thread_local std::string g_init_msg;  // message of the last failed gks_init on this thread

int fail(gks_handle* h, int code, const std::string& m) {
  if (h) h->msg = m;
  return code;
}

#define HIP_OR(h, call)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      if (h) h->sticky = GKS_EDEVICE;                                                       \
      return fail(h, GKS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));       \
    }                                                                                       \
  } while (0)

double internal_dof(int dim, double gamma) {
  return dim == 2 ? (4.0 - 2.0 * gamma) / (gamma - 1.0) : (3.0 - gamma) / (gamma - 1.0);
}

void cons_of(int dim, double gamma, const double* q, double* W) {
  W[0] = q[0];
  W[1] = q[0] * q[1];
  if (dim == 2) {
    W[2] = q[0] * q[2];
    W[3] = q[3] / (gamma - 1.0) + 0.5 * q[0] * (q[1] * q[1] + q[2] * q[2]);
  } else {
    W[2] = q[3] / (gamma - 1.0) + 0.5 * q[0] * q[1] * q[1];
    W[3] = 0.0;
  }
}

std::string validate(const gks_problem& p) {
  if (p.dim != 1 && p.dim != 2) return "dim must be 1 or 2";
  if (p.dim == 2 && (p.nx < 2 || p.ny < 2)) return "nx, ny must be >= 2";
  if (p.dim == 1 && (p.nx < 2 || p.ny != 1)) return "1D: nx >= 2 and ny == 1 required";
  if ((long long)(p.nx + 4) * (p.ny + 4) > (1ll << 28)) return "grid too large";
  if (!(p.x1 > p.x0) || (p.dim == 2 && !(p.y1 > p.y0))) return "empty domain";
  if (!(p.gamma > 1.0) || !(p.gamma < 3.0)) return "gamma must lie in (1, 3)";
  if (!(internal_dof(p.dim, p.gamma) >= 0.0)) return "gamma gives negative internal degrees of freedom";
  if (p.viscous && !(p.mu >= 0.0 && p.prandtl > 0.0)) return "mu >= 0 and prandtl > 0 required";
  if (!(p.cfl > 0.0) || !(p.weno_eps > 0.0) || !(p.weno_c >= 0.0)) return "cfl, weno_eps must be > 0";
  if (!(p.tau_eps >= 0.0) || !(p.tau_c >= 0.0)) return "tau constants must be >= 0";
  if (!std::isfinite(p.t0)) return "t0 must be finite";
  if (p.recon_vars != 0 && p.recon_vars != 1) return "recon_vars must be 0 or 1";
  if (p.admissibility != 0 && p.admissibility != 1) return "admissibility must be 0 or 1";
  if (p.obstacle_nj != 0) {
    auto mirrors = [](int k) {
      return k == GKS_BC_OUTFLOW || k == GKS_BC_REFLECT || k == GKS_BC_NOSLIP_ISOTHERMAL ||
             k == GKS_BC_NOSLIP_ADIABATIC;
    };
    if (p.dim != 2) return "a solid step needs dim 2";
    if (p.obstacle_i0 < 2 || p.obstacle_i0 > p.nx - 4) return "step: obstacle_i0 must lie in [2, nx - 4]";
    if (p.obstacle_nj < 4 || p.obstacle_nj > p.ny - 3) return "step: obstacle_nj must lie in [4, ny - 3]";
    if (!mirrors(p.bc[1].kind) || !mirrors(p.bc[2].kind))
      return "step: the east and south boundaries must be mirror kinds (outflow, reflect, no-slip)";
  }
  if (p.precision != GKS_FP64 && p.precision != GKS_FP32_MIXED) return "unknown precision";
  if (p.mesh) {
    if (p.dim != 2) return "a curvilinear grid needs dim 2";
    if (p.obstacle_nj != 0) return "a curvilinear grid takes no solid step";
    if (p.recon_vars != 0) return "a curvilinear grid reconstructs in conservative variables (recon_vars 0)";
    for (int s = 0; s < 4; ++s) {
      const int k = p.bc[s].kind;
      if (k != GKS_BC_PERIODIC && k != GKS_BC_OUTFLOW && k != GKS_BC_NOSLIP_ISOTHERMAL && k != GKS_BC_NOSLIP_ADIABATIC &&
          k != GKS_BC_INFLOW)
        return "curvilinear grid: boundaries must be periodic, outflow, no-slip or inflow";
    }
  }
  for (int s = 0; s < (p.dim == 2 ? 4 : 2); ++s) {
    const double w = p.bc[s].wall_omega;
    if (!std::isfinite(w)) return "wall_omega must be finite";
    if (w != 0.0 && (!p.mesh || (p.bc[s].kind != GKS_BC_NOSLIP_ISOTHERMAL && p.bc[s].kind != GKS_BC_NOSLIP_ADIABATIC)))
      return "wall_omega is for the no-slip walls of a curvilinear grid";
  }
  const int nsides = p.dim == 2 ? 4 : 2;
  for (int s = 0; s < nsides; ++s) {
    const int k = p.bc[s].kind;
    if (k < GKS_BC_PERIODIC || k > GKS_BC_DMR_TOP) return "unknown boundary kind";
    if ((k == GKS_BC_PERIODIC) != (p.bc[s ^ 1].kind == GKS_BC_PERIODIC)) return "periodic sides must pair";
    if (k == GKS_BC_DMR_BOTTOM && s != 2) return "dmr_bottom only on the south side";
    if (k == GKS_BC_DMR_TOP && s != 3) return "dmr_top only on the north side";
  }
  return "";
}

// host description of a validated problem (no buffers)
void setup_problem(const gks_problem& s, Problem& p) {
  p.spec = s;
  p.mixed = s.precision == GKS_FP32_MIXED;
  {
    const int ny = s.dim == 2 ? s.ny : 1;
    const bool px = s.dim == 2 && s.bc[0].kind == GKS_BC_PERIODIC;
    const bool py = s.dim == 2 && s.bc[2].kind == GKS_BC_PERIODIC;
    p.ix = Idx{s.nx, ny, px ? s.nx : s.nx + 1, py ? ny : ny + 1};
  }
  p.geo = Geo{s.x0, s.y0, (s.x1 - s.x0) / s.nx, s.dim == 2 ? (s.y1 - s.y0) / s.ny : 1.0};
  if (s.mesh) p.geo = Geo{0.0, 0.0, 1.0, 1.0};  // logical coordinates
  Phys& P = p.phys;
  memset(&P, 0, sizeof(P));
  P.gamma = s.gamma;
  P.K = internal_dof(s.dim, s.gamma);
  P.nth = P.K + (s.dim == 2 ? 2.0 : 1.0);
  P.kp[0] = 1.0;
  for (int e = 1; e < 4; ++e) P.kp[e] = P.kp[e - 1] * (P.K + 2.0 * (e - 1));
  P.tau_eps = s.tau_eps;
  P.tau_c = s.tau_c;
  P.mu = s.viscous ? s.mu : 0.0;
  P.prfix = s.viscous ? 1.0 / s.prandtl - 1.0 : 0.0;
  P.weno_eps = s.weno_eps;
  P.weno_c = s.weno_c;
  P.cfl = s.cfl;
  P.viscous = s.viscous ? 1 : 0;
  for (int side = 0; side < 4; ++side) {
    BCDev& b = p.bc[side];
    memset(&b, 0, sizeof(b));
    b.kind = s.bc[side].kind;
    cons_of(s.dim, s.gamma, s.bc[side].state, b.state);
    cons_of(s.dim, s.gamma, s.bc[side].alt, b.alt);
    b.wu = s.bc[side].wall_u;
    b.wv = s.bc[side].wall_v;
    b.wT = s.bc[side].wall_T;
    b.wo = s.bc[side].wall_omega;
  }
}

// Geometry of a curvilinear grid (the CurvDev arrays, concatenated): every
// interface's frame and metric, the cell areas (edge ghosts: their image's),
// the widths of the CFL condition and the boundary vertices.  "" or the
// reason the grid is refused (a cell of nonpositive area, a centre on the
// wrong side of an interface, periodic edges that are not one translation
// apart, a non-finite coordinate).
std::string curvilinear_geometry(const gks_problem& s, std::vector<double>& out) {
  const int nx = s.nx, ny = s.ny;
  auto V = [&](int j, int i, int c) { return s.mesh[((size_t)j * (nx + 1) + i) * 2 + c]; };
  for (size_t q = 0; q < (size_t)(nx + 1) * (ny + 1) * 2; ++q)
    if (!std::isfinite(s.mesh[q])) return "mesh: non-finite coordinate";
  const size_t nfx = (size_t)ny * (nx + 1), nfy = (size_t)(ny + 1) * nx, nc = (size_t)nx * ny;
  const size_t o_fy = kFaceGeo * nfx, o_area = o_fy + kFaceGeo * nfy, o_wid = o_area + (size_t)(nx + 2) * (ny + 2),
               o_bnd = o_wid + 2 * nc;
  out.assign(o_bnd + 4 * (size_t)(ny + 1) + 4 * (size_t)(nx + 1), 0.0);
  std::vector<double> cx(nc), cy(nc), ar(nc);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t c = (size_t)j * nx + i;
      const double x0 = V(j, i, 0), y0 = V(j, i, 1), x1 = V(j, i + 1, 0), y1 = V(j, i + 1, 1);
      const double x2 = V(j + 1, i + 1, 0), y2 = V(j + 1, i + 1, 1), x3 = V(j + 1, i, 0), y3 = V(j + 1, i, 1);
      cx[c] = 0.25 * (x0 + x1 + x2 + x3);
      cy[c] = 0.25 * (y0 + y1 + y2 + y3);
      ar[c] = 0.5 * ((x2 - x0) * (y3 - y1) - (y2 - y0) * (x3 - x1));
      if (!(ar[c] > 0.0)) return "mesh: cell (" + std::to_string(i) + ", " + std::to_string(j) + ") has no positive area";
    }
  // periodic edges: one translation apart
  double per[2][2] = {{V(0, nx, 0) - V(0, 0, 0), V(0, nx, 1) - V(0, 0, 1)},
                      {V(ny, 0, 0) - V(0, 0, 0), V(ny, 0, 1) - V(0, 0, 1)}};
  double ext = 0.0;
  for (size_t q = 0; q < (size_t)(nx + 1) * (ny + 1) * 2; ++q) ext = std::max(ext, std::fabs(s.mesh[q]));
  if (s.bc[0].kind == GKS_BC_PERIODIC)
    for (int j = 0; j <= ny; ++j)
      if (std::fabs(V(j, nx, 0) - V(j, 0, 0) - per[0][0]) > 1e-12 * ext ||
          std::fabs(V(j, nx, 1) - V(j, 0, 1) - per[0][1]) > 1e-12 * ext)
        return "mesh: the periodic west and east edges are not one translation apart";
  if (s.bc[2].kind == GKS_BC_PERIODIC)
    for (int i = 0; i <= nx; ++i)
      if (std::fabs(V(ny, i, 0) - V(0, i, 0) - per[1][0]) > 1e-12 * ext ||
          std::fabs(V(ny, i, 1) - V(0, i, 1) - per[1][1]) > 1e-12 * ext)
        return "mesh: the periodic south and north edges are not one translation apart";
  // one interface: edge a -> b, cell centres c0 (lower index) and c1; the
  // normal is the tangent turned clockwise (x interfaces) or anticlockwise
  auto frame = [&](double* dst, size_t plane, size_t o, double ax, double ay, double bx, double by, bool xface,
                   double c0x, double c0y, double c1x, double c1y) -> bool {
    const double ex = bx - ax, ey = by - ay, L = std::sqrt(ex * ex + ey * ey);
    const double tx = ex / L, ty = ey / L, nxv = xface ? ty : -ty, nyv = xface ? -tx : tx;
    const double dx = c1x - c0x, dy = c1y - c0y, an = dx * nxv + dy * nyv, at = dx * tx + dy * ty;
    if (!(L > 0.0) || !(an > 0.0)) return false;
    const double f[kFaceGeo] = {nxv, nyv, tx, ty, L, 1.0 / an, -at / (an * L)};
    for (int q = 0; q < kFaceGeo; ++q) dst[q * plane + o] = f[q];
    return true;
  };
  // centre of the cell across a boundary interface: the periodic partner
  // translated, else the mirror image of the inside centre (ix, iy) across
  // the edge (a -> b)
  auto across = [&](bool periodic, int pc, double sx, double sy, double ix, double iy, double ax, double ay, double bx,
                    double by, double& ox, double& oy) {
    if (periodic) {
      ox = cx[pc] + sx;
      oy = cy[pc] + sy;
      return;
    }
    const double ex = bx - ax, ey = by - ay, L = std::sqrt(ex * ex + ey * ey), nxv = -ey / L, nyv = ex / L;
    const double d = (ix - ax) * nxv + (iy - ay) * nyv;
    ox = ix - 2.0 * d * nxv;
    oy = iy - 2.0 * d * nyv;
  };
  for (int j = 0; j < ny; ++j)
    for (int fi = 0; fi <= nx; ++fi) {
      const double ax = V(j, fi, 0), ay = V(j, fi, 1), bx = V(j + 1, fi, 0), by = V(j + 1, fi, 1);
      double c0x, c0y, c1x, c1y;
      const bool pw = s.bc[0].kind == GKS_BC_PERIODIC, pe = s.bc[1].kind == GKS_BC_PERIODIC;
      if (fi > 0) {
        c0x = cx[(size_t)j * nx + fi - 1];
        c0y = cy[(size_t)j * nx + fi - 1];
      } else {
        across(pw, j * nx + nx - 1, -per[0][0], -per[0][1], cx[(size_t)j * nx], cy[(size_t)j * nx], ax, ay, bx, by, c0x,
               c0y);
      }
      if (fi < nx) {
        c1x = cx[(size_t)j * nx + fi];
        c1y = cy[(size_t)j * nx + fi];
      } else {
        across(pe, j * nx, per[0][0], per[0][1], cx[(size_t)j * nx + nx - 1], cy[(size_t)j * nx + nx - 1], ax, ay, bx,
               by, c1x, c1y);
      }
      if (!frame(out.data(), nfx, (size_t)j * (nx + 1) + fi, ax, ay, bx, by, true, c0x, c0y, c1x, c1y))
        return "mesh: x interface (" + std::to_string(fi) + ", " + std::to_string(j) + ") has its cells on one side";
    }
  for (int fj = 0; fj <= ny; ++fj)
    for (int i = 0; i < nx; ++i) {
      const double ax = V(fj, i, 0), ay = V(fj, i, 1), bx = V(fj, i + 1, 0), by = V(fj, i + 1, 1);
      double c0x, c0y, c1x, c1y;
      const bool ps = s.bc[2].kind == GKS_BC_PERIODIC, pn = s.bc[3].kind == GKS_BC_PERIODIC;
      if (fj > 0) {
        c0x = cx[(size_t)(fj - 1) * nx + i];
        c0y = cy[(size_t)(fj - 1) * nx + i];
      } else {
        across(ps, (ny - 1) * nx + i, -per[1][0], -per[1][1], cx[i], cy[i], ax, ay, bx, by, c0x, c0y);
      }
      if (fj < ny) {
        c1x = cx[(size_t)fj * nx + i];
        c1y = cy[(size_t)fj * nx + i];
      } else {
        across(pn, i, per[1][0], per[1][1], cx[(size_t)(ny - 1) * nx + i], cy[(size_t)(ny - 1) * nx + i], ax, ay, bx,
               by, c1x, c1y);
      }
      if (!frame(out.data() + o_fy, nfy, (size_t)fj * nx + i, ax, ay, bx, by, false, c0x, c0y, c1x, c1y))
        return "mesh: y interface (" + std::to_string(i) + ", " + std::to_string(fj) + ") has its cells on one side";
    }
  // areas over cells -1..nx x -1..ny: an edge ghost takes its image's
  auto image = [](int q, int n, bool plo, bool phi) {
    if (q < 0) return plo ? q + n : -1 - q;
    if (q >= n) return phi ? q - n : 2 * n - 1 - q;
    return q;
  };
  for (int j = -1; j <= ny; ++j)
    for (int i = -1; i <= nx; ++i) {
      if ((i < 0 || i >= nx) && (j < 0 || j >= ny)) continue;
      const int ii = image(i, nx, s.bc[0].kind == GKS_BC_PERIODIC, s.bc[1].kind == GKS_BC_PERIODIC);
      const int jj = image(j, ny, s.bc[2].kind == GKS_BC_PERIODIC, s.bc[3].kind == GKS_BC_PERIODIC);
      out[o_area + (size_t)(j + 1) * (nx + 2) + (i + 1)] = ar[(size_t)jj * nx + ii];
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t c = (size_t)j * nx + i;
      const double lw = out[4 * nfx + (size_t)j * (nx + 1) + i], le = out[4 * nfx + (size_t)j * (nx + 1) + i + 1];
      const double ls = out[o_fy + 4 * nfy + (size_t)j * nx + i], ln = out[o_fy + 4 * nfy + (size_t)(j + 1) * nx + i];
      out[o_wid + c] = ar[c] / (0.5 * (lw + le));
      out[o_wid + nc + c] = ar[c] / (0.5 * (ls + ln));
    }
  double* b = out.data() + o_bnd;
  for (int j = 0; j <= ny; ++j)
    for (int c = 0; c < 2; ++c) {
      b[2 * j + c] = V(j, 0, c);
      b[2 * (ny + 1) + 2 * j + c] = V(j, nx, c);
    }
  for (int i = 0; i <= nx; ++i)
    for (int c = 0; c < 2; ++c) {
      b[4 * (ny + 1) + 2 * i + c] = V(0, i, c);
      b[4 * (ny + 1) + 2 * (nx + 1) + 2 * i + c] = V(ny, i, c);
    }
  return "";
}

// device CurvDev pointers into the geometry allocation of problem p
CurvDev curv_pointers(const Problem& p) {
  CurvDev c{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (!p.geom) return c;
  const size_t nx = p.ix.nx, ny = p.ix.ny;
  const double* g = (const double*)p.geom;
  c.fx = g;
  c.fy = c.fx + kFaceGeo * ny * (nx + 1);
  c.area = c.fy + kFaceGeo * (ny + 1) * nx;
  c.wid = c.area + (nx + 2) * (ny + 2);
  c.bnd = c.wid + 2 * nx * ny;
  return c;
}

size_t cells_of(const Problem& p) { return p.spec.dim == 2 ? (size_t)p.ix.nx * p.ix.ny : (size_t)p.ix.nx; }

size_t n_interfaces(const Idx& x) { return (size_t)x.fxr * x.ny + (size_t)x.nx * x.fyr; }

// bytes of the buffers W, FX, FY, PC, FLX, FLY, scal of a problem
constexpr int kBufs = 7;
void buffer_sizes(const Problem& p, size_t (&sizes)[kBufs]) {
  const size_t ts = p.mixed ? sizeof(float) : sizeof(double);
  const Idx& x = p.ix;
  const size_t nx = x.nx, ny = x.ny;
  if (p.spec.dim == 2) {
    const size_t sz[kBufs] = {4 * (ny + 4) * (nx + 4) * 8,      2 * 4 * (ny + 2) * (nx + 3) * ts,
                              2 * 4 * (ny + 3) * (nx + 2) * ts, 4 * 5 * (ny + 2) * (nx + 2) * ts,
                              4 * ny * (nx + 1) * 8,            4 * (ny + 1) * nx * 8,
                              scal_bytes(cells_of(p))};
    memcpy(sizes, sz, sizeof(sz));
  } else {
    const size_t sz[kBufs] = {3 * (nx + 4) * 8, 3 * (nx + 3) * ts, 0, 3 * 2 * (nx + 2) * ts, 3 * (nx + 1) * 8, 0,
                              scal_bytes(cells_of(p))};
    memcpy(sizes, sz, sizeof(sz));
  }
}

// a caller's buffer must be device memory of the current device with at
// least `bytes` left in its allocation from p (else "" is not returned)
std::string check_device_buffer(const char* name, const void* p, size_t bytes) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return std::string(name) + " is not device memory";
  }
  if (a.type != hipMemoryTypeDevice) return std::string(name) + " is not device memory";
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || a.device != dev)
    return std::string(name) + " is not memory of the current device";
  void* base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (void*)p) != hipSuccess) {
    (void)hipGetLastError();
    return std::string(name) + ": allocation range unknown";
  }
  if ((const char*)p < (const char*)base || (size_t)((const char*)p - (const char*)base) + bytes > size)
    return std::string(name) + " is smaller than the state extent (gks_state_extent)";
  return "";
}

// element counts of the ghosted state arrays W, FX, FY of a validated problem
void state_elems(const gks_problem& s, size_t e[3]) {
  const size_t nx = s.nx, ny = s.dim == 2 ? s.ny : 1;
  if (s.dim == 2) {
    e[0] = 4 * (ny + 4) * (nx + 4);
    e[1] = 2 * 4 * (ny + 2) * (nx + 3);
    e[2] = 2 * 4 * (ny + 3) * (nx + 2);
  } else {
    e[0] = 3 * (nx + 4);
    e[1] = 3 * (nx + 3);
    e[2] = 0;
  }
}

unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// threads of one problem in a launch of kind k (recon_rows > 0: the tiled
// reconstruction with blocks of bs threads, whole tiles)
size_t work_items(const Problem& p, int dim, int k, int recon_rows = 0, int bs = 256) {
  const size_t nx = p.ix.nx, ny = p.ix.ny;
  if (dim == 2) {
    switch (k) {
      case KK_GA: return 4 * ny + 4 * ny + 4 * (ny + 1) + 4 * (nx + 4) + 4 * nx + 4 * (nx + 1);
      case KK_RECON:
        if (recon_rows > 0) {
          const size_t tx = (size_t)bs / recon_rows;
          return ((nx + 2 + tx - 1) / tx) * ((ny + 2 + recon_rows - 1) / recon_rows) * (size_t)bs;
        }
        return (nx + 2) * (ny + 2);
      case KK_FACE: return n_interfaces(p.ix);
      case KK_OBST: return p.spec.obstacle_nj > 0 ? step_items((int)nx, p.spec.obstacle_i0, p.spec.obstacle_nj) : 0;
      default: return nx * ny;
    }
  }
  switch (k) {
    case KK_GA: return 6;
    case KK_RECON: return nx + 2;
    case KK_FACE: return nx + 1;
    case KK_OBST: return 0;
    default: return nx;
  }
}

template <typename TS, typename TP>
Grid<TS, TP> grid_of(Problem& p) {
  Grid<TS, TP> g;
  g.ix = p.ix;
  g.geo = p.geo;
  g.cv = curv_pointers(p);
  g.W = (double*)p.W;
  g.FX = (TS*)p.FX;
  g.FY = (TS*)p.FY;
  g.PC = (TP*)p.PC;
  g.FLX = (double*)p.FLX;
  g.FLY = (double*)p.FLY;
  double* s = (double*)p.scal;
  g.t = s;
  g.dt = s + 1;
  g.steps = (long long*)(s + 2);
  g.err = (unsigned long long*)(s + 3);
  g.nfall = (unsigned long long*)(s + 4);
  g.dtmin = (unsigned long long*)((char*)p.scal + kScalHead);
  g.dtmask = dt_slots(cells_of(p)) - 1;
  return g;
}

// device descriptor of one problem (its buffers must be set)
template <typename TS, typename TP, typename TC>
void make_desc(Problem& p, Prob<TS, TP, TC>& d) {
  memset(&d, 0, sizeof(d));
  d.g = grid_of<TS, TP>(p);
  d.P = p.phys;
  for (int s = 0; s < 4; ++s) d.bc[s] = p.bc[s];
  d.recon_vars = p.spec.recon_vars;
  d.admissibility = p.spec.admissibility;
  d.obst_i0 = p.spec.obstacle_i0;
  d.obst_nj = p.spec.obstacle_nj;
}

// descriptors and block-owner tables of a group for its present block sizes
template <typename TS, typename TP, typename TC>
int build_tables(gks_handle* h, Group& G) {
  using PR = Prob<TS, TP, TC>;
  const size_t n = G.members.size();
  std::vector<PR> host(n);
  std::vector<std::vector<uint32_t>> own(KK_COUNT);
  for (size_t m = 0; m < n; ++m) make_desc<TS, TP, TC>(h->probs[G.members[m]], host[m]);
  for (int k = 0; k < KK_COUNT; ++k) {
    for (size_t m = 0; m < n; ++m) {
      host[m].first[k] = (unsigned)own[k].size();
      const unsigned nb = cdiv(work_items(h->probs[G.members[m]], G.dim, k, G.recon_rows, G.bs[k]), (size_t)G.bs[k]);
      own[k].insert(own[k].end(), nb, (uint32_t)m);
    }
    G.nblk[k] = (unsigned)own[k].size();
    if (G.nblk[k] > G.cap[k]) {
      if (G.owner[k]) (void)hipFree(G.owner[k]);
      G.owner[k] = nullptr;
      G.cap[k] = 0;
      HIP_OR(h, hipMalloc(&G.owner[k], own[k].size() * sizeof(uint32_t)));
      G.cap[k] = G.nblk[k];
    }
    if (G.nblk[k]) HIP_OR(h, hipMemcpy(G.owner[k], own[k].data(), own[k].size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  }
  if (!G.dprobs) HIP_OR(h, hipMalloc(&G.dprobs, n * sizeof(PR)));
  HIP_OR(h, hipMemcpy(G.dprobs, host.data(), n * sizeof(PR), hipMemcpyHostToDevice));
  return GKS_OK;
}

int build_tables(gks_handle* h, Group& G) {
  return G.mixed ? build_tables<float, float, float>(h, G) : build_tables<double, double, double>(h, G);
}

// kernel timing: events around each kernel class when profiling is on
void record_begin(gks_handle* h, hipStream_t st) {
  if (!h || h->profiling != 1) return;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  (void)hipEventRecord(a, st);
  h->pend_a.push_back(a);
  h->pend_b.push_back(b);
  h->pend_k.push_back(-1);
}
void record_end(gks_handle* h, hipStream_t st, int kernel) {
  if (!h || h->profiling != 1 || h->pend_k.empty() || h->pend_k.back() != -1) return;
  (void)hipEventRecord(h->pend_b.back(), st);
  h->pend_k.back() = kernel;
}

void collect(gks_handle* h) {
  for (size_t n = 0; n < h->pend_k.size(); ++n) {
    float ms = 0.f;
    if (h->pend_k[n] >= 0) {
      (void)hipEventSynchronize(h->pend_b[n]);
      (void)hipEventElapsedTime(&ms, h->pend_a[n], h->pend_b[n]);
      h->ktime[h->pend_k[n]] += ms;
      h->klaunch[h->pend_k[n]] += 1;
    }
    (void)hipEventDestroy(h->pend_a[n]);
    (void)hipEventDestroy(h->pend_b[n]);
  }
  h->pend_a.clear();
  h->pend_b.clear();
  h->pend_k.clear();
}

// One step of a group of problems of dimension `dim` (2D: characteristic
// reconstruction if chr; the step-image launch if it has blocks): the launch
// arguments A and block sizes bs of each launch kind, the persistent grid of
// the 2D interface launch (0: one block per logical block), the per-problem
// fixed step / end time array ctl.  h (may be null) records kernel timing.
template <typename TS, typename TP, typename TC>
void launch_step(gks_handle* h, const KA<Prob<TS, TP, TC>> (&A)[KK_COUNT], const int (&bs)[KK_COUNT], int dim,
                 bool chr, unsigned face_grid, const double* ctl, hipStream_t st, bool curv = false,
                 int recon_rows = 0) {
  using PR = Prob<TS, TP, TC>;
  record_begin(h, st);
  if (dim == 2) {
    k_ghost_2d<TS, TP, TC><<<A[KK_GA].nblk, bs[KK_GA], 0, st>>>(A[KK_GA], ctl);
    if (A[KK_OBST].nblk) k_step_images_2d<TS, TP, TC><<<A[KK_OBST].nblk, bs[KK_OBST], 0, st>>>(A[KK_OBST]);
  } else {
    k_ghost_1d<TS, TP, TC><<<A[KK_GA].nblk, bs[KK_GA], 0, st>>>(A[KK_GA], ctl);
  }
  record_end(h, st, GKS_K_GHOST);  // includes the time step
  record_begin(h, st);
  const size_t rlds = recon_rows > 0 ? 4 * (size_t)(bs[KK_RECON] / recon_rows + 2) * (recon_rows + 2) * 8 : 0;
  if (dim == 2 && recon_rows > 0 && chr)
    k_recon_2d_tile<TS, TP, TC, true><<<A[KK_RECON].nblk, bs[KK_RECON], rlds, st>>>(A[KK_RECON], recon_rows);
  else if (dim == 2 && recon_rows > 0)
    k_recon_2d_tile<TS, TP, TC, false><<<A[KK_RECON].nblk, bs[KK_RECON], rlds, st>>>(A[KK_RECON], recon_rows);
  else if (dim == 2 && chr)
    k_recon_2d<TS, TP, TC, true><<<A[KK_RECON].nblk, bs[KK_RECON], 0, st>>>(A[KK_RECON]);
  else if (dim == 2)
    k_recon_2d<TS, TP, TC, false><<<A[KK_RECON].nblk, bs[KK_RECON], 0, st>>>(A[KK_RECON]);
  else
    k_recon_1d<TS, TP, TC><<<A[KK_RECON].nblk, bs[KK_RECON], 0, st>>>(A[KK_RECON]);
  record_end(h, st, GKS_K_RECON);
  record_begin(h, st);
  if (dim == 2) {
    if (curv)
      launch_iface_2d<TS, TP, TC, true>(A[KK_FACE], bs[KK_FACE], face_grid, st);
    else
      launch_iface_2d<TS, TP, TC, false>(A[KK_FACE], bs[KK_FACE], face_grid, st);
  } else {
    k_face_1d<TS, TP, TC><<<A[KK_FACE].nblk, bs[KK_FACE], 0, st>>>(A[KK_FACE]);
  }
  record_end(h, st, GKS_K_INTERFACE);
  record_begin(h, st);
  if (dim == 2)
    k_update_2d<TS, TP, TC, false><<<A[KK_CELL].nblk, bs[KK_CELL], 0, st>>>(A[KK_CELL]);
  else
    k_update_1d<TS, TP, TC, false><<<A[KK_CELL].nblk, bs[KK_CELL], 0, st>>>(A[KK_CELL]);
  record_end(h, st, GKS_K_UPDATE);
}

template <typename TS, typename TP, typename TC>
void enqueue_group(gks_handle* h, Group& G, hipStream_t st) {
  using PR = Prob<TS, TP, TC>;
  const PR* probs = (const PR*)G.dprobs;
  KA<PR> A[KK_COUNT];
  const int single = G.members.size() == 1;
  for (int k = 0; k < KK_COUNT; ++k) A[k] = KA<PR>{probs, G.owner[k], G.nblk[k], single};
  launch_step<TS, TP, TC>(h, A, G.bs, G.dim, G.chr, G.dim == 2 ? G.face_grid : 0u, G.ctl, st, G.curv,
                          G.dim == 2 ? G.recon_rows : 0);
}

void enqueue_step(gks_handle* h, hipStream_t st) {
  for (Group& G : h->groups) {
    if (G.mixed)
      enqueue_group<float, float, float>(h, G, st);
    else
      enqueue_group<double, double, double>(h, G, st);
  }
}

template <typename TS, typename TP, typename TC>
void enqueue_scan(Group& G, hipStream_t st) {
  using PR = Prob<TS, TP, TC>;
  KA<PR> a{(const PR*)G.dprobs, G.owner[KK_CELL], G.nblk[KK_CELL], (int)(G.members.size() == 1)};
  if (G.dim == 2)
    k_update_2d<TS, TP, TC, true><<<G.nblk[KK_CELL], G.bs[KK_CELL], 0, st>>>(a);
  else
    k_update_1d<TS, TP, TC, true><<<G.nblk[KK_CELL], G.bs[KK_CELL], 0, st>>>(a);
}

void drop_graph(gks_handle* h) {
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->exec = nullptr;
  h->graph = nullptr;
}

// capture one step of every group into a graph (kernel arguments are the
// fixed device tables, so the graph stays valid until the tables change)
int ensure_graph(gks_handle* h) {
  if (h->exec) return GKS_OK;
  HIP_OR(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  const int saved = h->profiling;
  h->profiling = 0;
  enqueue_step(h, h->cap_stream);
  h->profiling = saved;
  hipGraph_t gr = nullptr;
  HIP_OR(h, hipStreamEndCapture(h->cap_stream, &gr));
  h->graph = gr;
  HIP_OR(h, hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0));
  return GKS_OK;
}

// per-problem fixed step and end time; uploaded only when they change
int set_controls(gks_handle* h, const double* dt_fixed, const double* t_end) {
  bool synced = false;
  for (Group& G : h->groups) {
    std::vector<double> c(2 * G.members.size());
    for (size_t m = 0; m < G.members.size(); ++m) {
      const int p = G.members[m];
      c[2 * m] = dt_fixed ? dt_fixed[p] : 0.0;
      c[2 * m + 1] = t_end ? t_end[p] : 0.0;
    }
    if (c == G.ctl_host) continue;
    if (!synced) {
      // earlier steps may still read the old values
      HIP_OR(h, hipStreamSynchronize(h->stream));
      synced = true;
    }
    G.ctl_host = c;
    HIP_OR(h, hipMemcpy(G.ctl, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  return GKS_OK;
}

// gks_init (host arrays cell / face_x / face_y, copied in) and
// gks_init_device (device buffers dcell / dfx / dfy, borrowed) share this body
int init_handle(gks_handle** out, int32_t n_problems, const gks_problem* probs, const double* const* cell,
                const double* const* face_x, const double* const* face_y, void* const* dcell, void* const* dfx,
                void* const* dfy, void* stream) {
  if (!out) return GKS_EINVAL;
  *out = nullptr;
  g_init_msg.clear();
  const bool dev = dcell != nullptr;
  if (n_problems < 1 || n_problems > kMaxProblems || !probs || !(dev ? (bool)dfx : (cell && face_x))) {
    g_init_msg = "n_problems must lie in [1, 65535] and probs, cell, face_x must be given";
    return GKS_EINVAL;
  }
  gks_handle* h = new (std::nothrow) gks_handle();
  if (!h) return GKS_ENOMEM;
  auto init_fail = [&](int code, const std::string& m) {
    h->msg = m;
    g_init_msg = m;
    gks_destroy(h);
    return code;
  };
  h->probs.resize(n_problems);
  std::vector<std::vector<double>> geoms(n_problems);
  for (int n = 0; n < n_problems; ++n) {
    const gks_problem& s = probs[n];
    std::string why = validate(s);
    if (why.empty() && s.mesh) why = curvilinear_geometry(s, geoms[n]);
    const bool given = dev ? dcell[n] && dfx[n] && (s.dim == 1 || (dfy && dfy[n]))
                           : cell[n] && face_x[n] && (s.dim == 1 || (face_y && face_y[n]));
    if (why.empty() && !given) why = "null array";
    if (why.empty() && dev) {
      const size_t fe = s.precision == GKS_FP32_MIXED ? 4 : 8;
      size_t e[3];
      state_elems(s, e);
      if ((uintptr_t)dcell[n] % 8 || (uintptr_t)dfx[n] % fe || (s.dim == 2 && (uintptr_t)dfy[n] % fe))
        why = "device buffers must be aligned to their element size";
      if (why.empty()) why = check_device_buffer("d_cell", dcell[n], e[0] * 8);
      if (why.empty()) why = check_device_buffer("d_face_x", dfx[n], e[1] * fe);
      if (why.empty() && s.dim == 2) why = check_device_buffer("d_face_y", dfy[n], e[2] * fe);
    }
    if (!why.empty()) return init_fail(GKS_EINVAL, "problem " + std::to_string(n) + ": " + why);
    Problem& p = h->probs[n];
    setup_problem(s, p);
    // the initial state must be physical (device buffers: checked by the
    // initial CFL scan below)
    const size_t nc = dev ? 0 : (size_t)s.nx * p.ix.ny;
    for (size_t c = 0; c < nc; ++c) {
      const double r = cell[n][c], mu_ = cell[n][nc + c];
      const double mv = s.dim == 2 ? cell[n][2 * nc + c] : 0.0, E = cell[n][(s.dim + 1) * nc + c];
      const double pr = (s.gamma - 1.0) * (E - 0.5 * (mu_ * mu_ + mv * mv) / r);
      if (!(r > 0.0) || !(pr > 0.0) || !std::isfinite(pr))
        return init_fail(GKS_EINVAL, "problem " + std::to_string(n) + ": nonphysical initial cell " +
                                         std::to_string(c));
    }
  }
  if (stream) {
    h->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
      return init_fail(GKS_EDEVICE, "hipStreamCreateWithFlags failed");
    h->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return init_fail(GKS_EDEVICE, "hipStreamCreateWithFlags failed");
  for (int n = 0; n < n_problems; ++n) {
    Problem& p = h->probs[n];
    const gks_problem& s = p.spec;
    const size_t ts = p.mixed ? sizeof(float) : sizeof(double);
    const Idx& x = p.ix;
    const size_t nx = s.nx, ny = x.ny;
    void** bufs[kBufs] = {&p.W, &p.FX, &p.FY, &p.PC, &p.FLX, &p.FLY, &p.scal};
    size_t sizes[kBufs];
    buffer_sizes(p, sizes);
    if (dev) {
      p.borrowed = true;
      p.W = dcell[n];
      p.FX = dfx[n];
      p.FY = s.dim == 2 ? dfy[n] : nullptr;
    }
    for (int b = 0; b < kBufs; ++b) {
      if (!sizes[b] || (dev && b < 3)) continue;
      if (hipMalloc(bufs[b], sizes[b]) != hipSuccess) {
        *bufs[b] = nullptr;
        return init_fail(GKS_ENOMEM, "device allocation failed");
      }
      if (hipMemsetAsync(*bufs[b], 0, sizes[b], h->stream) != hipSuccess)
        return init_fail(GKS_EDEVICE, "hipMemsetAsync failed");
    }
    if (!geoms[n].empty()) {
      if (hipMalloc(&p.geom, geoms[n].size() * 8) != hipSuccess) {
        p.geom = nullptr;
        return init_fail(GKS_ENOMEM, "device allocation failed");
      }
      if (hipMemcpy(p.geom, geoms[n].data(), geoms[n].size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return init_fail(GKS_EDEVICE, "upload failed");
    }
    // a periodic seam is one interface: its values are those of the first
    if (dev && s.dim == 2) {
      bool ok = true;
      if (x.fxr == s.nx)
        ok = ok && hipMemcpy2DAsync((char*)p.FX + (nx + 1) * ts, (nx + 3) * ts, (const char*)p.FX + ts,
                                    (nx + 3) * ts, ts, 2 * 4 * (ny + 2), hipMemcpyDeviceToDevice,
                                    h->stream) == hipSuccess;
      if (x.fyr == s.ny)
        ok = ok && hipMemcpy2DAsync((char*)p.FY + (ny + 1) * (nx + 2) * ts, (ny + 3) * (nx + 2) * ts,
                                    (const char*)p.FY + (nx + 2) * ts, (ny + 3) * (nx + 2) * ts, (nx + 2) * ts,
                                    2 * 4, hipMemcpyDeviceToDevice, h->stream) == hipSuccess;
      if (!ok) return init_fail(GKS_EDEVICE, "seam copy failed");
    }
    // the clears above must land before the blocking uploads below
    if (hipStreamSynchronize(h->stream) != hipSuccess) return init_fail(GKS_EDEVICE, "hipStreamSynchronize failed");
    const double scal0[4] = {s.t0, 0.0, 0.0, 0.0};
    const size_t slot_words = (size_t)dt_slots(cells_of(p)) * kDtStride;
    const std::vector<unsigned long long> inf(slot_words, 0x7e37e43c8800759cull);  // bits of 1e300
    if (hipMemcpy(p.scal, scal0, sizeof(scal0), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((char*)p.scal + kScalHead, inf.data(), slot_words * 8, hipMemcpyHostToDevice) != hipSuccess)
      return init_fail(GKS_EDEVICE, "upload failed");
    if (dev) continue;
    // upload: host layouts without ghosts -> ghosted device layouts
    std::vector<double> W(sizes[0] / 8, 0.0), FX(sizes[1] / ts, 0.0), FY(sizes[2] / ts, 0.0);
    if (s.dim == 2) {
      for (int v = 0; v < 4; ++v)
        for (int j = 0; j < s.ny; ++j)
          for (int i = 0; i < s.nx; ++i) W[x.w(v, j, i)] = cell[n][((size_t)v * s.ny + j) * s.nx + i];
      for (int g = 0; g < 2; ++g)
        for (int v = 0; v < 4; ++v) {
          for (int j = 0; j < s.ny; ++j)
            for (int fi = 0; fi <= s.nx; ++fi)
              FX[x.fx(g, v, j, fi)] = face_x[n][(((size_t)g * 4 + v) * s.ny + j) * (s.nx + 1) + fi];
          for (int fj = 0; fj <= s.ny; ++fj)
            for (int i = 0; i < s.nx; ++i)
              FY[x.fy(g, v, fj, i)] = face_y[n][(((size_t)g * 4 + v) * (s.ny + 1) + fj) * s.nx + i];
          // a periodic seam is one interface: its values are those of the first
          if (x.fxr == s.nx)
            for (int j = 0; j < s.ny; ++j) FX[x.fx(g, v, j, s.nx)] = FX[x.fx(g, v, j, 0)];
          if (x.fyr == s.ny)
            for (int i = 0; i < s.nx; ++i) FY[x.fy(g, v, s.ny, i)] = FY[x.fy(g, v, 0, i)];
        }
    } else {
      for (int v = 0; v < 3; ++v) {
        for (int i = 0; i < s.nx; ++i) W[x.w1(v, i)] = cell[n][(size_t)v * s.nx + i];
        for (int fi = 0; fi <= s.nx; ++fi) FX[x.f1(v, fi)] = face_x[n][(size_t)v * (s.nx + 1) + fi];
      }
    }
    if (hipMemcpy(p.W, W.data(), W.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return init_fail(GKS_EDEVICE, "upload failed");
    bool up = true;
    if (p.mixed) {
      std::vector<float> fx(FX.begin(), FX.end()), fy(FY.begin(), FY.end());
      up = hipMemcpy(p.FX, fx.data(), fx.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
           (fy.empty() || hipMemcpy(p.FY, fy.data(), fy.size() * 4, hipMemcpyHostToDevice) == hipSuccess);
    } else {
      up = hipMemcpy(p.FX, FX.data(), FX.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
           (FY.empty() || hipMemcpy(p.FY, FY.data(), FY.size() * 8, hipMemcpyHostToDevice) == hipSuccess);
    }
    if (!up) return init_fail(GKS_EDEVICE, "upload failed");
  }
  // groups: problems of one dimension, precision and (2D) reconstruction
  // variables, in problem order (1D chooses the variables per problem in the
  // kernel)
  for (int n = 0; n < n_problems; ++n) {
    const Problem& p = h->probs[n];
    Group* G = nullptr;
    const bool chr = p.spec.dim == 2 && p.spec.recon_vars == 1;
    const bool curv = p.geom != nullptr;
    for (Group& g : h->groups)
      if (g.dim == p.spec.dim && g.mixed == p.mixed && g.chr == chr && g.curv == curv) G = &g;
    if (!G) {
      h->groups.emplace_back();
      G = &h->groups.back();
      G->dim = p.spec.dim;
      G->mixed = p.mixed;
      G->chr = chr;
      G->curv = curv;
    }
    G->members.push_back(n);
  }
  for (Group& G : h->groups) {
    const int rc = build_tables(h, G);
    if (rc != GKS_OK) return init_fail(rc, h->msg);
    if (hipMalloc(&G.ctl, 2 * G.members.size() * sizeof(double)) != hipSuccess)
      return init_fail(GKS_ENOMEM, "device allocation failed");
    G.ctl_host.assign(2 * G.members.size(), 0.0);
    if (hipMemcpy(G.ctl, G.ctl_host.data(), G.ctl_host.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return init_fail(GKS_EDEVICE, "upload failed");
    // CFL bound of the initial state
    if (G.mixed)
      enqueue_scan<float, float, float>(G, h->stream);
    else
      enqueue_scan<double, double, double>(G, h->stream);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
    return init_fail(GKS_EDEVICE, "initial CFL scan failed");
  // the scan flags a nonphysical initial cell in the error word
  for (int n = 0; n < n_problems; ++n) {
    unsigned long long err = 0;
    if (hipMemcpy(&err, (char*)h->probs[n].scal + 24, 8, hipMemcpyDeviceToHost) != hipSuccess)
      return init_fail(GKS_EDEVICE, "download failed");
    if (err)
      return init_fail(GKS_EINVAL, "problem " + std::to_string(n) + ": nonphysical initial cell (i, j) = (" +
                                       std::to_string((long long)(err & 0xffffffff) - 2) + ", " +
                                       std::to_string((long long)((err >> 32) & 0x3fffffff) - 1) + ")");
  }
  *out = h;
  return GKS_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free stepping of one problem (gks_step_noalloc): every internal
// buffer (descriptor, controls, scalars, reconstruction coefficients,
// fluxes, frame record) lives in one static device array per GPU.  Host code
// reaches that array only through the address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(128) << 20;  // per GPU, held until the process ends
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch array (looked up once per
// device)
int scratch_base(void** out, std::string* why) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *why = "no usable current device";
    return GKS_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      *why = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return GKS_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GKS_OK;
}

// the descriptor, the controls and the scalars of the step (time t0, no
// error, no fallbacks, empty CFL slots); one block
template <class PR>
__global__ void __launch_bounds__(256) k_noalloc_setup(PR desc, PR* dst, double* ctl, double fixed, double t_end,
                                                      double t0) {
  if (threadIdx.x == 0) {
    *dst = desc;
    ctl[0] = fixed;
    ctl[1] = t_end;
    *desc.g.t = t0;
    *desc.g.dt = 0.0;
    *desc.g.steps = 0;
    *desc.g.err = 0;
    *desc.g.nfall = 0;
  }
  for (unsigned q = threadIdx.x; q <= desc.g.dtmask; q += blockDim.x)
    desc.g.dtmin[q * kDtStride] = (unsigned long long)__double_as_longlong(1e300);
}

// periodic seams of the caller's point values: the last interface of a row
// (column) takes the first one's values, over the whole ghosted extent
template <typename TS>
__global__ void __launch_bounds__(256) k_noalloc_seams(TS* FX, TS* FY, int nx, int ny, int px, int py) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (px && id < 8 * (ny + 2)) {
    TS* row = FX + (size_t)id * (nx + 3);  // plane (g, v) and padded row of FX
    row[nx + 1] = row[1];
  }
  if (py && id < 8 * (nx + 2)) {
    const int pl = id / (nx + 2), c = id % (nx + 2);
    TS* plane = FY + (size_t)pl * (ny + 3) * (nx + 2);
    plane[(size_t)(ny + 1) * (nx + 2) + c] = plane[(size_t)(nx + 2) + c];
  }
}

// time, steps, error word and fallback count after the last step
template <class PR>
__global__ void k_noalloc_status(const PR* d, gks_noalloc_status* out) {
  out->t = *d->g.t;
  out->steps = (int64_t)*d->g.steps;
  out->error = (uint64_t)*d->g.err;
  out->fallbacks = (int64_t)*d->g.nfall;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

template <typename TS, typename TP, typename TC>
int noalloc_run(Problem& p, char* base, int32_t nsteps, double dt_fixed, double t_end, gks_noalloc_status* status,
                hipStream_t st) {
  using PR = Prob<TS, TP, TC>;
  const int dim = p.spec.dim;
  PR desc;
  make_desc<TS, TP, TC>(p, desc);
  PR* dprob = (PR*)(base);
  double* ctl = (double*)(base + align256(sizeof(PR)));
  k_noalloc_setup<PR><<<1, 256, 0, st>>>(desc, dprob, ctl, dt_fixed, t_end, p.spec.t0);
  if (dim == 2 && (p.ix.fxr == p.ix.nx || p.ix.fyr == p.ix.ny)) {
    const int n = 8 * ((p.ix.nx > p.ix.ny ? p.ix.nx : p.ix.ny) + 2);
    k_noalloc_seams<TS><<<cdiv((size_t)n, 256), 256, 0, st>>>((TS*)p.FX, (TS*)p.FY, p.ix.nx, p.ix.ny,
                                                               p.ix.fxr == p.ix.nx, p.ix.fyr == p.ix.ny);
  }
  const int bs[KK_COUNT] = {256, 256, 256, 256, 64};
  KA<PR> A[KK_COUNT];
  for (int k = 0; k < KK_COUNT; ++k)
    A[k] = KA<PR>{dprob, nullptr, cdiv(work_items(p, dim, k), (size_t)bs[k]), 1};
  // CFL bound of the initial state (and its nonphysical-cell check)
  if (dim == 2)
    k_update_2d<TS, TP, TC, true><<<A[KK_CELL].nblk, bs[KK_CELL], 0, st>>>(A[KK_CELL]);
  else
    k_update_1d<TS, TP, TC, true><<<A[KK_CELL].nblk, bs[KK_CELL], 0, st>>>(A[KK_CELL]);
  const bool chr = dim == 2 && p.spec.recon_vars == 1;
  for (int32_t n = 0; n < nsteps; ++n) launch_step<TS, TP, TC>(nullptr, A, bs, dim, chr, 0u, ctl, st);
  if (status) k_noalloc_status<PR><<<1, 1, 0, st>>>(dprob, status);
  return hipGetLastError() == hipSuccess ? GKS_OK : GKS_EDEVICE;
}

}  // namespace

// the persistent grid of a 2D group's interface launch: the blocks of its
// present size that fit on the device at once, a multiple of 8
template <typename TS, typename TP, typename TC>
int persistent_grid_of(gks_handle* h, int bs, unsigned* grid) {
  int per_cu = 0, cus = 0, dev = 0;
  HIP_OR(h, hipGetDevice(&dev));
  HIP_OR(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const size_t lds = (size_t)bs * iface_lds_per_thread<TC>();
  if (bs == 64)
    HIP_OR(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_iface_2d_loop<TS, TP, TC, false, 64>, bs, lds));
  else if (bs == 128)
    HIP_OR(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_iface_2d_loop<TS, TP, TC, false, 128>, bs, lds));
  else
    HIP_OR(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_iface_2d_loop<TS, TP, TC, false, 256>, bs, lds));
  const unsigned n = (unsigned)(per_cu > 0 ? per_cu : 1) * (unsigned)(cus > 0 ? cus : 8);
  *grid = n < 8 ? 8u : n & ~7u;
  return GKS_OK;
}

int persistent_face_grid(gks_handle* h, const Group& G, unsigned* grid) {
  return G.mixed ? persistent_grid_of<float, float, float>(h, G.bs[KK_FACE], grid)
                 : persistent_grid_of<double, double, double>(h, G.bs[KK_FACE], grid);
}

extern "C" {

int gks_init(gks_handle** out, int32_t n_problems, const gks_problem* probs, const double* const* cell,
             const double* const* face_x, const double* const* face_y, void* stream) {
  return init_handle(out, n_problems, probs, cell, face_x, face_y, nullptr, nullptr, nullptr, stream);
}

int gks_init_device(gks_handle** out, int32_t n_problems, const gks_problem* probs, void* const* d_cell,
                    void* const* d_face_x, void* const* d_face_y, void* stream) {
  if (!d_cell) {
    if (out) *out = nullptr;
    g_init_msg = "d_cell must be given";
    return GKS_EINVAL;
  }
  return init_handle(out, n_problems, probs, nullptr, nullptr, nullptr, d_cell, d_face_x, d_face_y, stream);
}

int gks_step_noalloc(const gks_problem* prob, void* d_cell, void* d_face_x, void* d_face_y, int32_t nsteps,
                     double dt_fixed, double t_end, gks_noalloc_status* d_status, void* stream) {
  g_init_msg.clear();
  if (!prob || !d_cell || !d_face_x || (prob->dim == 2 && !d_face_y)) {
    g_init_msg = "prob, d_cell, d_face_x (and d_face_y in 2D) must be given";
    return GKS_EINVAL;
  }
  std::string why = validate(*prob);
  if (why.empty() && prob->mesh) why = "curvilinear grids are stepped through a handle (gks_init, gks_init_device)";
  if (why.empty() && nsteps < 0) why = "nsteps < 0";
  if (why.empty() && !(dt_fixed >= 0.0 && std::isfinite(dt_fixed))) why = "dt_fixed must be >= 0 and finite";
  if (why.empty() && !(t_end >= 0.0 && std::isfinite(t_end))) why = "t_end must be >= 0 and finite";
  const size_t fe = prob->precision == GKS_FP32_MIXED ? 4 : 8;
  size_t e[3] = {0, 0, 0};
  if (why.empty()) {
    state_elems(*prob, e);
    if ((uintptr_t)d_cell % 8 || (uintptr_t)d_face_x % fe || (prob->dim == 2 && (uintptr_t)d_face_y % fe))
      why = "device buffers must be aligned to their element size";
  }
  if (why.empty()) why = check_device_buffer("d_cell", d_cell, e[0] * 8);
  if (why.empty()) why = check_device_buffer("d_face_x", d_face_x, e[1] * fe);
  if (why.empty() && prob->dim == 2) why = check_device_buffer("d_face_y", d_face_y, e[2] * fe);
  if (why.empty() && d_status) why = check_device_buffer("d_status", d_status, sizeof(gks_noalloc_status));
  if (!why.empty()) {
    g_init_msg = why;
    return GKS_EINVAL;
  }
  Problem p;
  setup_problem(*prob, p);
  p.W = d_cell;
  p.FX = d_face_x;
  p.FY = prob->dim == 2 ? d_face_y : nullptr;
  // the scratch layout: descriptor, controls, then the internal buffers
  size_t sizes[kBufs];
  buffer_sizes(p, sizes);
  const size_t head = align256(sizeof(Prob<double, double, double>)) + 256;
  size_t need = head;
  for (int b = 3; b < kBufs; ++b) need += align256(sizes[b]);
  if (need > kScratchBytes) {
    g_init_msg = "the problem needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                 std::to_string(kScratchBytes);
    return GKS_EINVAL;
  }
  void* base = nullptr;
  const int rc = scratch_base(&base, &why);
  if (rc != GKS_OK) {
    g_init_msg = why;
    return rc;
  }
  void** bufs[kBufs] = {&p.W, &p.FX, &p.FY, &p.PC, &p.FLX, &p.FLY, &p.scal};
  size_t off = head;
  for (int b = 3; b < kBufs; ++b) {
    *bufs[b] = sizes[b] ? (char*)base + off : nullptr;
    off += align256(sizes[b]);
  }
  const hipStream_t st = (hipStream_t)stream;
  const int r = p.mixed ? noalloc_run<float, float, float>(p, (char*)base, nsteps, dt_fixed, t_end, d_status, st)
                        : noalloc_run<double, double, double>(p, (char*)base, nsteps, dt_fixed, t_end, d_status, st);
  if (r != GKS_OK) g_init_msg = "kernel launch failed";
  return r;
}

int gks_state_extent(const gks_problem* prob, int64_t* cell_elems, int64_t* face_x_elems, int64_t* face_y_elems,
                     int32_t* face_elem_bytes) {
  g_init_msg.clear();
  if (!prob) {
    g_init_msg = "prob must be given";
    return GKS_EINVAL;
  }
  const std::string why = validate(*prob);
  if (!why.empty()) {
    g_init_msg = why;
    return GKS_EINVAL;
  }
  size_t e[3];
  state_elems(*prob, e);
  if (cell_elems) *cell_elems = (int64_t)e[0];
  if (face_x_elems) *face_x_elems = (int64_t)e[1];
  if (face_y_elems) *face_y_elems = (int64_t)e[2];
  if (face_elem_bytes) *face_elem_bytes = prob->precision == GKS_FP32_MIXED ? 4 : 8;
  return GKS_OK;
}

int gks_step(gks_handle* h, int32_t nsteps, const double* dt_fixed, const double* t_end) {
  if (!h) return GKS_EINVAL;
  if (h->sticky != GKS_OK) return fail(h, GKS_ESTATE, "handle in error state: " + h->msg);
  if (nsteps < 0) return fail(h, GKS_EINVAL, "nsteps < 0");
  for (size_t n = 0; n < h->probs.size(); ++n) {
    if (dt_fixed && !(dt_fixed[n] > 0.0 && std::isfinite(dt_fixed[n])))
      return fail(h, GKS_EINVAL, "dt_fixed must be positive and finite");
    if (t_end && !std::isfinite(t_end[n])) return fail(h, GKS_EINVAL, "t_end must be finite");
  }
  if (nsteps == 0) return GKS_OK;
  int rc = set_controls(h, dt_fixed, t_end);
  if (rc != GKS_OK) return rc;
  if (h->profiling == 1) {
    for (int s = 0; s < nsteps; ++s) enqueue_step(h, h->stream);
  } else {
    rc = ensure_graph(h);
    if (rc != GKS_OK) return rc;
    for (int s = 0; s < nsteps; ++s) HIP_OR(h, hipGraphLaunch(h->exec, h->stream));
  }
  HIP_OR(h, hipGetLastError());
  return GKS_OK;
}

int gks_fetch(gks_handle* h, int32_t problem, double* cell, double* face_x, double* face_y, double* t,
              int64_t* steps) {
  if (!h) return GKS_EINVAL;
  if (problem < 0 || problem >= (int)h->probs.size()) return fail(h, GKS_EINVAL, "problem index out of range");
  HIP_OR(h, hipStreamSynchronize(h->stream));
  Problem& p = h->probs[problem];
  const Idx& x = p.ix;
  const gks_problem& s = p.spec;
  double scal[4];
  HIP_OR(h, hipMemcpy(scal, p.scal, sizeof(scal), hipMemcpyDeviceToHost));
  if (t) *t = scal[0];
  if (steps) *steps = *(long long*)&scal[2];
  unsigned long long err = *(unsigned long long*)&scal[3];
  const size_t ts = p.mixed ? 4 : 8;
  auto fetch_ts = [&](const void* src, size_t count, std::vector<double>& dst) -> hipError_t {
    dst.resize(count);
    if (p.mixed) {
      std::vector<float> f(count);
      hipError_t e = hipMemcpy(f.data(), src, count * 4, hipMemcpyDeviceToHost);
      dst.assign(f.begin(), f.end());
      return e;
    }
    return hipMemcpy(dst.data(), src, count * 8, hipMemcpyDeviceToHost);
  };
  if (s.dim == 2) {
    if (cell) {
      std::vector<double> W((size_t)4 * (s.ny + 4) * (s.nx + 4));
      HIP_OR(h, hipMemcpy(W.data(), p.W, W.size() * 8, hipMemcpyDeviceToHost));
      for (int v = 0; v < 4; ++v)
        for (int j = 0; j < s.ny; ++j)
          for (int i = 0; i < s.nx; ++i) cell[((size_t)v * s.ny + j) * s.nx + i] = W[x.w(v, j, i)];
    }
    if (face_x || face_y) {
      std::vector<double> FX, FY;
      HIP_OR(h, fetch_ts(p.FX, (size_t)2 * 4 * (s.ny + 2) * (s.nx + 3), FX));
      HIP_OR(h, fetch_ts(p.FY, (size_t)2 * 4 * (s.ny + 3) * (s.nx + 2), FY));
      for (int g = 0; g < 2; ++g)
        for (int v = 0; v < 4; ++v) {
          if (face_x)
            for (int j = 0; j < s.ny; ++j)
              for (int fi = 0; fi <= s.nx; ++fi)
                face_x[(((size_t)g * 4 + v) * s.ny + j) * (s.nx + 1) + fi] = FX[x.fx(g, v, j, fi)];
          if (face_y)
            for (int fj = 0; fj <= s.ny; ++fj)
              for (int i = 0; i < s.nx; ++i)
                face_y[(((size_t)g * 4 + v) * (s.ny + 1) + fj) * s.nx + i] = FY[x.fy(g, v, fj, i)];
        }
    }
  } else {
    if (cell) {
      std::vector<double> W((size_t)3 * (s.nx + 4));
      HIP_OR(h, hipMemcpy(W.data(), p.W, W.size() * 8, hipMemcpyDeviceToHost));
      for (int v = 0; v < 3; ++v)
        for (int i = 0; i < s.nx; ++i) cell[(size_t)v * s.nx + i] = W[x.w1(v, i)];
    }
    if (face_x) {
      std::vector<double> F;
      HIP_OR(h, fetch_ts(p.FX, (size_t)3 * (s.nx + 3), F));
      for (int v = 0; v < 3; ++v)
        for (int fi = 0; fi <= s.nx; ++fi) face_x[(size_t)v * (s.nx + 1) + fi] = F[x.f1(v, fi)];
    }
  }
  (void)ts;
  if (err) {
    const int kind = (int)(err >> 62);
    const long long a = (long long)((err >> 32) & 0x3fffffff) - 1, b = (long long)(err & 0xffffffff) - 2;
    const char* where = kind == 2 ? "cell" : kind == 1 ? "y interface" : "x interface";
    h->sticky = GKS_ENONPHYS;
    return fail(h, GKS_ENONPHYS, "problem " + std::to_string(problem) + ": nonphysical state at " + where +
                                     " (i, j) = (" + std::to_string(b) + ", " + std::to_string(a) + ")");
  }
  return h->sticky;
}

int gks_fallbacks(gks_handle* h, int32_t problem, int64_t* cells) {
  if (!h || !cells) return GKS_EINVAL;
  if (problem < 0 || problem >= (int)h->probs.size()) return fail(h, GKS_EINVAL, "problem index out of range");
  HIP_OR(h, hipStreamSynchronize(h->stream));
  unsigned long long n = 0;
  HIP_OR(h, hipMemcpy(&n, (char*)h->probs[problem].scal + 32, 8, hipMemcpyDeviceToHost));
  *cells = (int64_t)n;
  return GKS_OK;
}

int gks_tune(gks_handle* h, int32_t steps) {
  if (!h) return GKS_EINVAL;
  if (h->sticky != GKS_OK) return fail(h, GKS_ESTATE, "handle in error state: " + h->msg);
  if (steps < 1 || steps > 1000) return fail(h, GKS_EINVAL, "steps must lie in [1, 1000]");
  HIP_OR(h, hipStreamSynchronize(h->stream));
  // save the state that a step changes (averages, point values, scalars)
  struct Saved {
    void* dst;
    void* copy;
    size_t bytes;
  };
  std::vector<Saved> saved;
  int rc = GKS_OK;
  for (Problem& p : h->probs) {
    const size_t ts = p.mixed ? 4 : 8;
    const size_t nx = p.ix.nx, ny = p.ix.ny;
    const bool two = p.spec.dim == 2;
    const Saved s[4] = {{p.W, nullptr, (two ? 4 * (ny + 4) : 3) * (nx + 4) * 8},
                        {p.FX, nullptr, (two ? 2 * 4 * (ny + 2) : 3) * (nx + 3) * ts},
                        {p.FY, nullptr, two ? 2 * 4 * (ny + 3) * (nx + 2) * ts : 0},
                        {p.scal, nullptr, scal_bytes(cells_of(p))}};
    for (const Saved& x : s) {
      if (!x.bytes) continue;
      Saved y = x;
      if (hipMalloc(&y.copy, y.bytes) != hipSuccess) {
        rc = fail(h, GKS_ENOMEM, "device allocation failed");
        break;
      }
      saved.push_back(y);
      if (hipMemcpy(y.copy, y.dst, y.bytes, hipMemcpyDeviceToDevice) != hipSuccess) {
        rc = fail(h, GKS_EDEVICE, "state copy failed");
        break;
      }
    }
    if (rc != GKS_OK) break;
  }
  auto restore = [&]() -> int {
    for (const Saved& y : saved)
      if (hipMemcpy(y.dst, y.copy, y.bytes, hipMemcpyDeviceToDevice) != hipSuccess)
        return fail(h, GKS_EDEVICE, "state restore failed");
    return GKS_OK;
  };
  // time every candidate block size for all kernel classes at once and
  // keep the fastest per class.  A later candidate (and below, the
  // persistent form and the reconstruction tiles) replaces the one kept only
  // if it is faster by more than kTuneMargin: shapes within timing noise of
  // each other would otherwise be picked at random from run to run
  constexpr double kTuneMargin = 0.98;
  static const int cand[3] = {64, 128, 256};
  static const int cls[KK_COUNT] = {GKS_K_GHOST, GKS_K_RECON, GKS_K_INTERFACE, GKS_K_UPDATE, GKS_K_GHOST};
  double best_t[GKS_K_COUNT];
  int best_bs[GKS_K_COUNT];
  for (int k = 0; k < GKS_K_COUNT; ++k) {
    best_t[k] = 1e300;
    best_bs[k] = 256;
  }
  const int saved_prof = h->profiling;
  double saved_time[GKS_K_COUNT];
  long long saved_launch[GKS_K_COUNT];
  collect(h);
  memcpy(saved_time, h->ktime, sizeof(saved_time));
  memcpy(saved_launch, h->klaunch, sizeof(saved_launch));
  // one warm-up step, then `steps` timed steps (kernel times in h->ktime),
  // then the saved state back
  auto time_steps = [&]() -> int {
    for (int k = 0; k < GKS_K_COUNT; ++k) h->ktime[k] = 0.0;
    h->profiling = 1;
    enqueue_step(h, h->stream);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, GKS_EDEVICE, "tuning step failed");
    collect(h);
    for (int k = 0; k < GKS_K_COUNT; ++k) h->ktime[k] = 0.0;
    for (int s = 0; s < steps; ++s) enqueue_step(h, h->stream);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, GKS_EDEVICE, "tuning step failed");
    collect(h);
    return restore();
  };
  for (Group& G : h->groups) {
    G.face_grid = 0;
    G.recon_rows = 0;
  }
  for (int c = 0; c < 3 && rc == GKS_OK; ++c) {
    for (Group& G : h->groups) {
      for (int k = 0; k < KK_COUNT; ++k) G.bs[k] = cand[c];
      if ((rc = build_tables(h, G)) != GKS_OK) break;
    }
    if (rc != GKS_OK || (rc = time_steps()) != GKS_OK) break;
    for (int k = 0; k < GKS_K_COUNT; ++k)
      if (k != GKS_K_DT && h->ktime[k] < kTuneMargin * best_t[k]) {
        best_t[k] = h->ktime[k];
        best_bs[k] = cand[c];
      }
  }
  if (rc == GKS_OK) {
    for (Group& G : h->groups) {
      for (int k = 0; k < KK_COUNT; ++k) G.bs[k] = best_bs[cls[k]];
      if ((rc = build_tables(h, G)) != GKS_OK) break;
    }
  }
  // then the persistent form of the 2D interface launch at that block size:
  // as many blocks as fit on the device at once (a multiple of 8)
  bool any2d = false;
  for (Group& G : h->groups) any2d |= G.dim == 2;
  if (rc == GKS_OK && any2d) {
    for (Group& G : h->groups)
      if (G.dim == 2 && (rc = persistent_face_grid(h, G, &G.face_grid)) != GKS_OK) break;
    if (rc == GKS_OK) rc = time_steps();
    if (rc == GKS_OK && !(h->ktime[GKS_K_INTERFACE] < kTuneMargin * best_t[GKS_K_INTERFACE]))
      for (Group& G : h->groups) G.face_grid = 0;
    // and the tiled reconstruction (averages staged in LDS) with 1, 2 or 4
    // rows per tile at that block size
    int best_rows = 0;
    for (int rows = 1; rows <= 4 && rc == GKS_OK; rows *= 2) {
      for (Group& G : h->groups) {
        G.recon_rows = G.dim == 2 ? rows : 0;
        if ((rc = build_tables(h, G)) != GKS_OK) break;
      }
      if (rc == GKS_OK && (rc = time_steps()) == GKS_OK && h->ktime[GKS_K_RECON] < kTuneMargin * best_t[GKS_K_RECON]) {
        best_t[GKS_K_RECON] = h->ktime[GKS_K_RECON];
        best_rows = rows;
      }
    }
    for (Group& G : h->groups) {
      if (rc != GKS_OK) break;
      G.recon_rows = G.dim == 2 ? best_rows : 0;
      rc = build_tables(h, G);
    }
  }
  h->profiling = saved_prof;
  memcpy(h->ktime, saved_time, sizeof(saved_time));
  memcpy(h->klaunch, saved_launch, sizeof(saved_launch));
  if (rc == GKS_OK) rc = restore();
  for (const Saved& y : saved) (void)hipFree(y.copy);
  if (rc != GKS_OK) h->sticky = rc;
  return rc;
}

int gks_block_size(gks_handle* h, int32_t kernel, int32_t* threads) {
  if (!h || !threads || kernel < 0 || kernel >= GKS_K_COUNT) return GKS_EINVAL;
  static const int kind_of[GKS_K_COUNT] = {KK_GA, -1, KK_RECON, KK_FACE, KK_CELL};
  *threads = kind_of[kernel] < 0 ? 64 : h->groups[0].bs[kind_of[kernel]];
  return GKS_OK;
}

int gks_launch_shape(gks_handle* h, int32_t kernel, int32_t* threads, int32_t* grid) {
  if (!h || !threads || !grid || kernel < 0 || kernel >= GKS_K_COUNT) return GKS_EINVAL;
  int rc = gks_block_size(h, kernel, threads);
  *grid = 0;
  for (const Group& G : h->groups)
    if (G.dim == 2) *grid = kernel == GKS_K_INTERFACE ? (int32_t)G.face_grid : kernel == GKS_K_RECON ? G.recon_rows : 0;
  return rc;
}

int gks_set_launch(gks_handle* h, int32_t kernel, int32_t threads, int32_t grid) {
  if (!h) return GKS_EINVAL;
  if (h->sticky != GKS_OK) return fail(h, GKS_ESTATE, "handle in error state: " + h->msg);
  if (kernel < 0 || kernel >= GKS_K_COUNT || kernel == GKS_K_DT)
    return fail(h, GKS_EINVAL, "no such kernel class");
  if (threads != 64 && threads != 128 && threads != 256) return fail(h, GKS_EINVAL, "threads must be 64, 128 or 256");
  if (kernel == GKS_K_RECON && grid != 0 && grid != 1 && grid != 2 && grid != 4)
    return fail(h, GKS_EINVAL, "reconstruction tiles have 1, 2 or 4 rows (0: row order)");
  if (kernel != GKS_K_RECON && grid != 0 && (kernel != GKS_K_INTERFACE || grid < 8 || grid > 65536 || grid % 8))
    return fail(h, GKS_EINVAL, "a persistent grid (a multiple of 8 in [8, 65536]) exists for the interface kernel only");
  HIP_OR(h, hipStreamSynchronize(h->stream));
  for (Group& G : h->groups) {
    for (int k = 0; k < KK_COUNT; ++k) {
      static const int cls[KK_COUNT] = {GKS_K_GHOST, GKS_K_RECON, GKS_K_INTERFACE, GKS_K_UPDATE, GKS_K_GHOST};
      if (cls[k] == kernel) G.bs[k] = threads;
    }
    if (kernel == GKS_K_INTERFACE) G.face_grid = G.dim == 2 ? (unsigned)grid : 0u;
    if (kernel == GKS_K_RECON) G.recon_rows = G.dim == 2 ? grid : 0;
    int rc = build_tables(h, G);
    if (rc != GKS_OK) return rc;
  }
  drop_graph(h);
  return GKS_OK;
}

int gks_destroy(gks_handle* h) {
  if (!h) return GKS_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  collect(h);
  drop_graph(h);
  for (Group& G : h->groups) {
    if (G.dprobs) (void)hipFree(G.dprobs);
    if (G.ctl) (void)hipFree(G.ctl);
    for (int k = 0; k < KK_COUNT; ++k)
      if (G.owner[k]) (void)hipFree(G.owner[k]);
  }
  for (Problem& p : h->probs) {
    if (p.geom) (void)hipFree(p.geom);
    void* bufs[kBufs] = {p.W, p.FX, p.FY, p.PC, p.FLX, p.FLY, p.scal};
    for (int b = p.borrowed ? 3 : 0; b < kBufs; ++b)
      if (bufs[b]) (void)hipFree(bufs[b]);
  }
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return GKS_OK;
}

const char* gks_last_error(const gks_handle* h) { return h ? h->msg.c_str() : g_init_msg.c_str(); }

int gks_profile(gks_handle* h, int32_t mode) {
  if (!h || mode < 0 || mode > 2) return GKS_EINVAL;
  if (mode == 2) {
    HIP_OR(h, hipStreamSynchronize(h->stream));
    collect(h);
    for (int k = 0; k < GKS_K_COUNT; ++k) {
      h->ktime[k] = 0.0;
      h->klaunch[k] = 0;
    }
    return GKS_OK;
  }
  h->profiling = mode;
  return GKS_OK;
}

int gks_kernel_time(gks_handle* h, int32_t kernel, double* ms, int64_t* launches) {
  if (!h || kernel < 0 || kernel >= GKS_K_COUNT) return GKS_EINVAL;
  HIP_OR(h, hipStreamSynchronize(h->stream));
  collect(h);
  if (ms) *ms = h->ktime[kernel];
  if (launches) *launches = h->klaunch[kernel];
  return GKS_OK;
}

}  // extern "C"
