// gks.hip -- kernels and C-ABI host library of the compact third-order
// gas-kinetic scheme (Pan & Xu, arXiv:1412.4489) for MI355X (gfx950).
//
// Per problem and step (all on one HIP stream, no host synchronisation):
//   k_ghost_we / k_ghost_sn  boundary images (cells: two layers incl. corners;
//                            interface point values of the edge ghost cells)
//   k_dt / k_set_dt          CFL time step (one block) or the fixed step
//   k_recon_2d               compact reconstruction of interior and edge
//                            ghost cells -> p2..p6 per variable (Sec. 3.2)
//   k_interfaces_2d          every x and y interface: flux and new point values
//                            (Sec. 2.2, 3.3, 4)
//   k_update_2d              conservative update (eq. finite), nonphysical-state
//                            flag, time and step counters
//
// Memory (per problem, structure of arrays, x fastest):
//   W  double [4][ny+4][nx+4]           cell averages with two ghost layers
//   FX TS     [2][4][ny+2][nx+3]        x-interface Gauss values, interfaces -1..nx+1, rows -1..ny
//   FY TS     [2][4][ny+3][nx+2]        y-interface Gauss values, interfaces -1..ny+1, cols -1..nx
//   PC TP     [4][5][ny+2][nx+2]        reconstruction coefficients, cells -1..nx
//   FLX double [4][ny][nx+1], FLY double [4][ny+1][nx]  integrated fluxes
// TS = TP = double (GKS_FP64) or float (GKS_FP32_MIXED).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

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
  __device__ __host__ size_t w(int v, int j, int i) const {
    return ((size_t)v * (ny + 4) + (size_t)(j + 2)) * (nx + 4) + (size_t)(i + 2);
  }
  __device__ __host__ size_t fx(int g, int v, int j, int fi) const {
    return (((size_t)g * 4 + v) * (ny + 2) + (size_t)(j + 1)) * (nx + 3) + (size_t)(fi + 1);
  }
  __device__ __host__ size_t fy(int g, int v, int fj, int i) const {
    return (((size_t)g * 4 + v) * (ny + 3) + (size_t)(fj + 1)) * (nx + 2) + (size_t)(i + 1);
  }
  __device__ __host__ size_t pc(int v, int m, int j, int i) const {
    return (((size_t)v * 5 + m) * (ny + 2) + (size_t)(j + 1)) * (nx + 2) + (size_t)(i + 1);
  }
  __device__ __host__ size_t flx(int v, int j, int fi) const { return ((size_t)v * ny + j) * (nx + 1) + fi; }
  __device__ __host__ size_t fly(int v, int fj, int i) const { return ((size_t)v * (ny + 1) + fj) * nx + i; }
  size_t nW() const { return (size_t)4 * (ny + 4) * (nx + 4); }
  size_t nFX() const { return (size_t)2 * 4 * (ny + 2) * (nx + 3); }
  size_t nFY() const { return (size_t)2 * 4 * (ny + 3) * (nx + 2); }
  size_t nPC() const { return (size_t)4 * 5 * (ny + 2) * (nx + 2); }
  size_t nFLX() const { return (size_t)4 * ny * (nx + 1); }
  size_t nFLY() const { return (size_t)4 * (ny + 1) * nx; }
};

struct BCDev {
  int kind;
  double state[4];  // conservative
  double alt[4];    // conservative
  double wu, wv, wT;
};

struct Geo {
  double x0, y0, h, k;
};

template <typename TS, typename TP>
struct Grid {
  Idx ix;
  Geo geo;
  double* W;
  TS* FX;
  TS* FY;
  TP* PC;
  double* FLX;
  double* FLY;
  double* t;      // time
  double* dt;     // step of the current step
  long long* steps;
  unsigned long long* err;
  unsigned long long* dtmin;  // running minimum of the CFL bound (double bits)  // 0, or 1 + (j+1) * 65536 * 65536 + (i+1) * 65536 ... of the first bad cell
};

// ---------------------------------------------------------------------------
// boundary images
// ---------------------------------------------------------------------------

// fixed state at location (x, y) at time t; false where the boundary mirrors
__device__ bool bc_fixed(const BCDev& b, double x, double y, double t, double* out) {
  if (b.kind == GKS_BC_INFLOW) {
    for (int v = 0; v < 4; ++v) out[v] = b.state[v];
    return true;
  }
  if (b.kind == GKS_BC_DMR_BOTTOM) {
    if (!(x < 1.0 / 6.0)) return false;
    for (int v = 0; v < 4; ++v) out[v] = b.state[v];
    return true;
  }
  if (b.kind == GKS_BC_DMR_TOP) {
    const double xs = 1.0 / 6.0 + (y + 20.0 * t) * 0.57735026918962576451;
    const double* src = x < xs ? b.state : b.alt;
    for (int v = 0; v < 4; ++v) out[v] = src[v];
    return true;
  }
  return false;
}

// mirror image of a state across a boundary with normal `axis`
__device__ void bc_mirror(const BCDev& b, int axis, double gamma, const double* s, double* o) {
  for (int v = 0; v < 4; ++v) o[v] = s[v];
  const int kind = b.kind;
  if (kind == GKS_BC_REFLECT || kind == GKS_BC_DMR_BOTTOM) {
    o[1 + axis] = -s[1 + axis];
  } else if (kind == GKS_BC_NOSLIP_ISOTHERMAL || kind == GKS_BC_NOSLIP_ADIABATIC) {
    const double rho = s[0], u = s[1] / rho, v = s[2] / rho;
    const double p = (gamma - 1.0) * (s[3] - 0.5 * rho * (u * u + v * v));
    const double T = p / rho;
    const double Tg = kind == GKS_BC_NOSLIP_ISOTHERMAL ? 2.0 * b.wT - T : T;
    const double ug = 2.0 * b.wu - u, vg = 2.0 * b.wv - v;
    o[0] = rho;
    o[1] = rho * ug;
    o[2] = rho * vg;
    o[3] = rho * Tg / (gamma - 1.0) + 0.5 * rho * (ug * ug + vg * vg);
  }
}

// West (side 0) / east (side 1): ghost cells of rows 0..ny-1, ghost x
// interfaces -1 / nx+1, and the y interfaces of the ghost columns -1 / nx.
template <typename TS, typename TP>
__global__ void k_ghost_we(Grid<TS, TP> g, BCDev bw, BCDev be, double gamma) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int ncell = 2 * ny * 2, nfx = 2 * ny * 2, nfy = 2 * (ny + 1) * 2;
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ncell + nfx + nfy) return;
  const double t = *g.t, h = g.geo.h, k = g.geo.k;
  double src[4], out[4];
  if (id < ncell) {
    const int side = id / (2 * ny), r = id % (2 * ny), j = r / 2, m = r % 2;
    const BCDev& b = side == 0 ? bw : be;
    const int ig = side == 0 ? -1 - m : nx + m;
    const double xc = g.geo.x0 + (ig + 0.5) * h, yc = g.geo.y0 + (j + 0.5) * k;
    if (!bc_fixed(b, xc, yc, t, out)) {
      int is;
      if (b.kind == GKS_BC_PERIODIC)
        is = side == 0 ? ig + nx : ig - nx;
      else
        is = side == 0 ? -1 - ig : 2 * nx - 1 - ig;
      for (int v = 0; v < 4; ++v) src[v] = g.W[g.ix.w(v, j, is)];
      if (b.kind == GKS_BC_PERIODIC)
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      else
        bc_mirror(b, 0, gamma, src, out);
    }
    for (int v = 0; v < 4; ++v) g.W[g.ix.w(v, j, ig)] = out[v];
    return;
  }
  id -= ncell;
  if (id < nfx) {
    const int side = id / (2 * ny), r = id % (2 * ny), j = r / 2, gp = r % 2;
    const BCDev& b = side == 0 ? bw : be;
    const int fg = side == 0 ? -1 : nx + 1;
    const double xg = g.geo.x0 + fg * h, yg = g.geo.y0 + (j + 0.5 + (gp ? kGaussOffset : -kGaussOffset)) * k;
    if (!bc_fixed(b, xg, yg, t, out)) {
      const int fs = b.kind == GKS_BC_PERIODIC ? (side == 0 ? nx - 1 : 1) : (side == 0 ? 1 : nx - 1);
      for (int v = 0; v < 4; ++v) src[v] = (double)g.FX[g.ix.fx(gp, v, j, fs)];
      if (b.kind == GKS_BC_PERIODIC)
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      else
        bc_mirror(b, 0, gamma, src, out);
    }
    for (int v = 0; v < 4; ++v) g.FX[g.ix.fx(gp, v, j, fg)] = (TS)out[v];
    return;
  }
  id -= nfx;
  {
    const int side = id / (2 * (ny + 1)), r = id % (2 * (ny + 1)), fj = r / 2, gp = r % 2;
    const BCDev& b = side == 0 ? bw : be;
    const int ig = side == 0 ? -1 : nx;
    const double xg = g.geo.x0 + (ig + 0.5 + (gp ? kGaussOffset : -kGaussOffset)) * h, yg = g.geo.y0 + fj * k;
    if (!bc_fixed(b, xg, yg, t, out)) {
      const bool per = b.kind == GKS_BC_PERIODIC;
      const int is = per ? (side == 0 ? nx - 1 : 0) : (side == 0 ? 0 : nx - 1);
      const int gs = per ? gp : 1 - gp;  // a mirror swaps the tangential Gauss points
      for (int v = 0; v < 4; ++v) src[v] = (double)g.FY[g.ix.fy(gs, v, fj, is)];
      if (per)
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      else
        bc_mirror(b, 0, gamma, src, out);
    }
    for (int v = 0; v < 4; ++v) g.FY[g.ix.fy(gp, v, fj, ig)] = (TS)out[v];
  }
}

// South (side 2) / north (side 3): ghost cells of columns -2..nx+1 (corners
// from the west/east images), ghost y interfaces -1 / ny+1, and the x
// interfaces of the ghost rows -1 / ny.
template <typename TS, typename TP>
__global__ void k_ghost_sn(Grid<TS, TP> g, BCDev bs, BCDev bn, double gamma) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int ncell = 2 * (nx + 4) * 2, nfy = 2 * nx * 2, nfx = 2 * (nx + 1) * 2;
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ncell + nfy + nfx) return;
  const double t = *g.t, h = g.geo.h, k = g.geo.k;
  double src[4], out[4];
  if (id < ncell) {
    const int side = id / (2 * (nx + 4)), r = id % (2 * (nx + 4)), i = r / 2 - 2, m = r % 2;
    const BCDev& b = side == 0 ? bs : bn;
    const int jg = side == 0 ? -1 - m : ny + m;
    const double xc = g.geo.x0 + (i + 0.5) * h, yc = g.geo.y0 + (jg + 0.5) * k;
    if (!bc_fixed(b, xc, yc, t, out)) {
      int js;
      if (b.kind == GKS_BC_PERIODIC)
        js = side == 0 ? jg + ny : jg - ny;
      else
        js = side == 0 ? -1 - jg : 2 * ny - 1 - jg;
      for (int v = 0; v < 4; ++v) src[v] = g.W[g.ix.w(v, js, i)];
      if (b.kind == GKS_BC_PERIODIC)
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      else
        bc_mirror(b, 1, gamma, src, out);
    }
    for (int v = 0; v < 4; ++v) g.W[g.ix.w(v, jg, i)] = out[v];
    return;
  }
  id -= ncell;
  if (id < nfy) {
    const int side = id / (2 * nx), r = id % (2 * nx), i = r / 2, gp = r % 2;
    const BCDev& b = side == 0 ? bs : bn;
    const int fg = side == 0 ? -1 : ny + 1;
    const double xg = g.geo.x0 + (i + 0.5 + (gp ? kGaussOffset : -kGaussOffset)) * h, yg = g.geo.y0 + fg * k;
    if (!bc_fixed(b, xg, yg, t, out)) {
      const int fs = b.kind == GKS_BC_PERIODIC ? (side == 0 ? ny - 1 : 1) : (side == 0 ? 1 : ny - 1);
      for (int v = 0; v < 4; ++v) src[v] = (double)g.FY[g.ix.fy(gp, v, fs, i)];
      if (b.kind == GKS_BC_PERIODIC)
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      else
        bc_mirror(b, 1, gamma, src, out);
    }
    for (int v = 0; v < 4; ++v) g.FY[g.ix.fy(gp, v, fg, i)] = (TS)out[v];
    return;
  }
  id -= nfy;
  {
    const int side = id / (2 * (nx + 1)), r = id % (2 * (nx + 1)), fi = r / 2, gp = r % 2;
    const BCDev& b = side == 0 ? bs : bn;
    const int jg = side == 0 ? -1 : ny;
    const double xg = g.geo.x0 + fi * h, yg = g.geo.y0 + (jg + 0.5 + (gp ? kGaussOffset : -kGaussOffset)) * k;
    if (!bc_fixed(b, xg, yg, t, out)) {
      const bool per = b.kind == GKS_BC_PERIODIC;
      const int js = per ? (side == 0 ? ny - 1 : 0) : (side == 0 ? 0 : ny - 1);
      const int gs = per ? gp : 1 - gp;
      for (int v = 0; v < 4; ++v) src[v] = (double)g.FX[g.ix.fx(gs, v, js, fi)];
      if (per)
        for (int v = 0; v < 4; ++v) out[v] = src[v];
      else
        bc_mirror(b, 1, gamma, src, out);
    }
    for (int v = 0; v < 4; ++v) g.FX[g.ix.fx(gp, v, jg, fi)] = (TS)out[v];
  }
}

// ---------------------------------------------------------------------------
// time step: dt = cfl * min over cells of min(h/(|u|+c+2nu/h), k/(|v|+c+2nu/k))
// The per-cell bound is reduced into g.dtmin (bits of a positive double,
// ordered like unsigned integers) by k_update_2d for the next step, and by
// k_dt_scan for the initial state; k_dt_finalize turns it into the step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cell_dt_bound(const double* W, const Phys& P, double h, double k) {
  const double rho = W[0], u = W[1] / rho, v = W[2] / rho;
  const double p = (P.gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v));
  const double cs = sqrt(P.gamma * p / rho);
  const double nu = P.viscous ? P.mu / rho : 0.0;
  return fmin(h / (fabs(u) + cs + 2.0 * nu / h), k / (fabs(v) + cs + 2.0 * nu / k));
}

// wave minimum of a positive bound, one atomic per wave (NaN bounds of a
// nonphysical cell are skipped; the update flags that cell)
__device__ __forceinline__ void reduce_dt_bound(double b, unsigned long long* slot) {
  if (!(b > 0.0) || !isfinite(b)) b = 1e300;
  for (int off = 32; off > 0; off >>= 1) b = fmin(b, __shfl_down(b, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMin(slot, (unsigned long long)__double_as_longlong(b));
}

template <typename TS, typename TP>
__global__ void __launch_bounds__(256) k_dt_scan(Grid<TS, TP> g, Phys P) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  double b = 1e300;
  if (c < nx * ny) {
    const int j = c / nx, i = c % nx;
    double W[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) W[v] = g.W[g.ix.w(v, j, i)];
    b = cell_dt_bound(W, P, g.geo.h, g.geo.k);
  }
  reduce_dt_bound(b, g.dtmin);
}

template <typename TS, typename TP>
__global__ void k_dt_finalize(Grid<TS, TP> g, double cfl, double t_end) {
  double dt = cfl * __longlong_as_double((long long)*g.dtmin);
  if (t_end > 0.0) dt = fmin(dt, fmax(t_end - *g.t, 0.0));
  *g.dt = dt;
  *g.dtmin = (unsigned long long)__double_as_longlong(1e300);
}

template <typename TS, typename TP>
__global__ void k_set_dt(Grid<TS, TP> g, double dt, double t_end) {
  if (t_end > 0.0) dt = fmin(dt, fmax(t_end - *g.t, 0.0));
  *g.dt = dt;
  *g.dtmin = (unsigned long long)__double_as_longlong(1e300);
}

// ---------------------------------------------------------------------------
// reconstruction: cells -1..nx x -1..ny except the four corners
// ---------------------------------------------------------------------------
template <typename TS, typename TP>
__global__ void __launch_bounds__(256) k_recon_2d(Grid<TS, TP> g, double eps, double Cw, double gamma) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x) - 1;
  const int j = (int)blockIdx.y - 1;
  if (i > nx) return;
  if ((i < 0 || i >= nx) && (j < 0 || j >= ny)) return;
  const double h = g.geo.h, k = g.geo.k;
  const Idx& x = g.ix;
  double p[4][5], Wc[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    Wc[v] = g.W[x.w(v, j, i)];
    recon_2d(Wc[v], g.W[x.w(v, j, i + 1)], g.W[x.w(v, j, i - 1)], g.W[x.w(v, j + 1, i)], g.W[x.w(v, j - 1, i)],
             (double)g.FX[x.fx(1, v, j, i + 1)], (double)g.FX[x.fx(0, v, j, i + 1)], (double)g.FX[x.fx(1, v, j, i)],
             (double)g.FX[x.fx(0, v, j, i)], (double)g.FY[x.fy(1, v, j + 1, i)], (double)g.FY[x.fy(0, v, j + 1, i)],
             (double)g.FY[x.fy(1, v, j, i)], (double)g.FY[x.fy(0, v, j, i)], h, k, eps, Cw, p[v]);
  }
  // a polynomial that is nonphysical at the centre of one of the cell's
  // interfaces is replaced by the constant cell average for this step
  const bool ok = recon_admissible_2d(Wc, p, h, k, gamma);
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int m = 0; m < 5; ++m) g.PC[x.pc(v, m, j, i)] = ok ? (TP)p[v][m] : TP(0);
}

// ---------------------------------------------------------------------------
// interfaces: one thread per interface, x interfaces first, then y
// interfaces; three phase kernels (prologue, hydrodynamic part, kinetic part
// of each side) communicating through the frame record R.
// ---------------------------------------------------------------------------
struct Face {
  bool isx;   // x interface (else y)
  int a, b;   // x: (j, fi); y: (fj, i)
};

__device__ __forceinline__ Face face_of(const Idx& x, int id) {
  const int nfx = (x.nx + 1) * x.ny;
  Face F;
  F.isx = id < nfx;
  if (F.isx) {
    F.a = id / (x.nx + 1);
    F.b = id % (x.nx + 1);
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

template <typename TS, typename TP, typename TC>
__global__ void __launch_bounds__(256) k_iface_pro_2d(Grid<TS, TP> g, Phys P, Rec<TC> R) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int nf = (nx + 1) * ny + nx * (ny + 1);
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nf) return;
  const double dt = *g.dt;
  if (!(dt > 0.0)) return;
  const Idx& x = g.ix;
  const Face F = face_of(x, id);
  double Wc[2][4], pc[2][4][5], Ueq[2][3][4], flux[4], pv[4];
  if (F.isx) {
    const int j = F.a, fi = F.b;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int ic = fi - 1 + s;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Wc[s][v] = g.W[x.w(v, j, ic)];
        pc[s][v][0] = (double)g.PC[x.pc(v, 0, j, ic)];  // p_n  = p2
        pc[s][v][1] = (double)g.PC[x.pc(v, 1, j, ic)];  // p_s  = p3
        pc[s][v][2] = (double)g.PC[x.pc(v, 2, j, ic)];  // p_nn = p4
        pc[s][v][3] = (double)g.PC[x.pc(v, 3, j, ic)];  // p_ss = p5
        pc[s][v][4] = (double)g.PC[x.pc(v, 4, j, ic)];  // p_ns = p6
      }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int v = 0; v < 4; ++v) Ueq[m][n][v] = g.W[x.w(v, j - 1 + n, fi - 1 + m)];
  } else {
    const int fj = F.a, i = F.b;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int jc = fj - 1 + s;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int vl = loc(false, v);
        Wc[s][vl] = g.W[x.w(v, jc, i)];
        pc[s][vl][0] = (double)g.PC[x.pc(v, 1, jc, i)];  // p_n  = p3
        pc[s][vl][1] = (double)g.PC[x.pc(v, 0, jc, i)];  // p_s  = p2
        pc[s][vl][2] = (double)g.PC[x.pc(v, 3, jc, i)];  // p_nn = p5
        pc[s][vl][3] = (double)g.PC[x.pc(v, 2, jc, i)];  // p_ss = p4
        pc[s][vl][4] = (double)g.PC[x.pc(v, 4, jc, i)];  // p_ns = p6
      }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int v = 0; v < 4; ++v) Ueq[m][n][loc(false, v)] = g.W[x.w(v, fj - 1 + m, i - 1 + n)];
  }
  const double hn = F.isx ? g.geo.h : g.geo.k, hs = F.isx ? g.geo.k : g.geo.h;
  const bool ok = iface_prologue_2d<TC>(P, dt, hn, hs, Wc, pc, Ueq, R, (size_t)id, flux, pv);
  if (!ok) {
    R.D(D_RHO0, id) = 0.0;  // marks the record invalid for the later phases
    atomicCAS(g.err, 0ull,
              1ull + ((unsigned long long)(F.a + 1) << 32) + (unsigned long long)(F.b + 1) + (F.isx ? 0ull : 1ull << 62));
#pragma unroll
    for (int v = 0; v < 4; ++v) flux[v] = pv[v] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int vl = loc(F.isx, v);
    if (F.isx) {
      g.FLX[x.flx(v, F.a, F.b)] = flux[vl];
      g.FX[x.fx(0, v, F.a, F.b)] = (TS)pv[vl];
      g.FX[x.fx(1, v, F.a, F.b)] = (TS)pv[vl];
    } else {
      g.FLY[x.fly(v, F.a, F.b)] = flux[vl];
      g.FY[x.fy(0, v, F.a, F.b)] = (TS)pv[vl];
      g.FY[x.fy(1, v, F.a, F.b)] = (TS)pv[vl];
    }
  }
}

// adds interface-frame corrections to the stored flux and point values
template <typename TS, typename TP>
__device__ __forceinline__ void add_corrections(Grid<TS, TP>& g, const Face& F, const double (&flux)[4],
                                                const double (&pvm)[4], const double (&pvp)[4]) {
  const Idx& x = g.ix;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int vl = loc(F.isx, v);
    if (F.isx) {
      g.FLX[x.flx(v, F.a, F.b)] += flux[vl];
      TS* a = &g.FX[x.fx(0, v, F.a, F.b)];
      TS* b = &g.FX[x.fx(1, v, F.a, F.b)];
      *a = (TS)((double)*a + pvm[vl]);
      *b = (TS)((double)*b + pvp[vl]);
    } else {
      g.FLY[x.fly(v, F.a, F.b)] += flux[vl];
      TS* a = &g.FY[x.fy(0, v, F.a, F.b)];
      TS* b = &g.FY[x.fy(1, v, F.a, F.b)];
      *a = (TS)((double)*a + pvm[vl]);
      *b = (TS)((double)*b + pvp[vl]);
    }
  }
}

template <typename TS, typename TP, typename TC>
__global__ void __launch_bounds__(256) k_iface_hydro_2d(Grid<TS, TP> g, Phys P, Rec<TC> R) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int nf = (nx + 1) * ny + nx * (ny + 1);
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nf) return;
  if (!(*g.dt > 0.0) || !(R.D(D_RHO0, id) > 0.0)) return;
  const Face F = face_of(g.ix, id);
  const double hs = F.isx ? g.geo.k : g.geo.h;
  double flux[4], pvm[4], pvp[4], E[4];
  iface_hydro_2d<TC>(P, hs, R, (size_t)id, flux, pvm, pvp, E);
  add_corrections(g, F, flux, pvm, pvp);
  if (P.viscous)
#pragma unroll
    for (int v = 0; v < 4; ++v) R.D(D_E0 + v, id) += E[v];
}

template <typename TS, typename TP, typename TC>
__global__ void __launch_bounds__(256) k_iface_kin_2d(Grid<TS, TP> g, Phys P, Rec<TC> R, int side) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int nf = (nx + 1) * ny + nx * (ny + 1);
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nf) return;
  if (!(*g.dt > 0.0) || !(R.D(D_RHO0, id) > 0.0)) return;
  const Face F = face_of(g.ix, id);
  const double hs = F.isx ? g.geo.k : g.geo.h;
  double flux[4], pvm[4], pvp[4], E[4];
  iface_kinetic_2d<TC>(P, hs, side, R, (size_t)id, flux, pvm, pvp, E);
  add_corrections(g, F, flux, pvm, pvp);
  if (P.viscous) {
#pragma unroll
    for (int v = 0; v < 4; ++v) R.D(D_E0 + v, id) += E[v];
    if (side == 1) {
      // Prandtl-number fix on the complete flux: energy flux += (1/Pr - 1) q,
      // q the heat flux relative to the velocity of g0 (interface frame)
      const Idx& x = g.ix;
      double Fl[4], Ed[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Fl[loc(F.isx, v)] = F.isx ? g.FLX[x.flx(v, F.a, F.b)] : g.FLY[x.fly(v, F.a, F.b)];
        Ed[v] = R.D(D_E0 + v, id);
      }
      const double U0 = R.D(D_U0, id), V0 = R.D(D_V0, id), k2 = 0.5 * (U0 * U0 + V0 * V0);
      const double qh = Fl[3] - U0 * Fl[1] - V0 * Fl[2] + k2 * Fl[0] - U0 * (Ed[3] - U0 * Ed[1] - V0 * Ed[2] + k2 * Ed[0]);
      if (F.isx)
        g.FLX[x.flx(3, F.a, F.b)] += P.prfix * qh;
      else
        g.FLY[x.fly(3, F.a, F.b)] += P.prfix * qh;
    }
  }
}

// ---------------------------------------------------------------------------
// conservative update
// ---------------------------------------------------------------------------
template <typename TS, typename TP>
__global__ void __launch_bounds__(256) k_update_2d(Grid<TS, TP> g, Phys P) {
  const int nx = g.ix.nx, ny = g.ix.ny;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  const double dt = *g.dt;
  double bound = 1e300;
  if (i < nx) {
    const Idx& x = g.ix;
    double W[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) W[v] = g.W[x.w(v, j, i)];
    if (dt > 0.0) {
      const double ia = 1.0 / (g.geo.h * g.geo.k);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double d = g.FLX[x.flx(v, j, i)] - g.FLX[x.flx(v, j, i + 1)] + g.FLY[x.fly(v, j, i)] -
                         g.FLY[x.fly(v, j + 1, i)];
        W[v] += d * ia;
        g.W[x.w(v, j, i)] = W[v];
      }
      const double p = (P.gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0]);
      if (!(W[0] > 0.0) || !(p > 0.0) || !isfinite(p))
        atomicCAS(g.err, 0ull,
                  1ull + ((unsigned long long)(j + 1) << 32) + (unsigned long long)(i + 1) + (1ull << 63));
      if (i == 0 && j == 0) {
        *g.t += dt;
        *g.steps += 1;
      }
    }
    bound = cell_dt_bound(W, P, g.geo.h, g.geo.k);
  }
  reduce_dt_bound(bound, g.dtmin);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

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
  void* scal = nullptr;  // t, dt, steps, err
  void* recd = nullptr;  // interface frame record, double fields
  void* rect = nullptr;  // interface frame record, compute-type fields
};

}  // namespace

struct gks_handle {
  std::vector<Problem> probs;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int sticky = GKS_OK;
  std::string msg;
  int profiling = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  double ktime[GKS_K_COUNT] = {0};
  long long klaunch[GKS_K_COUNT] = {0};
  std::vector<hipEvent_t> pend_a, pend_b;
  std::vector<int> pend_k;
};

namespace {

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
  if (p.dim != 2) return "only dim == 2 is available in this build";
  if (p.nx < 2 || p.ny < 2) return "nx, ny must be >= 2";
  if ((long long)(p.nx + 4) * (p.ny + 4) > (1ll << 30)) return "grid too large";
  if (!(p.x1 > p.x0) || !(p.y1 > p.y0)) return "empty domain";
  if (!(p.gamma > 1.0) || !(p.gamma < 3.0)) return "gamma must lie in (1, 3)";
  if (!(internal_dof(p.dim, p.gamma) >= 0.0)) return "gamma gives negative internal degrees of freedom";
  if (p.viscous && !(p.mu >= 0.0 && p.prandtl > 0.0)) return "mu >= 0 and prandtl > 0 required";
  if (!(p.cfl > 0.0) || !(p.weno_eps > 0.0) || !(p.weno_c >= 0.0)) return "cfl, weno_eps must be > 0";
  if (!(p.tau_eps >= 0.0) || !(p.tau_c >= 0.0)) return "tau constants must be >= 0";
  if (!std::isfinite(p.t0)) return "t0 must be finite";
  if (p.recon_vars != 0) return "2D reconstruction is in conservative variables (recon_vars = 0)";
  if (p.precision != GKS_FP64 && p.precision != GKS_FP32_MIXED) return "unknown precision";
  for (int s = 0; s < 4; ++s) {
    const int k = p.bc[s].kind;
    if (k < GKS_BC_PERIODIC || k > GKS_BC_DMR_TOP) return "unknown boundary kind";
    if ((k == GKS_BC_PERIODIC) != (p.bc[s ^ 1].kind == GKS_BC_PERIODIC)) return "periodic sides must pair";
    if (k == GKS_BC_DMR_BOTTOM && s != 2) return "dmr_bottom only on the south side";
    if (k == GKS_BC_DMR_TOP && s != 3) return "dmr_top only on the north side";
  }
  return "";
}

size_t n_interfaces(const Idx& x) { return (size_t)(x.nx + 1) * x.ny + (size_t)x.nx * (x.ny + 1); }

template <typename TC>
Rec<TC> rec_of(Problem& p) {
  Rec<TC> r;
  r.d = (double*)p.recd;
  r.t = (TC*)p.rect;
  r.nf = n_interfaces(p.ix);
  return r;
}

template <typename TS, typename TP>
Grid<TS, TP> grid_of(Problem& p) {
  Grid<TS, TP> g;
  g.ix = p.ix;
  g.geo = p.geo;
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
  g.dtmin = (unsigned long long*)(s + 4);
  return g;
}

unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

int record_begin(gks_handle* h) {
  if (h->profiling != 1) return 0;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
  (void)hipEventRecord(a, h->stream);
  h->pend_a.push_back(a);
  h->pend_b.push_back(b);
  return 0;
}
void record_end(gks_handle* h, int kernel) {
  if (h->profiling != 1) return;
  (void)hipEventRecord(h->pend_b.back(), h->stream);
  h->pend_k.push_back(kernel);
}

void collect(gks_handle* h) {
  for (size_t n = 0; n < h->pend_k.size(); ++n) {
    float ms = 0.f;
    (void)hipEventSynchronize(h->pend_b[n]);
    (void)hipEventElapsedTime(&ms, h->pend_a[n], h->pend_b[n]);
    h->ktime[h->pend_k[n]] += ms;
    h->klaunch[h->pend_k[n]] += 1;
    (void)hipEventDestroy(h->pend_a[n]);
    (void)hipEventDestroy(h->pend_b[n]);
  }
  h->pend_a.clear();
  h->pend_b.clear();
  h->pend_k.clear();
}

template <typename TS, typename TP, typename TC>
int step_problem(gks_handle* h, Problem& p, const double* dtf, double t_end) {
  Grid<TS, TP> g = grid_of<TS, TP>(p);
  const int nx = p.ix.nx, ny = p.ix.ny;
  hipStream_t st = h->stream;
  record_begin(h);
  {
    const int n1 = 4 * ny + 4 * ny + 4 * (ny + 1);
    k_ghost_we<TS, TP><<<cdiv(n1, 256), 256, 0, st>>>(g, p.bc[0], p.bc[1], p.phys.gamma);
    const int n2 = 4 * (nx + 4) + 4 * nx + 4 * (nx + 1);
    k_ghost_sn<TS, TP><<<cdiv(n2, 256), 256, 0, st>>>(g, p.bc[2], p.bc[3], p.phys.gamma);
  }
  record_end(h, GKS_K_GHOST);
  record_begin(h);
  if (dtf)
    k_set_dt<TS, TP><<<1, 1, 0, st>>>(g, *dtf, t_end);
  else
    k_dt_finalize<TS, TP><<<1, 1, 0, st>>>(g, p.phys.cfl, t_end);
  record_end(h, GKS_K_DT);
  record_begin(h);
  k_recon_2d<TS, TP><<<dim3(cdiv(nx + 2, 256), ny + 2), 256, 0, st>>>(g, p.phys.weno_eps, p.phys.weno_c,
                                                                         p.phys.gamma);
  record_end(h, GKS_K_RECON);
  record_begin(h);
  {
    const size_t nf = n_interfaces(p.ix);
    Rec<TC> R = rec_of<TC>(p);
    k_iface_pro_2d<TS, TP, TC><<<cdiv(nf, 256), 256, 0, st>>>(g, p.phys, R);
    k_iface_hydro_2d<TS, TP, TC><<<cdiv(nf, 256), 256, 0, st>>>(g, p.phys, R);
    k_iface_kin_2d<TS, TP, TC><<<cdiv(nf, 256), 256, 0, st>>>(g, p.phys, R, 0);
    k_iface_kin_2d<TS, TP, TC><<<cdiv(nf, 256), 256, 0, st>>>(g, p.phys, R, 1);
  }
  record_end(h, GKS_K_INTERFACE);
  record_begin(h);
  k_update_2d<TS, TP><<<dim3(cdiv(nx, 256), ny), 256, 0, st>>>(g, p.phys);
  record_end(h, GKS_K_UPDATE);
  HIP_OR(h, hipGetLastError());
  return GKS_OK;
}

}  // namespace

extern "C" {

int gks_init(gks_handle** out, int32_t n_problems, const gks_problem* probs, const double* const* cell,
             const double* const* face_x, const double* const* face_y, void* stream) {
  if (!out) return GKS_EINVAL;
  *out = nullptr;
  if (n_problems < 1 || !probs || !cell || !face_x) return GKS_EINVAL;
  gks_handle* h = new (std::nothrow) gks_handle();
  if (!h) return GKS_ENOMEM;
  h->probs.resize(n_problems);
  for (int n = 0; n < n_problems; ++n) {
    const gks_problem& s = probs[n];
    std::string why = validate(s);
    if (!why.empty() || !cell[n] || !face_x[n] || (s.dim == 2 && (!face_y || !face_y[n]))) {
      int rc = fail(h, GKS_EINVAL, "problem " + std::to_string(n) + ": " + (why.empty() ? "null array" : why));
      g_init_msg = h->msg;
      gks_destroy(h);
      return rc;
    }
    Problem& p = h->probs[n];
    p.spec = s;
    p.mixed = s.precision == GKS_FP32_MIXED;
    p.ix = Idx{s.nx, s.ny};
    p.geo = Geo{s.x0, s.y0, (s.x1 - s.x0) / s.nx, (s.y1 - s.y0) / s.ny};
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
      b.kind = s.bc[side].kind;
      cons_of(s.dim, s.gamma, s.bc[side].state, b.state);
      cons_of(s.dim, s.gamma, s.bc[side].alt, b.alt);
      b.wu = s.bc[side].wall_u;
      b.wv = s.bc[side].wall_v;
      b.wT = s.bc[side].wall_T;
    }
    // initial state must be physical
    const size_t nc = (size_t)s.nx * s.ny;
    for (size_t c = 0; c < nc; ++c) {
      const double r = cell[n][c], mu_ = cell[n][nc + c], mv = cell[n][2 * nc + c], E = cell[n][3 * nc + c];
      const double pr = (s.gamma - 1.0) * (E - 0.5 * (mu_ * mu_ + mv * mv) / r);
      if (!(r > 0.0) || !(pr > 0.0) || !std::isfinite(pr)) {
        int rc = fail(h, GKS_EINVAL, "problem " + std::to_string(n) + ": nonphysical initial cell " +
                                         std::to_string(c));
        g_init_msg = h->msg;
        gks_destroy(h);
        return rc;
      }
    }
  }
  if (stream) {
    h->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
      gks_destroy(h);
      return GKS_EDEVICE;
    }
    h->own_stream = true;
  }
  for (int n = 0; n < n_problems; ++n) {
    Problem& p = h->probs[n];
    const size_t ts = p.mixed ? sizeof(float) : sizeof(double);
    const Idx& x = p.ix;
    const size_t nf = n_interfaces(x);
    void** bufs[9] = {&p.W, &p.FX, &p.FY, &p.PC, &p.FLX, &p.FLY, &p.scal, &p.recd, &p.rect};
    size_t sizes[9] = {x.nW() * 8, x.nFX() * ts, x.nFY() * ts, x.nPC() * ts, x.nFLX() * 8, x.nFLY() * 8, 64,
                       (size_t)ND_REC * nf * 8, (size_t)NT_REC * nf * ts};
    for (int b = 0; b < 9; ++b) {
      if (hipMalloc(bufs[b], sizes[b]) != hipSuccess) {
        *bufs[b] = nullptr;
        int rc = fail(h, GKS_ENOMEM, "device allocation failed");
        gks_destroy(h);
        return rc;
      }
      if (hipMemsetAsync(*bufs[b], 0, sizes[b], h->stream) != hipSuccess) {
        gks_destroy(h);
        return GKS_EDEVICE;
      }
    }
    // the clears above must land before the blocking uploads below
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
      gks_destroy(h);
      return GKS_EDEVICE;
    }
    // upload: host layouts without ghosts -> ghosted device layouts
    const gks_problem& s = p.spec;
    std::vector<double> W(x.nW(), 0.0);
    for (int v = 0; v < 4; ++v)
      for (int j = 0; j < s.ny; ++j)
        for (int i = 0; i < s.nx; ++i) W[x.w(v, j, i)] = cell[n][((size_t)v * s.ny + j) * s.nx + i];
    std::vector<double> FX(x.nFX(), 0.0), FY(x.nFY(), 0.0);
    for (int g = 0; g < 2; ++g)
      for (int v = 0; v < 4; ++v) {
        for (int j = 0; j < s.ny; ++j)
          for (int fi = 0; fi <= s.nx; ++fi)
            FX[x.fx(g, v, j, fi)] = face_x[n][(((size_t)g * 4 + v) * s.ny + j) * (s.nx + 1) + fi];
        for (int fj = 0; fj <= s.ny; ++fj)
          for (int i = 0; i < s.nx; ++i)
            FY[x.fy(g, v, fj, i)] = face_y[n][(((size_t)g * 4 + v) * (s.ny + 1) + fj) * s.nx + i];
      }
    const double scal0[4] = {s.t0, 0.0, 0.0, 0.0};
    if (hipMemcpy(p.scal, scal0, sizeof(scal0), hipMemcpyHostToDevice) != hipSuccess) {
      gks_destroy(h);
      return GKS_EDEVICE;
    }
    if (hipMemcpy(p.W, W.data(), W.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      gks_destroy(h);
      return GKS_EDEVICE;
    }
    if (p.mixed) {
      std::vector<float> fx(FX.begin(), FX.end()), fy(FY.begin(), FY.end());
      if (hipMemcpy(p.FX, fx.data(), fx.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(p.FY, fy.data(), fy.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        gks_destroy(h);
        return GKS_EDEVICE;
      }
    } else {
      if (hipMemcpy(p.FX, FX.data(), FX.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(p.FY, FY.data(), FY.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        gks_destroy(h);
        return GKS_EDEVICE;
      }
    }
  }
  // CFL bound of the initial state
  for (int n = 0; n < n_problems; ++n) {
    Problem& p = h->probs[n];
    const unsigned long long inf = (unsigned long long)0x7e37e43c8800759cull;  // bits of 1e300
    if (hipMemcpy((char*)p.scal + 32, &inf, 8, hipMemcpyHostToDevice) != hipSuccess) {
      gks_destroy(h);
      return GKS_EDEVICE;
    }
    const unsigned nb = cdiv((size_t)p.ix.nx * p.ix.ny, 256);
    if (p.mixed)
      k_dt_scan<float, float><<<nb, 256, 0, h->stream>>>(grid_of<float, float>(p), p.phys);
    else
      k_dt_scan<double, double><<<nb, 256, 0, h->stream>>>(grid_of<double, double>(p), p.phys);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
    gks_destroy(h);
    return GKS_EDEVICE;
  }
  *out = h;
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
  for (int s = 0; s < nsteps; ++s)
    for (size_t n = 0; n < h->probs.size(); ++n) {
      Problem& p = h->probs[n];
      const double* dtf = dt_fixed ? &dt_fixed[n] : nullptr;
      const double te = t_end ? t_end[n] : 0.0;
      int rc = p.mixed ? step_problem<float, float, float>(h, p, dtf, te)
                       : step_problem<double, double, double>(h, p, dtf, te);
      if (rc != GKS_OK) return rc;
    }
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
  if (cell) {
    std::vector<double> W(x.nW());
    HIP_OR(h, hipMemcpy(W.data(), p.W, W.size() * 8, hipMemcpyDeviceToHost));
    for (int v = 0; v < 4; ++v)
      for (int j = 0; j < s.ny; ++j)
        for (int i = 0; i < s.nx; ++i) cell[((size_t)v * s.ny + j) * s.nx + i] = W[x.w(v, j, i)];
  }
  if (face_x || face_y) {
    std::vector<double> FX(x.nFX()), FY(x.nFY());
    if (p.mixed) {
      std::vector<float> fx(x.nFX()), fy(x.nFY());
      HIP_OR(h, hipMemcpy(fx.data(), p.FX, fx.size() * 4, hipMemcpyDeviceToHost));
      HIP_OR(h, hipMemcpy(fy.data(), p.FY, fy.size() * 4, hipMemcpyDeviceToHost));
      FX.assign(fx.begin(), fx.end());
      FY.assign(fy.begin(), fy.end());
    } else {
      HIP_OR(h, hipMemcpy(FX.data(), p.FX, FX.size() * 8, hipMemcpyDeviceToHost));
      HIP_OR(h, hipMemcpy(FY.data(), p.FY, FY.size() * 8, hipMemcpyDeviceToHost));
    }
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
  if (err) {
    const int kind = (int)(err >> 62);
    const long long a = (long long)((err >> 32) & 0x3fffffff) - 1, b = (long long)(err & 0xffffffff) - 2;
    const char* where = kind == 2 ? "cell (i, j) = (" : kind == 1 ? "y interface (i, j) = (" : "x interface (i, j) = (";
    h->sticky = GKS_ENONPHYS;
    return fail(h, GKS_ENONPHYS, "problem " + std::to_string(problem) + ": nonphysical state at " + where +
                                     std::to_string(b) + ", " + std::to_string(a) + ")");
  }
  return h->sticky;
}

int gks_destroy(gks_handle* h) {
  if (!h) return GKS_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  collect(h);
  for (Problem& p : h->probs) {
    void* bufs[9] = {p.W, p.FX, p.FY, p.PC, p.FLX, p.FLY, p.scal, p.recd, p.rect};
    for (void* b : bufs)
      if (b) (void)hipFree(b);
  }
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
