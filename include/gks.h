/*
 * gks.h -- C ABI of the MI355X (gfx950) implementation of the compact
 * third-order gas-kinetic scheme of Pan & Xu, "A Compact Third-order
 * Gas-kinetic Scheme for Compressible Euler and Navier-Stokes Equations"
 * (arXiv:1412.4489).
 *
 * One time step of the scheme (a single stage, no Runge-Kutta; Sec. 1, 5):
 *   1. boundary images of the cell averages and interface point values;
 *   2. time step from the CFL condition (Sec. 4) unless a fixed one is given;
 *   3. compact reconstruction of every cell from its average, its face
 *      neighbours' averages and the tracked interface Gauss-point values
 *      (Sec. 3.1, 3.2: one-sided stencils, limiter eq. limiter, central
 *      stencil, nonlinear weights eq. average; optionally with the limiter
 *      in characteristic variables, Sec. 4: in 1D the whole reconstruction,
 *      in 2D the limited normal pair of each direction in the eigenvector
 *      basis of that direction's flux Jacobian at the cell average);
 *   4. at every interface: the equilibrium state U0 (eq. compatibility2), its
 *      quadratic (Sec. 3.3), the collision time (Sec. 4), the expansion
 *      coefficients (system after eq. dis3), the time- and interface-integrated
 *      flux (eq. finite with eq. dis1 + eq. dis2) and the point values at the
 *      next time level (eq. point);
 *   5. the conservative update (eq. finite).
 *
 * A handle advances any number of independent problems (1D and 2D, both
 * precisions, uneven sizes) together: every step is one launch per phase for
 * all problems of a dimension, precision and (2D) reconstruction kind,
 * replayed from one captured HIP graph.  Where the paper leaves the
 * reconstruction's robustness open (end of Sec. 3.3), a reconstructed cell
 * polynomial whose density or pressure at an interface centre is nonpositive
 * (or, with gks_problem.admissibility = 1, more than a factor two outside the
 * range of the neighbouring averages) is replaced by the constant average for
 * the step; gks_fallbacks counts those cells.
 *
 * Every call returns an int status (GKS_OK or a negative GKS_E* code); no C++
 * exception crosses the ABI.  All arrays are plain memory with the layouts
 * stated below; the library never keeps a pointer to caller memory after a
 * call returns.
 */
#ifndef GKS_H
#define GKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  GKS_OK = 0,
  GKS_EINVAL = -1,   /* invalid argument (checked before any device work) */
  GKS_ENOMEM = -2,   /* device allocation failed */
  GKS_EDEVICE = -3,  /* HIP runtime error */
  GKS_ENONPHYS = -4, /* a cell reached rho <= 0, p <= 0 or a non-finite value */
  GKS_ESTATE = -5    /* the handle is in an error state (call gks_destroy) */
};

/* arithmetic of the interface evaluation */
enum {
  GKS_FP64 = 0,       /* double precision throughout */
  GKS_FP32_MIXED = 1  /* single precision for the derivative (correction) terms of the
                         interface distribution and for the stored point values and
                         reconstruction; double for the cell averages, the conservative
                         accumulation, the equilibrium state U0, the leading flux terms
                         and the exponential time integrals */
};

/* boundary kinds (one per side W, E, S, N) */
enum {
  GKS_BC_PERIODIC = 0,
  GKS_BC_OUTFLOW = 1,             /* zero normal gradient (mirror image) */
  GKS_BC_REFLECT = 2,             /* slip wall: mirror image, normal momentum negated; its
                                     interfaces pass normal momentum only and their new point
                                     values carry no normal momentum (the symmetry line of the
                                     image pair; the south edge of GKS_BC_DMR_BOTTOM likewise
                                     where it mirrors) */
  GKS_BC_NOSLIP_ISOTHERMAL = 3,   /* ghost velocity 2 u_w - u, ghost temperature 2 T_w - T */
  GKS_BC_NOSLIP_ADIABATIC = 4,    /* ghost velocity 2 u_w - u, temperature mirrored.
                                     2D no-slip edges are impermeable: their interfaces pass
                                     no mass, and the momentum and energy that the mass flux
                                     of the ghost-image evaluation would carry (F_rho times the
                                     velocity and total enthalpy of the cell beside the wall,
                                     its average at the start of the step) are removed with it */
  GKS_BC_INFLOW = 5,              /* fixed primitive state `state` */
  GKS_BC_DMR_BOTTOM = 6,          /* `state` for x < 1/6, slip wall beyond (Sec. 4.5) */
  GKS_BC_DMR_TOP = 7              /* `state` behind the Mach-10 shock line
                                     x = 1/6 + (y + 20 t)/sqrt(3), `alt` ahead of it */
};

typedef struct {
  int32_t kind;
  double state[4]; /* primitive (rho, u, v, p) */
  double alt[4];   /* second primitive state (DMR pre-shock) */
  double wall_u, wall_v, wall_T;
  /* no-slip walls of a curvilinear grid (gks_problem.mesh) only: the wall
   * also turns about the origin at this angular velocity, its velocity at
   * the wall point (x, y) being (wall_u - wall_omega y, wall_v + wall_omega x)
   * (the turning inner wall of the polar cavity, Sec. 4.8); 0 elsewhere */
  double wall_omega;
} gks_bc;

/* The problem, as the paper states it: Euler or Navier-Stokes for
 * W = (rho, rho u, rho v, rho E) in 2D, (rho, rho u, rho E) in 1D (eq. finite);
 * gamma fixes the internal degrees of freedom K = (4 - 2 gamma)/(gamma - 1) in
 * 2D and (3 - gamma)/(gamma - 1) in 1D (Sec. 2.1); collision time
 * tau = tau_eps dt + tau_c |p_l - p_r|/(p_l + p_r) dt (Euler) or
 * mu/p + tau_c |p_l - p_r|/(p_l + p_r) dt (Navier-Stokes) (Sec. 4). */
typedef struct {
  int32_t dim;              /* 1 or 2 */
  int32_t nx, ny;           /* cells; ny = 1 when dim == 1 */
  double x0, x1, y0, y1;    /* domain [x0, x1] x [y0, y1] */
  double gamma;
  int32_t viscous;          /* 0 Euler, 1 Navier-Stokes */
  double mu, prandtl;       /* constant viscosity; Prandtl number (1 = plain BGK) */
  double tau_eps, tau_c;
  double cfl;               /* dt = cfl * min over cells of min(dx/(|u|+c+2nu/dx), dy/(|v|+c+2nu/dy)) */
  double weno_eps, weno_c;  /* small number and C of I(U1) = C h^2 in the weights */
  int32_t recon_vars;       /* 0: conservative variables; 1: characteristic (see step 3) */
  int32_t precision;        /* GKS_FP64 or GKS_FP32_MIXED */
  gks_bc bc[4];             /* W, E, S, N */
  double t0;                /* time of the initial state (restart from a fetched state) */
  /* 2D solid step in the lower right corner (Sec. 4.6, forward-facing step):
   * the cells i >= obstacle_i0, j < obstacle_nj; obstacle_nj = 0 for none,
   * else 2 <= obstacle_i0 <= nx - 4, 4 <= obstacle_nj <= ny - 3, and the east
   * and south boundaries of a mirror kind (outflow, reflect, no-slip).  Its
   * faces are slip walls.  Its cells take no part in the update, the CFL
   * condition or the nonphysical-state check: the two layers along its faces
   * (and the point values between them) hold slip-wall images of the gas,
   * refreshed every step, the others keep their initial values. */
  int32_t obstacle_i0, obstacle_nj;
  /* A reconstructed cell polynomial is used only if, at the centre of every
   * interface of the cell, density and pressure are positive (0: the
   * interface Maxwellians of Sec. 2.2 exist); 1: and also lie within a factor
   * two of the range of the averages of the cell and its face neighbours
   * (needed by the Mach-10 double Mach reflection of Sec. 4.5).  Otherwise
   * the cell takes its constant average for the step. */
  int32_t admissibility;
  /* 2D curvilinear grid (the extension that the remark closing Sec. 3.3
   * points to; the polar cavity of Sec. 4.8), or NULL for the uniform grid
   * of [x0, x1] x [y0, y1].  Host memory, read during gks_init /
   * gks_init_device only: vertex coordinates [ny+1][nx+1][2] (x, y), cell
   * (i, j) being the straight-edged quadrilateral with corners (i, j),
   * (i+1, j), (i+1, j+1), (i, j+1) in counter-clockwise order (positive
   * area).  The scheme then runs in the grid's logical coordinates: the
   * compact reconstruction of Sec. 3.2 with unit spacing and I(U1) = C |K|
   * (|K| the cell's area); each interface is evaluated in the frame of its
   * edge (unit normal from the lower to the higher logical index, unit
   * tangent along the edge towards the higher index, its length as the
   * interface extent), the logical derivatives turned into frame derivatives
   * by the metric at the interface centre (the vector between the two cell
   * centres, the mean of each cell's corners, and the edge); the update
   * divides by the cell areas; the CFL condition takes the widths |K| / (mean
   * length of the two opposite edges) and the speed.  Allowed with: dim 2,
   * conservative variables (recon_vars 0), no solid step, boundaries
   * periodic (the opposite edges one translation apart), outflow, no-slip
   * (with wall_omega) or inflow.  x0..y1 are not used.  The "x" ("y")
   * interfaces and the point value layouts refer to the logical directions
   * i (j); momentum components and point values stay in (x, y). */
  const double* mesh;
} gks_problem;

typedef struct gks_handle gks_handle; /* opaque, owned by the library */

/* Create a handle for n_problems (1..65535) independent grids (more than one:
 * a batch, advanced together by gks_step) and upload their initial state.
 *   cell[p]   : host, [nvar][ny][nx] cell averages, nvar = dim + 2
 *   face_x[p] : host, [ng][nvar][ny][nx+1] point values on the x interfaces,
 *               ng = 2 (2D: Gauss points y_j -/+ sqrt(3)/6 dy, in that order) or 1 (1D)
 *   face_y[p] : host, [2][nvar][ny+1][nx] point values on the y interfaces
 *               (Gauss points x_i -/+ sqrt(3)/6 dx); NULL when dim == 1
 *   stream    : a hipStream_t the library launches on (borrowed; it must
 *               outlive the handle), or NULL for a stream of the library's own.
 * On a periodic axis the last interface is the first one: its point values
 * are taken from the first interface (face_x[..][0], face_y[..][0][..]) and it
 * is computed once per step.
 * Host arrays are read during the call only.  Returns GKS_EINVAL for an
 * inconsistent problem (sizes, gamma, unknown boundary kind, nonphysical
 * initial state), GKS_ENOMEM / GKS_EDEVICE on device failures. */
int gks_init(gks_handle** out, int32_t n_problems, const gks_problem* probs,
             const double* const* cell, const double* const* face_x,
             const double* const* face_y, void* stream);

/* Device-borrow form of gks_init, for callers that keep the state in device
 * memory of their own (e.g. PyTorch tensors): the library steps these buffers
 * in place and allocates only its scratch arrays (reconstruction coefficients,
 * fluxes, the interface frame record, scalars).  The scheme's state, as in
 * gks_init, is the cell averages plus the interface point values (Sec. 3.2:
 * the point values at t^{n+1} come from the interface distribution and feed
 * the next reconstruction).  The layouts carry the library's ghost regions;
 * x runs fastest:
 *   d_cell[p]   : double, 2D [4][ny+4][nx+4], cell (i, j) at [v][j+2][i+2];
 *                 1D [3][nx+4], cell i at [v][i+2]
 *   d_face_x[p] : TS, 2D [2][4][ny+2][nx+3], interface i-1/2 (i = 0..nx) of
 *                 row j at [g][v][j+1][i+1]; 1D [3][nx+3], interface i at [v][i+1]
 *   d_face_y[p] : TS, 2D [2][4][ny+3][nx+2], interface j-1/2 (j = 0..ny) of
 *                 column i at [g][v][j+1][i+1]; NULL when dim == 1
 * TS = double for GKS_FP64, float for GKS_FP32_MIXED; g and v as in gks_init.
 * Ghost entries are ignored on entry and overwritten by every step; on a
 * periodic axis the seam interface is overwritten with the first interface's
 * values, as in gks_init.  The buffers must hold the initial state when the
 * call is made (work that wrote them on another stream must be complete),
 * must not overlap, must be aligned to their element size and must outlive
 * the handle; the caller owns them.  Between gks_step and a read of them by
 * the caller, synchronise `stream`, or call gks_fetch (which waits for the
 * library's stream; all its arrays may be NULL).  With stream == NULL the
 * library launches on a non-blocking stream of its own, which the legacy
 * default stream does not wait for.  Errors as gks_init;
 * a nonphysical initial cell is found on the device and reported as
 * GKS_EINVAL. */
int gks_init_device(gks_handle** out, int32_t n_problems, const gks_problem* probs,
                    void* const* d_cell, void* const* d_face_x, void* const* d_face_y,
                    void* stream);

/* Allocation-free stepping, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): nsteps steps of one problem on caller-owned device buffers in
 * the layouts of gks_init_device (d_cell, d_face_x, d_face_y: stepped in
 * place; periodic seams overwritten as there), without a handle and without
 * any allocation.  Every internal buffer lives in one static device array of
 * 128 MiB per GPU (held by each GPU the library runs on until the process
 * ends); a problem that needs more is refused with GKS_EINVAL before any
 * device work (about 230 B per cell in GKS_FP64 and 150 B in
 * GKS_FP32_MIXED: 768^2 and 960^2 cells fit).  All calls on one GPU share
 * that array, which keeps the last call's contents (each call initialises
 * what it reads): calls that overlap on one GPU (other host threads, other
 * streams) race and must not be made.  The work is enqueued on `stream`
 * (a borrowed hipStream_t; NULL: the null stream) and the call returns
 * without waiting, so it may be captured into a graph.  prob->t0 is the
 * initial time; dt_fixed > 0 fixes the step (0: the CFL condition on the
 * device every step); t_end > 0 shortens the last step to end there (0:
 * none).  d_status (device memory, may be NULL) receives after the last step
 * the time, the step count, the error word (0, or nonzero once a step made a
 * nonphysical state, or when the initial state is nonphysical; later steps
 * then leave the problem unchanged) and the fallback count (see
 * gks_fallbacks).  The same kernels as gks_step give the same results as a
 * handle made by gks_init_device from the same buffers and stepped with the
 * same arguments.  Returns GKS_EINVAL (gks_last_error(NULL) says why) or
 * GKS_EDEVICE. */
typedef struct {
  double t;
  int64_t steps;
  uint64_t error;
  int64_t fallbacks;
} gks_noalloc_status;
int gks_step_noalloc(const gks_problem* prob, void* d_cell, void* d_face_x, void* d_face_y, int32_t nsteps,
                     double dt_fixed, double t_end, gks_noalloc_status* d_status, void* stream);

/* Element counts of the three device buffers of gks_init_device for one
 * problem, and the size in bytes of a face element (8 or 4).  Host-only: no
 * device call.  Any output pointer may be NULL.  GKS_EINVAL for an
 * inconsistent problem (gks_last_error(NULL) says why). */
int gks_state_extent(const gks_problem* prob, int64_t* cell_elems, int64_t* face_x_elems,
                     int64_t* face_y_elems, int32_t* face_elem_bytes);

/* Enqueue nsteps time steps of every problem (asynchronous; returns after the
 * launches: nsteps replays of the step graph, captured at the first call).  dt_fixed: NULL to take each step from the CFL condition on the
 * device, else dt_fixed[p] for every step of problem p.  t_end: NULL for no
 * limit, else the last step of problem p is shortened to end at t_end[p] and
 * later steps leave it unchanged.  Once a step has produced a nonphysical
 * state in problem p (see gks_fetch), later steps leave p unchanged too, so
 * that gks_fetch returns the state of the failing step.  Arguments are
 * validated before anything is enqueued (GKS_EINVAL). */
int gks_step(gks_handle* h, int32_t nsteps, const double* dt_fixed, const double* t_end);

/* Wait for the enqueued work and copy the state of one problem to host
 * arrays with the layouts of gks_init (any pointer may be NULL to skip it),
 * plus its time and number of steps taken.  Returns the first sticky error:
 * GKS_ENONPHYS if some step produced rho <= 0, p <= 0 or a non-finite value
 * (gks_last_error names the problem and cell), after which the handle only
 * accepts gks_fetch, gks_last_error and gks_destroy (GKS_ESTATE). */
int gks_fetch(gks_handle* h, int32_t problem, double* cell, double* face_x, double* face_y,
              double* t, int64_t* steps);

/* Release all device memory, streams and events of the handle. */
int gks_destroy(gks_handle* h);

/* Human-readable description of the last error on this handle (static
 * storage owned by the handle, valid until the next call on it).  With
 * h == NULL: the reason of the last gks_init that failed on this thread. */
const char* gks_last_error(const gks_handle* h);

/* Kernel timing.  gks_profile(h, 1) makes every following gks_step record
 * HIP events on the library's stream around each kernel launch; the
 * accumulated time (ms) and launch count of kernel k (GKS_K_*) since the last
 * reset are returned by gks_kernel_time (which synchronises the stream).
 * gks_profile(h, 0) stops recording; gks_profile(h, 2) resets the sums. */
enum { GKS_K_GHOST = 0,  /* boundary images, with the time step */
       GKS_K_DT = 1,     /* (kept for the ABI: the step is taken in the boundary kernel; no launches) */
       GKS_K_RECON = 2, GKS_K_INTERFACE = 3, GKS_K_UPDATE = 4, GKS_K_COUNT = 5 };
int gks_profile(gks_handle* h, int32_t mode);
int gks_kernel_time(gks_handle* h, int32_t kernel, double* ms, int64_t* launches);

/* Number of (interior cell, step) pairs of problem `problem` whose
 * reconstruction fell back to the constant average (see admissibility),
 * summed over the steps since gks_init.  Waits for the enqueued work.
 * GKS_EINVAL for a bad index or a NULL pointer. */
int gks_fallbacks(gks_handle* h, int32_t problem, int64_t* cells);

/* Autotuner of the launch shapes (not part of the method): every kernel class
 * of the handle's launch sequence is timed with 64, 128 and 256 threads per
 * block over `steps` steps (1..1000) of the handle's own problems, with HIP
 * events as above, and the fastest size is kept per class.  The averages,
 * point values, times and step counts are restored afterwards, so the call
 * does not advance any problem; results of later steps are bitwise those of
 * any block size (each thread's arithmetic does not depend on it).  Returns
 * GKS_EINVAL, GKS_ESTATE, GKS_ENOMEM or GKS_EDEVICE (the latter two leave the
 * handle in its error state).
 * gks_block_size reports the present block size of kernel class `kernel`
 * (GKS_K_*; GKS_K_DT, which has no launches of its own, reports 64). */
int gks_tune(gks_handle* h, int32_t steps);
int gks_block_size(gks_handle* h, int32_t kernel, int32_t* threads);

/* Launch shape of kernel class `kernel` (GKS_K_GHOST, GKS_K_RECON,
 * GKS_K_INTERFACE or GKS_K_UPDATE; not part of the method): `threads` per
 * block (64, 128 or 256) and `grid`: for the 2D interface kernel, the
 * persistent form, `grid` blocks (a multiple of 8 in [8, 65536]; the eight
 * XCDs get equal shares) that take the interface tiles in turn, each block
 * staying on its XCD's range of tiles (0: one block per tile); for the 2D
 * reconstruction, the rows of its LDS tiles (1, 2 or 4: a block takes
 * threads / rows x rows cells and stages their averages and the one-cell
 * ring around them in LDS first; 0: one thread per cell in row order
 * reading the averages directly); 0 for the other classes.  gks_tune
 * chooses the block sizes as above, then keeps the persistent interface form,
 * with as many blocks as fit on the device at once, and the reconstruction
 * tile rows where they time faster.  Every shape gives bitwise the same
 * results.  gks_set_launch waits for the enqueued work and applies to
 * every problem of the handle; GKS_EINVAL for a bad value, GKS_ESTATE on a
 * handle in its error state.  gks_launch_shape reports the present shape of
 * a class (grid 0 where it is not persistent). */
int gks_set_launch(gks_handle* h, int32_t kernel, int32_t threads, int32_t grid);
int gks_launch_shape(gks_handle* h, int32_t kernel, int32_t* threads, int32_t* grid);

#ifdef __cplusplus
}
#endif
#endif /* GKS_H */
