/*
 * fargo.h - C ABI of libfargo, an MI355X (gfx950) implementation of the
 * hydrodynamics step of the FARGO3D method (Benitez-Llambay & Masset 2016,
 * ApJS 223, 11; arXiv:1602.02359).
 *
 * One call of fargo_step performs one full update of the paper's flow chart
 * (Sect. 3, Fig. "flowchart") restricted to hydrodynamics with a static
 * potential: boundary fill (box 2), bulk azimuthal velocity (box 3), pressure
 * (box 4), time step (box 6, Eq. cfl2 and Eq. 38), source step (boxes 7a-7c,
 * Sect. 3.3), boundary fill (box 9) and transport (box 12, Sect. 3.4-3.5:
 * left/right momenta, van Leer upwind sweeps in Y, Z and X, orbital advection
 * by integer circular shift and PPA fractional residual, velocities from
 * momenta).
 *
 * Mesh and storage (Sect. 2.2-2.3, Tab. "corresp", Sect. 4.1):
 *   X = azimuth (periodic, uniform, no ghosts), Y = radius, Z = z or colatitude.
 *   Every field is a device array [nz_g][ny_g][pitch] of the state element
 *   type (double, or float with FARGO_FP32_BULK; see `precision`; pot is
 *   double in both), X fastest,
 *   with ny_g = ny + 6, nz_g = nz + 6 (3D) or 1 (2D, nz == 1) and pitch from
 *   fargo_layout (a multiple of 64 elements, >= nx; columns nx..pitch-1 are
 *   padding, never read or written).  Three ghost layers in Y and Z.
 *   vx[k][j][i] sits on the lower X face of zone i, vy[k][j][i] on the face at
 *   ymin[j], vz[k][j][i] on the face at zmin[k]; rho, e, cs and pot are zone
 *   centred.
 *
 * Conventions.
 *   - Every call returns an int status (FARGO_OK = 0, negative on error); no
 *     exception crosses the ABI and nothing aborts.
 *   - All device work is enqueued on the caller's HIP stream (`stream`, a
 *     hipStream_t passed as void*; NULL means the default stream) and is
 *     stream-ordered.  fargo_step never synchronises the host.
 *   - Ownership: the caller owns the state arrays, the optional workspace and
 *     the stream; the library never frees caller memory.  The library owns the
 *     context and, when no workspace is given, one device allocation made in
 *     fargo_init and released in fargo_destroy.
 *   - A context is not thread safe and its calls must not overlap in time on
 *     different streams; separate contexts are independent.
 *   - Asynchronous problems found on the device (non-finite or non-positive
 *     density, bad time step) set an error word in the context; it is reported
 *     by the next fargo_check, and by fargo_cfl_dt when it reads dt back.
 */
#ifndef FARGO_H
#define FARGO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FARGO_ABI_VERSION 1
#define FARGO_NGH 3

/* status codes */
#define FARGO_OK 0
#define FARGO_EINVAL (-1)      /* invalid argument or parameter */
#define FARGO_ENOMEM (-2)      /* device or host allocation failed, or workspace too small */
#define FARGO_EHIP (-3)        /* a HIP runtime call failed */
#define FARGO_ENONFINITE (-4)  /* non-finite or non-positive state seen on the device */
#define FARGO_ECFL (-5)        /* the time step came out non-positive or non-finite */
#define FARGO_EUNSUPPORTED (-6)

/* geometry (Tab. "corresp") */
#define FARGO_CARTESIAN 0
#define FARGO_CYLINDRICAL 1
#define FARGO_SPHERICAL 2
/* equation of state: Eq. eos1 (static c_s field) or Eq. eos2 */
#define FARGO_ISOTHERMAL 0
#define FARGO_ADIABATIC 1
/* boundary kinds, per side (ymin, ymax, zmin, zmax).  PERIODIC must be set on
   both sides of a direction (Cartesian Y, Cartesian or cylindrical Z);
   REFLECT mirrors scalars and tangential velocities and makes the normal
   velocity antisymmetric with a zero boundary face; OUTFLOW copies the edge
   zone and the first interior face; FIXED leaves the caller's ghost values
   (and the boundary face) untouched. */
#define FARGO_BC_PERIODIC 0
#define FARGO_BC_REFLECT 1
#define FARGO_BC_OUTFLOW 2
#define FARGO_BC_FIXED 3
/* bulk azimuthal velocity of each ring (box 3): Eq. 37 or the azimuthal mean */
#define FARGO_V0_MINMAX 0
#define FARGO_V0_MEAN 1
/* precision of the evolved state (Sect. 6 discusses single vs double):
   FARGO_FP64: every field is double and all arithmetic is FP64.
   FARGO_FP32_BULK: the evolved fields (rho, v, e) and cs and nu are float
   and the bulk arithmetic of boxes 2, 7, 9 and 12 is FP32; the steps whose
   accuracy needs it stay FP64: the time step (box 6, from the stored
   values), each ring's bulk velocity v0 and the split of Eq. 29 into N and
   xi, the conserved sums, and the potential, which stays a double array
   with its gradient formed in FP64 (a difference of nearly equal values:
   FP32 storage would make its relative error eps r/dr, the round-off the
   paper's Sect. 6 traces through derivatives).  The geometric coefficients
   are FP64 tables rounded to FP32 where they enter bulk arithmetic.
   In FP32_BULK the vx array holds v_x - vb[k][j], the deviation from a
   per-ring FP64 background vb set with fargo_set_vx_background (zero until
   set), and the X momenta are transported as the same deviations: FP32
   rounding is then relative to the deviation, not to the orbital speed,
   whose rounding (eps v_K per zone and step) would otherwise enter the
   divergence of the residual velocity at every step (Sect. 6, through
   derivatives).  Box 6, the split and the sums use vb + vx in FP64. */
#define FARGO_FP64 0
#define FARGO_FP32_BULK 1

typedef struct {
  int32_t abi_version;     /* FARGO_ABI_VERSION */
  int32_t geometry;        /* FARGO_CARTESIAN / _CYLINDRICAL / _SPHERICAL */
  int32_t nx, ny, nz;      /* active zones; 1 <= nx <= 2^22, ny >= 3, nz == 1 (2D) or >= 3;
                              spherical needs nz >= 3; every field below 2^31 elements */
  double xmin, xmax;       /* azimuthal (X) extent; dx = (xmax - xmin)/nx */
  const double *ymin;      /* host, ny + 7 increasing face coordinates (ghosts included);
                              copied at fargo_init */
  const double *zmin;      /* host, nz + 7 face coordinates (3D) or 2 (2D); copied */
  int32_t eos;             /* FARGO_ISOTHERMAL or FARGO_ADIABATIC */
  double gamma;            /* ratio of specific heats (adiabatic), > 1 */
  double omega;            /* constant rotation rate of the frame */
  double courant;          /* Courant number C of Eq. cfl2 (paper: 0.44) */
  double cvnr;             /* artificial-viscosity constant: q = cvnr^2 rho dv^2 for dv < 0 */
  double shear_c0;         /* C0 of Eq. 38; <= 0 switches the shear limit off */
  int32_t fargo;           /* 1: orbital advection (Sect. 3.5.1), 0: plain transport */
  int32_t v0_mode;         /* FARGO_V0_MINMAX or FARGO_V0_MEAN */
  int32_t bc[4];           /* boundary kind of the ymin, ymax, zmin, zmax sides */
  int32_t precision;       /* FARGO_FP64 or FARGO_FP32_BULK */
  int32_t visc;            /* 1: kinematic viscosity (box 7d, App. B) from the static field nu, with
                              item 4 of Eq. cfl2; cylindrical 2D isothermal meshes only
                              (FARGO_EUNSUPPORTED otherwise) */
} fargo_params;

/* Device pointers to the state, each laid out as described above, with
   elements of type double (FARGO_FP64) or float (FARGO_FP32_BULK), except
   pot, which is always double.  rho, vx,
   vy are always required; vz in 3D only (NULL in 2D); e (volumic internal
   energy) for FARGO_ADIABATIC, cs (isothermal sound speed, static) for
   FARGO_ISOTHERMAL; pot (static potential, ghosts included) always; nu
   (static kinematic viscosity, zone centred, ghosts included) when visc is
   set, else NULL.  Arrays must be aligned to their element size. */
typedef struct {
  void *rho, *vx, *vy, *vz, *e;
  const void *cs, *pot, *nu;
} fargo_state;

typedef struct fargo_ctx fargo_ctx;

/* Version of this ABI (FARGO_ABI_VERSION). */
int fargo_abi_version(void);

/* Static description of a status code; never NULL. */
const char *fargo_strerror(int status);

/* Array layout for the given parameters: pitch (elements per X row), ny_g,
   nz_g.  Any output may be NULL.  Validates the parameters (FARGO_EINVAL). */
int fargo_layout(const fargo_params *params, int32_t *pitch, int32_t *ny_g, int32_t *nz_g);

/* Bytes of device workspace fargo_init needs for these parameters. */
int fargo_workspace_bytes(const fargo_params *params, size_t *bytes);

/* Create a context on the current HIP device.  `workspace` is a device buffer
   of at least fargo_workspace_bytes bytes, owned by the caller and kept alive
   until fargo_destroy; NULL makes the library allocate it (hipMalloc).
   Computes the geometric coefficients of Appendix A (Tab. "geom", Eqs. 70-71)
   on the host in FP64 and uploads them (synchronously).  *out is set on
   success only. */
int fargo_init(const fargo_params *params, void *workspace, size_t ws_bytes, fargo_ctx **out);

/* FARGO_FP32_BULK contexts only (FARGO_EINVAL otherwise): set the FP64
   background vb of the azimuthal velocity, one value per ring of the whole
   mesh, ghosts included: `vb` is host memory of nz_g * ny_g doubles indexed
   [k][j] (finite; FARGO_EINVAL otherwise), copied synchronously.  From then
   on the context reads and writes the state's vx as v_x - vb (see
   FARGO_FP32_BULK); a caller that changes vb must rewrite vx to match.  A
   good background is the ring's mean azimuthal velocity (for a disk, its
   rotation curve in the frame); any choice gives the same step in exact
   arithmetic. */
int fargo_set_vx_background(fargo_ctx *ctx, const double *vb);

/* Release the context (synchronises the device first).  NULL is a no-op. */
void fargo_destroy(fargo_ctx *ctx);

/* Boxes 2, 3, 4 and 6: fill the state's ghost layers (box 2; only ghosts and
   boundary faces are written), compute each ring's bulk velocity and the time
   step of Eq. cfl2 (items 1-3, and 4 with viscosity; the residual velocity and the shear limit
   of Eq. 38 under orbital advection), minimised over active zones.  The step
   stays on the device for the next fargo_step(dt <= 0); if dt_host is not
   NULL the call waits for the stream and copies it back, returning
   FARGO_ENONFINITE / FARGO_ECFL if the device flagged a problem. */
int fargo_cfl_dt(fargo_ctx *ctx, fargo_state *state, double *dt_host, void *stream);

/* One full update of the state, in place.  dt > 0 imposes the time step; dt
   <= 0 computes it on the device (box 6) without any host synchronisation.
   The step defines the active zones and the owned faces (all X faces,
   interior Y/Z faces, and the lower Y/Z boundary face in a periodic
   direction).  Ghost zones and the other boundary faces of the state keep
   the box-2 fill of this call (box 9 acts on internal copies); the next call
   refills them, and FIXED sides are never written. */
int fargo_step(fargo_ctx *ctx, fargo_state *state, double dt, void *stream);

/* Eq. 32 on one field: every active ring (j, k) is circularly permuted in
   place, Q_i <- Q_{(i - N) mod nx}, with N = nshift[(k - k0)*ny + (j - j0)]
   read from a device array of ny*nz int32 (k0 = 3 in 3D, 0 in 2D).  The
   field has the state element type of the context.  Ghost rows are not
   touched.  Bit-exact (a pure permutation).  A ring of at most 64 KiB is
   staged in LDS; a longer one is shifted out of place through the context's
   workspace (so calls on one context must not overlap a step). */
int fargo_shift(fargo_ctx *ctx, void *field, const int32_t *nshift, void *stream);

/* Box 3 and the split of Eq. 29 for a given dt, on active rings: v0 (Eq. 37
   or mean), N = nearest integer to D = (v0 dt)/dX with ties away from zero,
   xi = D - N, all in FP64 (vx has the state element type and is read
   exactly).  Outputs are device arrays of ny*nz elements indexed as in
   fargo_shift.  dX is the azimuthal zone length at the v_phi face centre
   (dx, r dphi or r sin(theta) dphi). */
int fargo_ring_split(fargo_ctx *ctx, const void *vx, double dt, double *v0, int32_t *nshift, double *xi,
                     void *stream);

/* Conserved sums over active zones (waits for the stream): out[0] = mass
   sum(rho V); out[1..3] = X, Y, Z momenta sum(rho m(<v>) V) with <v> the mean
   of the two faces (Eq. 19) and m the factor of Tab. "momenta" (X: r(v + r
   Omega) or R(v + R Omega); Z: r v_theta in spherical geometry); out[4] =
   sum(e V) (0 if isothermal).  Double-double accumulation in a fixed order
   (deterministic).  Upper faces in periodic directions are read through the
   wrap.  `out` is host memory. */
int fargo_conserved_sums(fargo_ctx *ctx, const fargo_state *state, double out[5], void *stream);

/* fargo_conserved_sums for callers that cannot allocate device memory (code
   under stream or graph capture, tight serving loops, harnesses that forbid
   allocation): the same kernels and the same results, bit for bit, but the
   per-ring partial sums and the five results are staged in a static device
   array of the library (10.5 MB per device, for at most 131072 = 2^17 active
   rings, ny * nz) instead of the context's workspace.  Nothing is allocated:
   no hipMalloc, hipFree or allocating library call.  The array's device
   address is looked up once per device by fargo_init, with that device
   current; the array lives until the process ends.  Every call on one device
   shares that device's array and keeps the last call's contents, which the
   next call overwrites entirely (nothing needs to start at zero): calls that
   overlap in time on one device (different streams or threads) race, and
   must be serialised by the caller.  The current device must be the
   context's (FARGO_EINVAL otherwise); more than 2^17 active rings give
   FARGO_ENOMEM.  Waits for the stream; `out` is host memory. */
int fargo_conserved_sums_noalloc(fargo_ctx *ctx, const fargo_state *state, double out[5], void *stream);

/* Bandwidth probe (no part of the method): a plain streaming copy of `bytes`
   (a multiple of 16) from src to dst, device buffers aligned to 16 bytes
   that do not overlap, by `blocks` workgroups of 256 threads, each thread
   moving four 16-byte vectors per round, loads before stores; blocks = 0
   launches one thread per 16-byte vector instead.  It measures
   the HBM bandwidth a hand-written kernel reaches on this device, the
   practical ceiling the step's kernels are compared with besides the
   vendor peak.  Enqueued on `stream`; FARGO_EINVAL for a bad argument. */
int fargo_hbm_copy(const void *src, void *dst, size_t bytes, int blocks, void *stream);

/* Bandwidth probe of a column sweep's access pattern (no part of the
   method): nin FP64 fields in[0..nin-1] are read and the first nout written,
   out[q] = in[q] + in[nin - 1], each field nx * ny * nz doubles, x fastest
   (1 <= nout <= nin <= 9; device buffers aligned to 8 bytes; no output may
   overlap an input or another output).  march = 0: one element per thread;
   march = 1: one (x, y) column per thread, walking its nz planes with the
   loads of plane k + 1 issued before the stores of plane k, as the Y and Z
   sweeps (Sect. 3.4) walk theirs.  The rate it reaches with the field counts
   of a sweep is the ceiling of that sweep's memory access pattern, with
   none of its arithmetic.  Enqueued on `stream`; FARGO_EINVAL for a bad
   argument (the arrays `in` and `out` are host memory, read before return). */
int fargo_hbm_streams(const double *const *in, int nin, double *const *out, int nout, int nx, int ny, int nz,
                      int march, void *stream);

/* Copy the time step last computed or imposed on the device into *dt_host
   (waits for the stream). */
int fargo_get_dt(fargo_ctx *ctx, double *dt_host, void *stream);

/* Wait for the device and report (then clear) the asynchronous error word. */
int fargo_check(fargo_ctx *ctx);

/* Per-kernel timing with HIP events on the caller's stream.  While enabled,
   every kernel launch of the library is bracketed by events.
   fargo_profile_enable waits for the device and resets the accumulators;
   fargo_timings (which waits for the stream) returns, for up to `cap` kernel
   kinds, their names (static strings), launch counts and total milliseconds
   since the last fargo_profile_enable, and the number of kinds returned. */
int fargo_profile_enable(fargo_ctx *ctx, int on);
int fargo_timings(fargo_ctx *ctx, const char **names, int64_t *counts, double *total_ms, int cap, int *n_out,
                  void *stream);

/* ---- Batches of independent contexts (parameter sweeps over many disks) ----
   A batch advances `count` contexts (any sizes and parameters, one device)
   together.  fargo_batch_create captures one fargo_step(dt <= 0) of every
   context into a hipGraph: the contexts are spread round-robin over `lanes`
   streams that fork from and join into an origin stream, so that independent
   disks run concurrently; each keeps its own device time step (box 6).  The
   contexts, states and workspaces must outlive the batch and must not be
   used by other calls while a batch step runs.  `states` is an array of
   `count` states (copied).  Profiling events are not recorded inside the
   graph.
   lanes == 0 selects the fused form: each kernel of the step is launched once
   for all contexts, its workgroups mapped to (context, workgroup) through a
   device table, so a step is seven or eight launches (captured into one
   graph) whatever the number of disks; the results are those of fargo_step
   context by context, bit for bit.  It requires 2D meshes (nz == 1) of one
   configuration (precision, geometry, equation of state, viscosity, orbital
   advection, v0 mode, boundary kinds), FIXED radial sides, and nx at most
   1792 (FARGO_EUNSUPPORTED otherwise; lanes 1..64 take any contexts). */
typedef struct fargo_batch fargo_batch;
int fargo_batch_create(fargo_ctx *const *ctxs, const fargo_state *states, int count, int lanes,
                       fargo_batch **out);
/* One step of every context: a single graph launch on `stream`. */
int fargo_batch_step(fargo_batch *batch, void *stream);
/* The column sweeps' zones per thread each context uses in the batch (n ==
   count entries). */
int fargo_batch_chunks(const fargo_batch *batch, int32_t *chunk, int n);
/* Autotuner (the block-size tuning of Sect. 4.2, for batches).  Fused form:
   the zones per thread of the column sweep are chosen per size class of
   contexts (floor(log2 ny)), class after class, from chunks[], each
   candidate timed over `steps` graph launches (lanes is ignored; best[0] =
   0, best[1] = the last context's choice; fargo_batch_chunks gives all).
   Other forms: for every pair (lanes[a], chunks[c]) - the graph's stream count
   and the zones per thread of the Y/Z column sweeps - re-capture the batch,
   time `steps` graph launches with HIP events on `stream`, and keep the
   fastest pair (written to best[0], best[1]) with the graph captured and
   timed for it (a new capture of the same pair can run at another speed,
   since its streams differ).  The evolving fields of every
   state are saved first and restored after each candidate (one temporary
   device allocation), so the call leaves the states as it found them.
   Waits for the stream. */
int fargo_batch_tune(fargo_batch *batch, const int32_t *lanes, int nlanes, const int32_t *chunks, int nchunks,
                     int steps, void *stream, int32_t best[2]);
/* Release the graph and streams (waits for the device).  NULL is a no-op. */
void fargo_batch_destroy(fargo_batch *batch);

/* ------------------------------------------------------------------------ */
/* Learned flux correction (an extension; the paper has no learned part)    */
/* ------------------------------------------------------------------------ */
/* A three-layer 3 x 3 convolutional net (4 -> 32 -> 32 -> 2 channels, ReLU
   after the first two layers) on the active zones of a 2D cylindrical FP64
   context predicts corrections to the mass fluxes through each zone's lower
   X (azimuthal) and lower Y (radial) face.  They are applied as a
   conservative flux-divergence update of the density,
     drho_ij = -(1/V_j) [dFx_{i+1,j} - dFx_ij + dFy_{i,j+1} - dFy_ij],
   with no correction through the two radial boundary faces, so the total mass
   is unchanged (the telescoping argument of Sect. 3.4).  Features of a zone:
   rho/rho_s - 1, v_y/u_s, v_x/u_s (the face velocities stored with the
   zone) and (r - r_mid)/r_span; convolutions are periodic in X and zero
   beyond the active radial rows.  Products run on the bfloat16 matrix cores
   (operands rounded to nearest even, FP32 accumulation); the FP32 master
   parameters are trained on the device with Adam (beta1 0.9, beta2 0.999,
   eps 1e-8) on the loss mean(((drho - target)/sigma)^2), the mean taken over
   every zone of every sample of a training batch (1 to max_batch states of
   the context's mesh per Adam step).
   Requirements: cylindrical, nz == 1, FARGO_FP64, nx a multiple of 64
   (FARGO_EUNSUPPORTED otherwise). */
typedef struct fargo_lfc fargo_lfc;
typedef struct {
  double rho_s, u_s, r_mid, r_span; /* feature scales */
  double flux_scale;                /* dF = flux_scale x net output */
  double sigma;                     /* loss scale (> 0) */
  double guard;                     /* apply only if rho + drho > 0 and |drho| <= guard rho in every zone */
  int32_t max_batch;                /* samples per batch the buffers hold, 1..32 (0 means 1) */
} fargo_lfc_params;
/* Parameter vector (FP32): W1 [32][3][3][4], b1 [32], W2 [32][3][3][32],
   b2 [32], W3 [2][3][3][32], b3 [2]; weights [out][ty][tx][in]. */
#define FARGO_LFC_NPARAM 11010
/* Device buffers of the last forward / training batch, for inspection:
   f [sample][pixel][4], h1, h2 [sample][pixel][32] (bfloat16 bits as
   uint16), o [sample][pixel][2] (float), drho [sample][pixel] (double), g3
   [sample][pixel][4], g2, g1 [sample][pixel][32] (bfloat16 layer
   gradients); pixel = j nx + i over the active zones, samples in the order
   they were passed. */
typedef struct {
  const void *f, *h1, *h2, *o, *drho, *g3, *g2, *g1;
} fargo_lfc_views;
/* Bind a net to `ctx` (which must outlive it); allocates its device
   buffers, for p->max_batch samples.  Parameters start at zero: set them
   with fargo_lfc_set_params.  FARGO_EINVAL for max_batch outside 0..32. */
int fargo_lfc_create(fargo_ctx *ctx, const fargo_lfc_params *p, fargo_lfc **out);
/* Free the buffers (waits for the device).  NULL is a no-op. */
void fargo_lfc_destroy(fargo_lfc *l);
/* Copy n == FARGO_LFC_NPARAM host floats in (resets Adam's moments and step
   count) or out; fargo_lfc_get_grad copies the last gradient out.  These
   synchronize the device. */
int fargo_lfc_set_params(fargo_lfc *l, const float *host, int32_t n);
int fargo_lfc_get_params(fargo_lfc *l, float *host, int32_t n);
int fargo_lfc_get_grad(fargo_lfc *l, float *host, int32_t n);
/* The net on `state` and the density change it implies (views.drho). */
int fargo_lfc_forward(fargo_lfc *l, const fargo_state *state, void *stream);
/* The same on n states (an array, 1 <= n <= max_batch, each of the context's
   mesh; FARGO_EINVAL otherwise), sample s in slot s of every view. */
int fargo_lfc_forward_batch(fargo_lfc *l, const fargo_state *states, int32_t n, void *stream);
/* One Adam step with learning rate lr on the loss against `target` (device,
   double [ny][nx] over the active zones, the wanted density change). */
int fargo_lfc_train_step(fargo_lfc *l, const fargo_state *state, const double *target, double lr,
                         void *stream);
/* One Adam step on a batch: n states and n targets (host array of device
   pointers, as for train_step), the loss the mean over all n samples.  Every
   convolution of the forward and backward pass runs once over the whole
   batch. */
int fargo_lfc_train_batch(fargo_lfc *l, const fargo_state *states, const double *const *targets, int32_t n,
                          double lr, void *stream);
/* Forward, then the guarded update of state->rho: if the guard rejects the
   correction anywhere, the density is left as it is and the skip flag is
   set (read with fargo_lfc_result). */
int fargo_lfc_apply(fargo_lfc *l, fargo_state *state, void *stream);
/* Loss of the last training step and skip flag of the last apply (waits for
   `stream`); either pointer may be NULL. */
int fargo_lfc_result(fargo_lfc *l, double *loss, int32_t *skipped, void *stream);
int fargo_lfc_get_views(fargo_lfc *l, fargo_lfc_views *v);
/* R x R conservative restriction (R = 4, or 2) of the active zones of a fine
   2D cylindrical FP64 state onto a coarse one (fine nx, ny = R coarse nx, ny;
   every coarse face a fine face): density = mass / volume of the coarse
   zone; v_x on a coarse X face = the radial-width-weighted mean of the R fine
   X faces on it; v_y on a coarse Y face = the mean of the R fine Y faces on
   it.  Ghost zones of the coarse state are not written. */
int fargo_lfc_restrict(const fargo_ctx *fine, const fargo_state *fs, const fargo_ctx *coarse, fargo_state *cs,
                       void *stream);
/* Training target over the active zones of a 2D cylindrical FP64 context:
   target[j nx + i] = ref.rho - plain.rho (device, double [ny][nx]), the
   density change that takes the plain coarse step to the restricted fine
   solution. */
int fargo_lfc_target(const fargo_ctx *ctx, const fargo_state *ref, const fargo_state *plain, double *target,
                     void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FARGO_H */
