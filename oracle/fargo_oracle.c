/*
 * FP64 CPU oracle of one hydrodynamics step of the FARGO3D method
 * (Benitez-Llambay & Masset 2016, ApJS 223, 11; arXiv:1602.02359).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares no code, header,
 * table or helper with the GPU library; it is written directly from the paper,
 * in the paper's order and notation, as plain loops over the mesh ("mesh
 * functions", Sect. 4.2).  Build: gcc -O3 -ffp-contract=off -fopenmp (no
 * fast-math; -march=native for the timed CPU baseline); OpenMP only splits
 * independent cells between threads.
 *
 * One full update (Sect. 3, Fig. "flowchart"):
 *   box 2   boundary fill (ghost layers)
 *   box 3   per-ring bulk azimuthal velocity v0 (Eq. 37)
 *   box 4   pressure from the equation of state (Eqs. eos1, eos2)
 *   box 6   time step (Eq. cfl2, items 1-4; Eq. 38 with orbital advection)
 *   box 7a  pressure and potential gradients, centrifugal terms (Sect. 3.3, Eq. 12)
 *   box 7b  von Neumann-Richtmyer artificial viscosity and its heating
 *   box 7d  kinematic viscosity (App. B, Eqs. 73 and 76; cylindrical 2D),
 *           applied after 7b and before 7c
 *   box 7c  compressional heating (time-centred, gamma-law gas)
 *   box 9   boundary fill
 *   box 12a left/right momenta (Eqs. 16-17, Tab. "momenta")
 *   box 12b/c directional upwind transport with van Leer slopes and
 *           consistent transport (Eqs. flux, 14, 15); in X with orbital
 *           advection: residual sweep (Eq. fargo1), integer circular shift
 *           (Eq. 32) and PPA fractional residual (Eqs. 34-36)
 *   box 12d velocities from momenta (Eq. 18)
 *
 * Readings where the paper is silent or garbled (each listed in the design
 * notes of the repository): sweep order Y, Z, X; nearest integer with ties
 * away from zero; |xi| in both PPA branches; slope ratio "<= 0 -> 0"; van
 * Leer v<0 branch with the downstream cell width; artificial viscosity
 * q = C^2 rho dv^2 (dv < 0) with time-step term L/(4 C^2 |dv|); heating
 * e(1 - a)/(1 + a), a = dt(gamma-1)div(v)/2; Jacobi source updates; cell
 * centres at arithmetic midpoints; azimuthal length X = r sin(theta) dphi.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NGH 3

enum { GEO_CART = 0, GEO_CYL = 1, GEO_SPH = 2 };
enum { EOS_ISO = 0, EOS_ADI = 1 };
enum { BC_PERIODIC = 0, BC_REFLECT = 1, BC_OUTFLOW = 2, BC_FIXED = 3 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENONFINITE = -4, ORC_ECFL = -5 };

/* Run parameters, filled by the Python side of the test harness. */
typedef struct {
  int32_t geometry, nx, ny, nz;
  double xmin, xmax;
  const double *ymin; /* ny + 2*NGH + 1 face coordinates */
  const double *zmin; /* nz + 2*NGH + 1 face coordinates (3D), 2 (2D) */
  int32_t eos;
  double gamma;
  double omega;    /* frame rotation rate (constant) */
  double courant;  /* C of Eq. cfl2 */
  double cvnr;     /* artificial-viscosity constant */
  double shear_c0; /* C0 of Eq. 38; <= 0 switches the shear limit off */
  int32_t fargo, v0_mean;
  int32_t bc[4];   /* ymin, ymax, zmin, zmax sides */
  int32_t visc;    /* 1: viscous stress (box 7d) with the static field nu */
} orc_params;

/* Arrays (nz_g, ny_g, nx), X fastest, ghosts included. */
typedef struct {
  double *rho, *vx, *vy, *vz, *e; /* vz NULL in 2D; e NULL if isothermal */
  const double *cs, *pot;         /* static fields; cs NULL if adiabatic */
  const double *nu;               /* static kinematic viscosity (zone centred); NULL without viscosity */
} orc_state;

/* ------------------------------------------------------------------------ */
/* Mesh and the geometric coefficients of Appendix A (Tab. "geom", Eqs. 70-71) */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_params *p;
  int geo, nx, ny, nz, nyg, nzg, j0, jn, k0, kn, d3;
  size_t nc;
  double dx;
  double *ymin, *ymed, *zmin, *zmed;
  /* one-dimensional factors: S_x = sxj*sxk, S_y = syj*syk, S_z = szj*szk,
     1/V = invVj/syk.  syj is given per Y face (nyg+1), szk per Z face (nzg+1). */
  double *sxj, *sxk, *syj, *syk, *szj, *szk, *invVj;
  double *sinzmed; /* sin of the colatitude at cell centres (spherical) */
} mesh_t;

#define IX(i, j, k) ((((size_t)(k)) * (size_t)m->nyg + (size_t)(j)) * (size_t)m->nx + (size_t)(i))

static void mesh_free(mesh_t *m) {
  free(m->ymin); free(m->ymed); free(m->zmin); free(m->zmed);
  free(m->sxj); free(m->sxk); free(m->syj); free(m->syk); free(m->szj); free(m->szk);
  free(m->invVj); free(m->sinzmed);
  memset(m, 0, sizeof(*m));
}

static int check_params(const orc_params *p) {
  if (!p || p->nx < 1 || p->ny < 3) return ORC_EINVAL;
  if (p->nz != 1 && p->nz < 3) return ORC_EINVAL;
  if (p->geometry < 0 || p->geometry > 2) return ORC_EINVAL;
  if (p->geometry == GEO_SPH && p->nz < 3) return ORC_EINVAL;
  if (!p->ymin || !p->zmin || !(p->xmax > p->xmin)) return ORC_EINVAL;
  if (p->eos != EOS_ISO && p->eos != EOS_ADI) return ORC_EINVAL;
  if (p->eos == EOS_ADI && !(p->gamma > 1.0)) return ORC_EINVAL;
  for (int s = 0; s < 4; s++)
    if (p->bc[s] < 0 || p->bc[s] > 3) return ORC_EINVAL;
  /* periodicity must hold on both sides of a direction */
  if ((p->bc[0] == BC_PERIODIC) != (p->bc[1] == BC_PERIODIC)) return ORC_EINVAL;
  if (p->nz > 1 && (p->bc[2] == BC_PERIODIC) != (p->bc[3] == BC_PERIODIC)) return ORC_EINVAL;
  if (p->geometry != GEO_CART && p->bc[0] == BC_PERIODIC) return ORC_EINVAL;
  if (p->geometry == GEO_SPH && p->bc[2] == BC_PERIODIC) return ORC_EINVAL;
  if (p->visc && (p->geometry != GEO_CYL || p->nz != 1)) return ORC_EINVAL; /* 7d: cylindrical 2D only */
  return ORC_OK;
}

static int mesh_init(mesh_t *m, const orc_params *p) {
  memset(m, 0, sizeof(*m));
  int rc = check_params(p);
  if (rc) return rc;
  m->p = p;
  m->geo = p->geometry;
  m->nx = p->nx; m->ny = p->ny; m->nz = p->nz;
  m->d3 = p->nz > 1;
  m->nyg = p->ny + 2 * NGH;
  m->nzg = m->d3 ? p->nz + 2 * NGH : 1;
  m->j0 = NGH; m->jn = NGH + p->ny;
  m->k0 = m->d3 ? NGH : 0; m->kn = m->d3 ? NGH + p->nz : 1;
  m->nc = (size_t)m->nx * m->nyg * m->nzg;
  m->dx = (p->xmax - p->xmin) / p->nx;
  int nyg = m->nyg, nzg = m->nzg;
  m->ymin = malloc(sizeof(double) * (nyg + 1));
  m->ymed = malloc(sizeof(double) * nyg);
  m->zmin = malloc(sizeof(double) * (nzg + 1));
  m->zmed = malloc(sizeof(double) * nzg);
  m->sxj = malloc(sizeof(double) * nyg);
  m->syj = malloc(sizeof(double) * (nyg + 1));
  m->szj = malloc(sizeof(double) * nyg);
  m->invVj = malloc(sizeof(double) * nyg);
  m->sxk = malloc(sizeof(double) * nzg);
  m->syk = malloc(sizeof(double) * nzg);
  m->szk = malloc(sizeof(double) * (nzg + 1));
  m->sinzmed = malloc(sizeof(double) * nzg);
  if (!m->ymin || !m->ymed || !m->zmin || !m->zmed || !m->sxj || !m->syj || !m->szj ||
      !m->invVj || !m->sxk || !m->syk || !m->szk || !m->sinzmed) {
    mesh_free(m);
    return ORC_ENOMEM;
  }
  memcpy(m->ymin, p->ymin, sizeof(double) * (nyg + 1));
  memcpy(m->zmin, p->zmin, sizeof(double) * (nzg + 1));
  for (int j = 0; j < nyg; j++) {
    if (!(m->ymin[j + 1] > m->ymin[j])) { mesh_free(m); return ORC_EINVAL; }
    m->ymed[j] = 0.5 * (m->ymin[j] + m->ymin[j + 1]);
  }
  for (int k = 0; k < nzg; k++) {
    if (!(m->zmin[k + 1] > m->zmin[k])) { mesh_free(m); return ORC_EINVAL; }
    m->zmed[k] = 0.5 * (m->zmin[k] + m->zmin[k + 1]);
    m->sinzmed[k] = sin(m->zmed[k]);
  }
  if (m->geo != GEO_CART && !(m->ymin[0] > 0.0)) { mesh_free(m); return ORC_EINVAL; }
  if (m->geo == GEO_SPH && !(m->zmin[0] > 0.0 && m->zmin[nzg] < M_PI)) { mesh_free(m); return ORC_EINVAL; }
  double dx = m->dx;
  /* Tab. "geom": Y-dependent factors */
  for (int j = 0; j <= nyg; j++) {
    double Ymin = m->ymin[j];
    if (j < nyg) {
      double Ymax = m->ymin[j + 1];
      switch (m->geo) {
      case GEO_CART:
        m->sxj[j] = Ymax - Ymin;
        m->szj[j] = dx * (Ymax - Ymin);
        m->invVj[j] = 1.0 / (Ymax - Ymin);
        break;
      case GEO_CYL:
        m->sxj[j] = Ymax - Ymin;
        m->szj[j] = 0.5 * dx * (Ymax * Ymax - Ymin * Ymin);
        m->invVj[j] = 2.0 / ((Ymax * Ymax - Ymin * Ymin) * dx);
        break;
      default:
        m->sxj[j] = 0.5 * (Ymax * Ymax - Ymin * Ymin);
        m->szj[j] = 0.5 * dx * (Ymax * Ymax - Ymin * Ymin);
        m->invVj[j] = 3.0 / ((Ymax * Ymax * Ymax - Ymin * Ymin * Ymin) * dx);
        break;
      }
    }
    switch (m->geo) {
    case GEO_CART: m->syj[j] = 1.0; break;
    case GEO_CYL: m->syj[j] = Ymin * dx; break;
    default: m->syj[j] = Ymin * Ymin * dx; break;
    }
  }
  /* Tab. "geom": Z-dependent factors */
  for (int k = 0; k <= nzg; k++) {
    double Zmin = m->zmin[k];
    if (k < nzg) {
      double Zmax = m->zmin[k + 1];
      switch (m->geo) {
      case GEO_CART:
        m->sxk[k] = Zmax - Zmin;
        m->syk[k] = dx * (Zmax - Zmin);
        break;
      case GEO_CYL:
        m->sxk[k] = Zmax - Zmin;
        m->syk[k] = Zmax - Zmin;
        break;
      default:
        m->sxk[k] = Zmax - Zmin;
        m->syk[k] = cos(Zmin) - cos(Zmax);
        break;
      }
    }
    m->szk[k] = (m->geo == GEO_SPH) ? sin(Zmin) : 1.0;
  }
  return ORC_OK;
}

/* face areas (lower face of cell j,k), inverse volume, volume (Eqs. 70, 71) */
static inline double Sx(const mesh_t *m, int j, int k) { return m->sxj[j] * m->sxk[k]; }
static inline double Sy(const mesh_t *m, int j, int k) { return m->syj[j] * m->syk[k]; }
static inline double Sz(const mesh_t *m, int j, int k) { return m->szj[j] * m->szk[k]; }
static inline double Vinv(const mesh_t *m, int j, int k) { return m->invVj[j] / m->syk[k]; }
static inline double Vol(const mesh_t *m, int j, int k) { return m->syk[k] / m->invVj[j]; }

/* Lengths.  Azimuthal zone length at the v_phi face centre: dx, r dphi,
   r sin(theta) dphi (cartesian, cylindrical, spherical). */
static inline double DXlen(const mesh_t *m, int j, int k) {
  switch (m->geo) {
  case GEO_CART: return m->dx;
  case GEO_CYL: return m->ymed[j] * m->dx;
  default: return m->ymed[j] * m->sinzmed[k] * m->dx;
  }
}
/* radial zone width, and the distance between centres j-1 and j (at face j) */
static inline double Ly(const mesh_t *m, int j) { return m->ymin[j + 1] - m->ymin[j]; }
static inline double hy(const mesh_t *m, int j) { return m->ymed[j] - m->ymed[j - 1]; }
/* Z zone width and centre distance; in spherical geometry r dtheta */
static inline double Lz(const mesh_t *m, int j, int k) {
  double d = m->zmin[k + 1] - m->zmin[k];
  return (m->geo == GEO_SPH) ? d * m->ymed[j] : d;
}
static inline double hz(const mesh_t *m, int j, int k) {
  double d = m->zmed[k] - m->zmed[k - 1];
  return (m->geo == GEO_SPH) ? d * m->ymed[j] : d;
}
/* cylindrical radius of a v_phi face centre (distance to the rotation axis) */
static inline double Rcyl(const mesh_t *m, int j, int k) {
  return (m->geo == GEO_SPH) ? m->ymed[j] * m->sinzmed[k] : m->ymed[j];
}

static inline int wrap(int c, int lo, int n) { /* periodic index within [lo, lo+n) */
  int r = (c - lo) % n;
  if (r < 0) r += n;
  return lo + r;
}
static inline int imod(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

/* ------------------------------------------------------------------------ */
/* Boxes 2 and 9: boundary conditions in the three ghost layers (Sect. 4.1)  */
/* ------------------------------------------------------------------------ */
/* Scalars and velocities tangential to a side are mirrored (REFLECT), copied
   from the opposite edge (PERIODIC) or from the edge zone (OUTFLOW); the normal
   velocity is antisymmetric about the boundary face, which is set to zero
   (REFLECT), or copied from the first interior face (OUTFLOW).  FIXED sides are
   left as the caller wrote them.  The boundary faces are set first, so that
   the ghost faces mirror final values. */

/* generic side fill along a direction d in {Y, Z}: zone index a = j or k */
typedef struct {
  const mesh_t *m;
  int dir; /* 1 = Y, 2 = Z */
} side_t;

static inline size_t at(const side_t *sd, int i, int a, int b) {
  const mesh_t *m = sd->m;
  return sd->dir == 1 ? IX(i, a, b) : IX(i, b, a);
}

static void bc_faces(const side_t *sd, int side, int kind, double *vn) {
  const mesh_t *m = sd->m;
  int lo = sd->dir == 1 ? m->j0 : m->k0, hi = sd->dir == 1 ? m->jn : m->kn;
  int nb = sd->dir == 1 ? m->nzg : m->nyg; /* extent of the other mesh direction */
  int bf = side == 0 ? lo : hi;
  if (kind == BC_FIXED) return;
  for (int b = 0; b < nb; b++)
    for (int i = 0; i < m->nx; i++) {
      if (kind == BC_REFLECT) vn[at(sd, i, bf, b)] = 0.0;
      else if (kind == BC_OUTFLOW) vn[at(sd, i, bf, b)] = vn[at(sd, i, side == 0 ? lo + 1 : hi - 1, b)];
      else if (side == 1) vn[at(sd, i, bf, b)] = vn[at(sd, i, lo, b)]; /* periodic image */
    }
}

static void bc_ghosts(const side_t *sd, int side, int kind, double *const *cen, int ncen, double *vn) {
  const mesh_t *m = sd->m;
  int lo = sd->dir == 1 ? m->j0 : m->k0, hi = sd->dir == 1 ? m->jn : m->kn;
  int nb = sd->dir == 1 ? m->nzg : m->nyg;
  if (kind == BC_FIXED) return;
  for (int g = 0; g < NGH; g++) {
    int dst, src, fdst = -1, fsrc = -1;
    double fsign = 1.0;
    if (side == 0) {
      dst = lo - 1 - g;
      fdst = lo - 1 - g;
      if (kind == BC_PERIODIC) { src = hi - 1 - g; fsrc = hi - 1 - g; }
      else if (kind == BC_REFLECT) { src = lo + g; fsrc = lo + 1 + g; fsign = -1.0; }
      else { src = lo; fsrc = lo; }
    } else {
      dst = hi + g;
      if (g < NGH - 1) fdst = hi + 1 + g; /* the top face of the last ghost is not stored */
      if (kind == BC_PERIODIC) { src = lo + g; fsrc = lo + 1 + g; }
      else if (kind == BC_REFLECT) { src = hi - 1 - g; fsrc = hi - 1 - g; fsign = -1.0; }
      else { src = hi - 1; fsrc = hi; }
    }
    for (int b = 0; b < nb; b++) {
      for (int q = 0; q < ncen; q++) {
        double *a = cen[q];
        for (int i = 0; i < m->nx; i++) a[at(sd, i, dst, b)] = a[at(sd, i, src, b)];
      }
      if (fdst >= 0)
        for (int i = 0; i < m->nx; i++) vn[at(sd, i, fdst, b)] = fsign * vn[at(sd, i, fsrc, b)];
    }
  }
}

/* Y sides over every Z row, then Z sides over every Y column. */
static void boundary_fill(const mesh_t *m, orc_state *s) {
  const orc_params *p = m->p;
  side_t sy = {m, 1}, sz = {m, 2};
  double *cy[4];
  int n = 0;
  cy[n++] = s->rho;
  if (s->e) cy[n++] = s->e;
  cy[n++] = s->vx;
  if (m->d3) cy[n++] = s->vz;
  bc_faces(&sy, 0, p->bc[0], s->vy);
  bc_faces(&sy, 1, p->bc[1], s->vy);
  bc_ghosts(&sy, 0, p->bc[0], cy, n, s->vy);
  bc_ghosts(&sy, 1, p->bc[1], cy, n, s->vy);
  if (!m->d3) return;
  double *cz[4];
  n = 0;
  cz[n++] = s->rho;
  if (s->e) cz[n++] = s->e;
  cz[n++] = s->vx;
  cz[n++] = s->vy;
  bc_faces(&sz, 0, p->bc[2], s->vz);
  bc_faces(&sz, 1, p->bc[3], s->vz);
  bc_ghosts(&sz, 0, p->bc[2], cz, n, s->vz);
  bc_ghosts(&sz, 1, p->bc[3], cz, n, s->vz);
}

/* ------------------------------------------------------------------------ */
/* Box 3: bulk azimuthal velocity of each ring (Eq. 37, or the azimuthal mean) */
/* ------------------------------------------------------------------------ */
static void ring_v0(const mesh_t *m, const double *vx, double *v0 /* [nz][ny] active */) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      double vmax = vx[IX(0, j, k)], vmin = vmax, sum = 0.0;
      for (int i = 0; i < m->nx; i++) {
        double v = vx[IX(i, j, k)];
        if (v > vmax) vmax = v;
        if (v < vmin) vmin = v;
        sum += v;
      }
      v0[(size_t)(k - m->k0) * m->ny + (j - m->j0)] =
          m->p->v0_mean ? sum / m->nx : 0.5 * (vmax + vmin);
    }
}

/* Box 4: pressure, Eq. eos1 (c_s static) or Eq. eos2 */
static inline double pressure(const mesh_t *m, const orc_state *s, size_t c) {
  if (m->p->eos == EOS_ISO) return s->cs[c] * s->cs[c] * s->rho[c];
  return (m->p->gamma - 1.0) * s->e[c];
}

/* ------------------------------------------------------------------------ */
/* Box 6: time step, Eq. cfl2 with items 1-4, and Eq. 38                     */
/* ------------------------------------------------------------------------ */
/* Eq. cfl2 as written: every item of the list is a time step Delta_j over a
   speed, taken in each direction j of the mesh; the item's step dt_i is the
   smallest over the directions.  A cell combines its items as
   (sum_i dt_i^-2)^(-1/2), and the mesh step is C times the smallest cell step
   over the active zones.  An item that does not apply, or whose speed
   vanishes, is an infinite step and adds nothing to the sum.  Readings: the
   speed of item 2 is the larger magnitude of the two faces bounding the cell
   along j, with the residual velocity under orbital advection (Sect. 3.5.2);
   item 3 acts on compressed directions only, as L / (4 C_av^2 |dv|); item 4 is
   Delta^2 / (4 nu).  With orbital advection the shear limit of Eq. 38 is the
   smallest C0 / |v_x(j)/dX_j - v_x(j+1)/dX_(j+1)| over radially adjacent
   active zones, and the step is the smaller of the two. */
static double cfl_dt(const mesh_t *m, const orc_state *s, const double *v0, int *err) {
  const orc_params *p = m->p;
  double min_cell = INFINITY;  /* smallest (sum dt_i^-2)^(-1/2) */
  double min_shear = INFINITY; /* smallest shear step of Eq. 38 */
  int bad = 0;
  const double c2av = p->cvnr * p->cvnr;
  const int nd = m->d3 ? 3 : 2;
#pragma omp parallel for collapse(2) schedule(static) reduction(min : min_cell) reduction(min : min_shear) reduction(| : bad)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      double vbulk = p->fargo ? v0[(size_t)(k - m->k0) * m->ny + (j - m->j0)] : 0.0;
      double L[3] = {DXlen(m, j, k), Ly(m, j), m->d3 ? Lz(m, j, k) : 0.0};
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k);
        int ip = imod(i + 1, m->nx);
        /* velocities on the lower and upper faces of the cell along X, Y, Z */
        double vlo[3] = {s->vx[c], s->vy[c], m->d3 ? s->vz[c] : 0.0};
        double vup[3] = {s->vx[IX(ip, j, k)], s->vy[IX(i, j + 1, k)], m->d3 ? s->vz[IX(i, j, k + 1)] : 0.0};
        double rho = s->rho[c];
        /* sound speed: the static c_s, or sqrt(gamma P / rho) */
        double cw = (p->eos == EOS_ISO) ? s->cs[c] : sqrt(p->gamma * ((p->gamma - 1.0) * s->e[c]) / rho);
        if (!(rho > 0.0) || !isfinite(rho) || !isfinite(cw) || !isfinite(vlo[0]) || !isfinite(vlo[1]) ||
            !isfinite(vlo[2]))
          bad = 1;
        double dt1 = INFINITY, dt2 = INFINITY, dt3 = INFINITY, dt4 = INFINITY;
        for (int d = 0; d < nd; d++) {
          /* item 1: sound waves */
          if (cw > 0.0) dt1 = fmin(dt1, L[d] / cw);
          /* item 2: fluid motion (residual azimuthal velocity with orbital advection) */
          double blk = d == 0 ? vbulk : 0.0;
          double u = fmax(fabs(vlo[d] - blk), fabs(vup[d] - blk));
          if (u > 0.0) dt2 = fmin(dt2, L[d] / u);
          /* item 3: artificial viscosity, where the flow is compressed along d */
          double dv = vup[d] - vlo[d];
          if (dv < 0.0 && c2av > 0.0) dt3 = fmin(dt3, L[d] / (4.0 * c2av * fabs(dv)));
          /* item 4: kinematic viscosity */
          if (p->visc && s->nu[c] > 0.0) dt4 = fmin(dt4, L[d] * L[d] / (4.0 * s->nu[c]));
        }
        double sum = 1.0 / (dt1 * dt1) + 1.0 / (dt2 * dt2) + 1.0 / (dt3 * dt3) + 1.0 / (dt4 * dt4);
        double cell = 1.0 / sqrt(sum);
        if (cell < min_cell) min_cell = cell;
        /* Eq. 38 between this zone and its radial neighbour j + 1, both active */
        if (p->fargo && p->shear_c0 > 0.0 && j + 1 < m->jn) {
          double rate = fabs(s->vx[c] / L[0] - s->vx[IX(i, j + 1, k)] / DXlen(m, j + 1, k));
          if (rate > 0.0) {
            double tsh = p->shear_c0 / rate;
            if (tsh < min_shear) min_shear = tsh;
          }
        }
      }
    }
  double dt = p->courant * min_cell;
  if (p->fargo && p->shear_c0 > 0.0) dt = fmin(dt, min_shear);
  if (bad) *err = ORC_ENONFINITE;
  else if (!(dt > 0.0) || !isfinite(dt)) *err = ORC_ECFL;
  return dt;
}

/* ------------------------------------------------------------------------ */
/* Box 7: source step (Sect. 3.3)                                            */
/* ------------------------------------------------------------------------ */
/* Owned faces: all X faces; interior Y/Z faces, plus the lower boundary face
   in a periodic direction (whose upper boundary face is its ghost copy). */
static inline int ylo_face(const mesh_t *m) { return m->p->bc[0] == BC_PERIODIC ? m->j0 : m->j0 + 1; }
static inline int zlo_face(const mesh_t *m) { return m->p->bc[2] == BC_PERIODIC ? m->k0 : m->k0 + 1; }
/* neighbour below along Y/Z; periodic directions wrap within the active range */
static inline int jbelow(const mesh_t *m, int j) { return m->p->bc[0] == BC_PERIODIC ? wrap(j - 1, m->j0, m->ny) : j - 1; }
static inline int kbelow(const mesh_t *m, int k) { return m->p->bc[2] == BC_PERIODIC ? wrap(k - 1, m->k0, m->nz) : k - 1; }
static inline int jabove(const mesh_t *m, int j) { return m->p->bc[0] == BC_PERIODIC ? wrap(j + 1, m->j0, m->ny) : j + 1; }
static inline int kabove(const mesh_t *m, int k) { return m->p->bc[2] == BC_PERIODIC ? wrap(k + 1, m->k0, m->nz) : k + 1; }

/* Box 7a, substep 1 (Jacobi: every face reads only v^n, P, rho, Phi).
   Pressure term as in Eq. 20 (arithmetic mean of the face density), potential
   gradient across the face, centrifugal terms as arithmetic averages of four
   face velocities, then squared (Eq. 12 and its generalisation). */
static void substep1(const mesh_t *m, const orc_state *s, const double *P, double dt,
                     double *vx1, double *vy1, double *vz1) {
  const orc_params *p = m->p;
  const double om = p->omega;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      double dX = DXlen(m, j, k);
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k), cm = IX(imod(i - 1, m->nx), j, k);
        double gradP = 2.0 * (P[c] - P[cm]) / ((s->rho[c] + s->rho[cm]) * dX);
        double gradPhi = (s->pot[c] - s->pot[cm]) / dX;
        vx1[c] = s->vx[c] - dt * (gradP + gradPhi);
      }
    }
  /* Y faces */
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = ylo_face(m); j < m->jn; j++) {
      int jm = jbelow(m, j);
      double h = hy(m, j);
      for (int i = 0; i < m->nx; i++) {
        int ip = imod(i + 1, m->nx);
        size_t c = IX(i, j, k), cm = IX(i, jm, k);
        double gradP = 2.0 * (P[c] - P[cm]) / ((s->rho[c] + s->rho[cm]) * h);
        double gradPhi = (s->pot[c] - s->pot[cm]) / h;
        double src = 0.0;
        if (m->geo == GEO_CYL) {
          double vt = 0.25 * ((s->vx[c] + m->ymed[j] * om) + (s->vx[IX(ip, j, k)] + m->ymed[j] * om) +
                              (s->vx[cm] + m->ymed[jm] * om) + (s->vx[IX(ip, jm, k)] + m->ymed[jm] * om));
          src = vt * vt / m->ymin[j];
        } else if (m->geo == GEO_SPH) {
          double R0 = m->ymed[j] * m->sinzmed[k], R1 = m->ymed[jm] * m->sinzmed[k];
          double vt = 0.25 * ((s->vx[c] + R0 * om) + (s->vx[IX(ip, j, k)] + R0 * om) +
                              (s->vx[cm] + R1 * om) + (s->vx[IX(ip, jm, k)] + R1 * om));
          int kp = kabove(m, k);
          double vth = 0.25 * (s->vz[c] + s->vz[IX(i, j, kp)] + s->vz[cm] + s->vz[IX(i, jm, kp)]);
          src = (vt * vt + vth * vth) / m->ymin[j];
        }
        vy1[c] = s->vy[c] - dt * (gradP + gradPhi) + dt * src;
      }
    }
  if (!m->d3) return;
  /* Z faces */
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = zlo_face(m); k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      int km = kbelow(m, k);
      double h = hz(m, j, k);
      for (int i = 0; i < m->nx; i++) {
        int ip = imod(i + 1, m->nx);
        size_t c = IX(i, j, k), cm = IX(i, j, km);
        double gradP = 2.0 * (P[c] - P[cm]) / ((s->rho[c] + s->rho[cm]) * h);
        double gradPhi = (s->pot[c] - s->pot[cm]) / h;
        double src = 0.0;
        if (m->geo == GEO_SPH) {
          double R0 = m->ymed[j] * m->sinzmed[k], R1 = m->ymed[j] * m->sinzmed[km];
          double vt = 0.25 * ((s->vx[c] + R0 * om) + (s->vx[IX(ip, j, k)] + R0 * om) +
                              (s->vx[cm] + R1 * om) + (s->vx[IX(ip, j, km)] + R1 * om));
          src = vt * vt * (cos(m->zmin[k]) / sin(m->zmin[k])) / m->ymed[j];
        }
        vz1[c] = s->vz[c] - dt * (gradP + gradPhi) + dt * src;
      }
    }
}

/* Box 7b, substep 2: artificial viscous pressure per direction,
   q_d = C^2 rho (dv_d)^2 for dv_d < 0, its gradient on the owned faces (same
   momentum-conserving form as Eq. 20) and the heating -q_d dv_d / L_d. */
static void substep2(const mesh_t *m, orc_state *s, const double *vx1, const double *vy1, const double *vz1,
                     double dt, double *qx, double *qy, double *qz) {
  const orc_params *p = m->p;
  const double c2 = p->cvnr * p->cvnr;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      int jp = jabove(m, j), kp = m->d3 ? kabove(m, k) : k;
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k);
        double rho = s->rho[c];
        double dvx = vx1[IX(imod(i + 1, m->nx), j, k)] - vx1[c];
        double dvy = vy1[IX(i, jp, k)] - vy1[c];
        qx[c] = dvx < 0.0 ? c2 * rho * dvx * dvx : 0.0;
        qy[c] = dvy < 0.0 ? c2 * rho * dvy * dvy : 0.0;
        double heat = qx[c] * dvx / DXlen(m, j, k) + qy[c] * dvy / Ly(m, j);
        if (m->d3) {
          double dvz = vz1[IX(i, j, kp)] - vz1[c];
          qz[c] = dvz < 0.0 ? c2 * rho * dvz * dvz : 0.0;
          heat += qz[c] * dvz / Lz(m, j, k);
        }
        if (p->eos == EOS_ADI) s->e[c] = s->e[c] - dt * heat;
      }
    }
  /* velocity update from the viscous pressure gradient: v'' -> state arrays */
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      double dX = DXlen(m, j, k);
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k), cm = IX(imod(i - 1, m->nx), j, k);
        s->vx[c] = vx1[c] - dt * 2.0 * (qx[c] - qx[cm]) / ((s->rho[c] + s->rho[cm]) * dX);
      }
    }
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = ylo_face(m); j < m->jn; j++) {
      int jm = jbelow(m, j);
      double h = hy(m, j);
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k), cm = IX(i, jm, k);
        s->vy[c] = vy1[c] - dt * 2.0 * (qy[c] - qy[cm]) / ((s->rho[c] + s->rho[cm]) * h);
      }
    }
  if (!m->d3) return;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = zlo_face(m); k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      int km = kbelow(m, k);
      double h = hz(m, j, k);
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k), cm = IX(i, j, km);
        s->vz[c] = vz1[c] - dt * 2.0 * (qz[c] - qz[cm]) / ((s->rho[c] + s->rho[cm]) * h);
      }
    }
}

/* Box 7d: viscous stress of a kinematic viscosity nu, cylindrical 2D
   (phi, r), in the component forms of App. B (Eq. 73) and their divergence
   (Eq. 76).  The diagonal components sit at zone centres; tau_rphi sits on
   the zone's lower edge in both X and Y (Fig. "stress"), where rho and nu
   are the means of the four zones sharing it and v_phi/r is the mean of
   v_phi/r on the two X faces it joins.  All components come from the
   velocities after 7b (Jacobi); then v_phi (X faces of active zones) and v_r
   (owned Y faces) are updated, with the face density of Eq. 20. */
static void substep_visc(const mesh_t *m, orc_state *s, double dt, double *tpp, double *trr, double *trp) {
  const double dphi = m->dx;
  const int nx = m->nx;
  /* zone-centred components on the active rows */
#pragma omp parallel for schedule(static)
  for (int j = m->j0; j < m->jn; j++) {
    double r = m->ymed[j];
    for (int i = 0; i < nx; i++) {
      size_t c = IX(i, j, 0), cxp = IX(imod(i + 1, nx), j, 0), cyp = IX(i, j + 1, 0);
      double divv = Vinv(m, j, 0) * (Sx(m, j, 0) * (s->vx[cxp] - s->vx[c]) +
                                     (Sy(m, j + 1, 0) * s->vy[cyp] - Sy(m, j, 0) * s->vy[c]));
      double rn = s->rho[c] * s->nu[c];
      double ur = 0.5 * (s->vy[c] + s->vy[cyp]);
      tpp[c] = -rn * (2.0 * ((s->vx[cxp] - s->vx[c]) / (r * dphi) + ur / r) - 2.0 / 3.0 * divv);
      trr[c] = -rn * (2.0 * (s->vy[cyp] - s->vy[c]) / Ly(m, j) - 2.0 / 3.0 * divv);
    }
  }
  /* edge component on the Y faces j0 .. jn (the edge at the lower X face) */
#pragma omp parallel for schedule(static)
  for (int j = m->j0; j <= m->jn; j++) {
    for (int i = 0; i < nx; i++) {
      int im = imod(i - 1, nx);
      size_t c = IX(i, j, 0), cw = IX(im, j, 0), cs_ = IX(i, j - 1, 0), csw = IX(im, j - 1, 0);
      double rho4 = 0.25 * (s->rho[c] + s->rho[cw] + s->rho[cs_] + s->rho[csw]);
      double nu4 = 0.25 * (s->nu[c] + s->nu[cw] + s->nu[cs_] + s->nu[csw]);
      double dvphi_dr = (s->vx[c] - s->vx[cs_]) / hy(m, j);
      double vphi_r = 0.5 * (s->vx[c] / m->ymed[j] + s->vx[cs_] / m->ymed[j - 1]);
      double dvr_dphi = (s->vy[c] - s->vy[cw]) / (m->ymin[j] * dphi);
      trp[c] = -rho4 * nu4 * (dvphi_dr - vphi_r + dvr_dphi);
    }
  }
  /* v_phi on the X faces of the active zones */
#pragma omp parallel for schedule(static)
  for (int j = m->j0; j < m->jn; j++) {
    double r = m->ymed[j], a = m->ymin[j], b = m->ymin[j + 1];
    for (int i = 0; i < nx; i++) {
      int im = imod(i - 1, nx);
      size_t c = IX(i, j, 0), cw = IX(im, j, 0), cn = IX(i, j + 1, 0);
      double rho_f = 0.5 * (s->rho[c] + s->rho[cw]);
      double div = (b * b * trp[cn] - a * a * trp[c]) / (r * r * Ly(m, j)) + (tpp[c] - tpp[cw]) / (r * dphi);
      s->vx[c] -= dt * div / rho_f;
    }
  }
  /* v_r on the owned Y faces */
#pragma omp parallel for schedule(static)
  for (int j = ylo_face(m); j < m->jn; j++) {
    double a = m->ymin[j];
    for (int i = 0; i < nx; i++) {
      size_t c = IX(i, j, 0), cs_ = IX(i, j - 1, 0), ce = IX(imod(i + 1, nx), j, 0);
      double rho_f = 0.5 * (s->rho[c] + s->rho[cs_]);
      double div = (m->ymed[j] * trr[c] - m->ymed[j - 1] * trr[cs_]) / (a * hy(m, j)) +
                   (trp[ce] - trp[c]) / (a * dphi) - 0.5 * (tpp[c] + tpp[cs_]) / a;
      s->vy[c] -= dt * div / rho_f;
    }
  }
}

/* Box 7c, substep 3: work of the pressure forces on a gamma-law gas,
   time-centred: e <- e (1 - a)/(1 + a), a = dt (gamma-1) div(v) / 2, with the
   divergence from the face fluxes of the updated velocities. */
static void substep3(const mesh_t *m, orc_state *s, double dt) {
  const double gm1 = m->p->gamma - 1.0;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      int jp = jabove(m, j), kp = m->d3 ? kabove(m, k) : k;
      double sx = Sx(m, j, k), sy0 = Sy(m, j, k), sy1 = Sy(m, j + 1, k), vinv = Vinv(m, j, k);
      double sz0 = m->d3 ? Sz(m, j, k) : 0.0, sz1 = m->d3 ? Sz(m, j, k + 1) : 0.0;
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k);
        double flux = sx * (s->vx[IX(imod(i + 1, m->nx), j, k)] - s->vx[c]) +
                      (sy1 * s->vy[IX(i, jp, k)] - sy0 * s->vy[c]);
        if (m->d3) flux += sz1 * s->vz[IX(i, j, kp)] - sz0 * s->vz[c];
        double divv = vinv * flux;
        double a = 0.5 * dt * gm1 * divv;
        s->e[c] = s->e[c] * (1.0 - a) / (1.0 + a);
      }
    }
}

/* ------------------------------------------------------------------------ */
/* Box 12: transport                                                          */
/* ------------------------------------------------------------------------ */
/* van Leer slope of cell c (Sect. 3.4): harmonic mean of the one-sided
   differences per unit length, zero unless both have the same sign. */
static inline double vanleer(double qm, double q0, double qp, double hm, double hp) {
  double dl = (q0 - qm) / hm, dr = (qp - q0) / hp;
  double pr = dl * dr;
  return pr > 0.0 ? 2.0 * pr / (dl + dr) : 0.0;
}

/* One directional upwind update of rho and of nq other cell-centred
   quantities along a line of n zones (Eqs. flux, 14, 15 and consistent
   transport).  Zone c in [-2, n+1] is stored at index c+2; face f in [0, n]
   separates zones f-1 and f and carries the normal velocity w[f], the area
   S[f]; h[f+1] is the distance between the centres of zones f-1 and f for
   f in [-1, n+1]; L[c+2] is the width of zone c; Vi[c] the inverse volume of
   active zone c.  rho and Q[q] are updated on zones 0..n-1 only.  `work`
   holds 4*(n+5) doubles. */
static void sweep_line(int n, int nq, double *rho, double **Q, const double *w, const double *L,
                       const double *h, const double *S, const double *Vi, double dt, double *work) {
  double *slope = work;            /* zones -1..n at index c+1 */
  double *Frho = work + (n + 5);   /* faces 0..n */
  double *qq = work + 2 * (n + 5); /* zones -2..n+1 at index c+2 */
  double *FQ = work + 3 * (n + 5); /* faces 0..n */
#define VL(arr, c) vanleer(arr[(c) + 1], arr[(c) + 2], arr[(c) + 3], h[(c) + 1], h[(c) + 2])
  /* interface value at face f at half time step, upwinded on w[f] (Eq. 15) */
#define STAR(arr, f)                                                                              \
  (w[f] >= 0.0 ? arr[(f) - 1 + 2] + slope[(f) - 1 + 1] * (L[(f) - 1 + 2] - w[f] * dt) * 0.5 \
               : arr[(f) + 2] - slope[(f) + 1] * (L[(f) + 2] + w[f] * dt) * 0.5)
  for (int c = -1; c <= n; c++) slope[c + 1] = VL(rho, c);
  for (int f = 0; f <= n; f++) Frho[f] = w[f] * STAR(rho, f) * S[f] * dt;
  for (int q = 0; q < nq; q++) {
    double *a = Q[q];
    for (int c = -2; c <= n + 1; c++) qq[c + 2] = a[c + 2] / rho[c + 2];
    for (int c = -1; c <= n; c++) slope[c + 1] = VL(qq, c);
    for (int f = 0; f <= n; f++) FQ[f] = STAR(qq, f) * Frho[f];
    for (int c = 0; c < n; c++) a[c + 2] = a[c + 2] - Vi[c] * (FQ[c + 1] - FQ[c]);
  }
  for (int c = 0; c < n; c++) rho[c + 2] = rho[c + 2] - Vi[c] * (Frho[c + 1] - Frho[c]);
#undef VL
#undef STAR
}

/* PPA interface values of a periodic ring for a uniform fractional shift xi
   (Eqs. 34-36 and the interface formula of Sect. 3.5.1): qstar[f] at face f,
   between zones f-1 and f.  The upwind zone is f-1 for xi >= 0, f for xi < 0;
   the fraction is |xi|. */
static void ppa_faces(int n, const double *q, double xi, double *qstar, double *dm, double *QL, double *QR) {
  /* Eq. 34: monotonised centred slope */
  for (int i = 0; i < n; i++) {
    double qm = q[imod(i - 1, n)], q0 = q[i], qp = q[imod(i + 1, n)];
    double dq = 0.5 * (qp - qm);
    if ((qp - q0) * (q0 - qm) <= 0.0) dm[i] = 0.0;
    else {
      double mag = fmin(fmin(2.0 * fabs(q0 - qm), 2.0 * fabs(qp - q0)), fabs(dq));
      dm[i] = dq > 0.0 ? mag : -mag;
    }
  }
  /* Eq. 35: parabolic interface values, Q^R_i = Q^L_{i+1} */
  for (int i = 0; i < n; i++) {
    int ip = imod(i + 1, n);
    double qr = q[i] + 0.5 * (q[ip] - q[i]) - (dm[ip] - dm[i]) / 6.0;
    QR[i] = qr;
    QL[ip] = qr;
  }
  /* Eq. 36: remove extrema created by the parabola */
  for (int i = 0; i < n; i++) {
    double qm = q[imod(i - 1, n)], q0 = q[i], qp = q[imod(i + 1, n)];
    double l = QL[i], r = QR[i];
    double D = r - l, C = q0 - 0.5 * (l + r);
    if ((qp - q0) * (q0 - qm) <= 0.0) { l = q0; r = q0; }
    else if (D * C > D * D / 6.0) l = 3.0 * q0 - 2.0 * r;
    else if (-D * D / 6.0 > D * C) r = 3.0 * q0 - 2.0 * l;
    dm[i] = l; /* reuse as storage for the limited left value */
    QR[i] = r;
  }
  for (int i = 0; i < n; i++) QL[i] = dm[i];
  double x = fabs(xi);
  for (int f = 0; f < n; f++) {
    int u = xi >= 0.0 ? imod(f - 1, n) : f;
    if (xi >= 0.0)
      qstar[f] = QR[u] + x * (q[u] - QR[u]) + x * (1.0 - x) * (2.0 * q[u] - QR[u] - QL[u]);
    else
      qstar[f] = QL[u] + x * (q[u] - QL[u]) + x * (1.0 - x) * (2.0 * q[u] - QR[u] - QL[u]);
  }
}

/* Fractional uniform residual of orbital advection on one ring (Eq. 33), with
   PPA interface values and consistent transport.  The mass flux through a face
   is v^R dt S rho* = xi dX S rho*.  `work` holds 6*n doubles. */
static void ppa_ring(int n, int nq, double *rho, double **Q, double xi, double dX, double S, double vinv,
                     double *work) {
  double *Frho = work, *star = work + n, *qq = work + 2 * n, *a = work + 3 * n, *b = work + 4 * n,
         *c = work + 5 * n;
  ppa_faces(n, rho, xi, star, a, b, c);
  for (int f = 0; f < n; f++) Frho[f] = xi * dX * S * star[f];
  for (int q = 0; q < nq; q++) {
    double *A = Q[q];
    for (int i = 0; i < n; i++) qq[i] = A[i] / rho[i];
    ppa_faces(n, qq, xi, star, a, b, c);
    for (int f = 0; f < n; f++) star[f] = star[f] * Frho[f];
    for (int i = 0; i < n; i++) A[i] = A[i] - vinv * (star[imod(i + 1, n)] - star[i]);
  }
  for (int i = 0; i < n; i++) rho[i] = rho[i] - vinv * (Frho[imod(i + 1, n)] - Frho[i]);
}

/* Eq. 32: Q_i <- Q_{i-N}, a circular permutation of the ring */
static void shift_ring(int n, double *a, int N, double *tmp) {
  for (int i = 0; i < n; i++) tmp[i] = a[imod(i - N, n)];
  memcpy(a, tmp, sizeof(double) * n);
}

/* Split of the bulk displacement into an integer number of zones and a
   residual (Eq. 29): D = v0 dt / dX, N = nearest integer to D (ties away from
   zero), xi = D - N (exact in binary floating point, |xi| <= 1/2). */
static void split_shift(double v0, double dt, double dX, int32_t *N, double *xi) {
  double D = (v0 * dt) / dX;
  double r = round(D);
  *N = (int32_t)r;
  *xi = D - r;
}

/* X-momentum factor of Tab. "momenta": the transported quantity is rho*mx(v) */
static inline double mx_of(const mesh_t *m, int j, int k, double v) {
  if (m->geo == GEO_CART) return v;
  double R = Rcyl(m, j, k);
  return R * (v + R * m->p->omega);
}
static inline double vx_of(const mesh_t *m, int j, int k, double mom) {
  if (m->geo == GEO_CART) return mom;
  double R = Rcyl(m, j, k);
  return mom / R - R * m->p->omega;
}
/* Z-momentum factor: rho v_z, or rho r v_theta in spherical geometry */
static inline double mz_of(const mesh_t *m, int j, double v) { return m->geo == GEO_SPH ? m->ymed[j] * v : v; }

enum { T_RHO = 0, T_PXM, T_PXP, T_PYM, T_PYP, T_PZM, T_PZP, T_E, T_MAX };

typedef struct {
  double *a[T_MAX];
  int nq;              /* number of transported quantities other than rho */
  double *list[T_MAX]; /* the non-density quantities, in a fixed order */
} tset_t;

/* Box 12a: left and right momenta (Eqs. 16, 17 with Tab. "momenta"), computed
   in every zone whose faces exist, ghosts included. */
static void momenta(const mesh_t *m, const orc_state *s, tset_t *T) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < m->nzg; k++)
    for (int j = 0; j < m->nyg; j++)
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k);
        double rho = s->rho[c];
        T->a[T_RHO][c] = rho;
        T->a[T_PXM][c] = rho * mx_of(m, j, k, s->vx[c]);
        T->a[T_PXP][c] = rho * mx_of(m, j, k, s->vx[IX(imod(i + 1, m->nx), j, k)]);
        T->a[T_PYM][c] = rho * s->vy[c];
        T->a[T_PYP][c] = (j + 1 < m->nyg) ? rho * s->vy[IX(i, j + 1, k)] : 0.0;
        if (m->d3) {
          T->a[T_PZM][c] = rho * mz_of(m, j, s->vz[c]);
          T->a[T_PZP][c] = (k + 1 < m->nzg) ? rho * mz_of(m, j, s->vz[IX(i, j, k + 1)]) : 0.0;
        }
        if (s->e) T->a[T_E][c] = s->e[c];
      }
}

/* Y sweep (Eq. 1D-advection-Y) on active j, for the active Z rows and the two
   nearest ghost rows on each Z side, which the Z sweep reads next. */
static void sweep_y(const mesh_t *m, const orc_state *s, tset_t *T, double dt) {
  int n = m->ny;
  int klo = m->d3 ? m->k0 - 2 : 0, khi = m->d3 ? m->kn + 2 : 1;
#pragma omp parallel
  {
    double *buf = malloc(sizeof(double) * ((size_t)(T_MAX + 5) * (n + 5) + 4 * (n + 5)));
    double *rho = buf, *Q[T_MAX];
    for (int q = 0; q < T->nq; q++) Q[q] = buf + (size_t)(q + 1) * (n + 5);
    double *w = buf + (size_t)(T_MAX + 0) * (n + 5), *L = buf + (size_t)(T_MAX + 1) * (n + 5);
    double *h = buf + (size_t)(T_MAX + 2) * (n + 5), *S = buf + (size_t)(T_MAX + 3) * (n + 5);
    double *vi = buf + (size_t)(T_MAX + 4) * (n + 5);
    double *work = buf + (size_t)(T_MAX + 5) * (n + 5);
#pragma omp for collapse(2) schedule(static)
    for (int k = klo; k < khi; k++)
      for (int i = 0; i < m->nx; i++) {
        for (int c = -2; c <= n + 1; c++) {
          int j = m->j0 + c;
          rho[c + 2] = T->a[T_RHO][IX(i, j, k)];
          for (int q = 0; q < T->nq; q++) Q[q][c + 2] = T->list[q][IX(i, j, k)];
          L[c + 2] = Ly(m, j);
        }
        for (int f = -1; f <= n + 1; f++) h[f + 1] = hy(m, m->j0 + f);
        for (int f = 0; f <= n; f++) {
          w[f] = s->vy[IX(i, m->j0 + f, k)];
          S[f] = Sy(m, m->j0 + f, k);
        }
        for (int c = 0; c < n; c++) vi[c] = Vinv(m, m->j0 + c, k);
        sweep_line(n, T->nq, rho, Q, w, L, h, S, vi, dt, work);
        for (int c = 0; c < n; c++) {
          int j = m->j0 + c;
          T->a[T_RHO][IX(i, j, k)] = rho[c + 2];
          for (int q = 0; q < T->nq; q++) T->list[q][IX(i, j, k)] = Q[q][c + 2];
        }
      }
    free(buf);
  }
}

/* Z sweep (Eq. 1D-advection-Z) on active zones */
static void sweep_z(const mesh_t *m, const orc_state *s, tset_t *T, double dt) {
  int n = m->nz;
#pragma omp parallel
  {
    double *buf = malloc(sizeof(double) * ((size_t)(T_MAX + 5) * (n + 5) + 4 * (n + 5)));
    double *rho = buf, *Q[T_MAX];
    for (int q = 0; q < T->nq; q++) Q[q] = buf + (size_t)(q + 1) * (n + 5);
    double *w = buf + (size_t)(T_MAX + 0) * (n + 5), *L = buf + (size_t)(T_MAX + 1) * (n + 5);
    double *h = buf + (size_t)(T_MAX + 2) * (n + 5), *S = buf + (size_t)(T_MAX + 3) * (n + 5);
    double *vi = buf + (size_t)(T_MAX + 4) * (n + 5);
    double *work = buf + (size_t)(T_MAX + 5) * (n + 5);
#pragma omp for collapse(2) schedule(static)
    for (int j = m->j0; j < m->jn; j++)
      for (int i = 0; i < m->nx; i++) {
        for (int c = -2; c <= n + 1; c++) {
          int k = m->k0 + c;
          rho[c + 2] = T->a[T_RHO][IX(i, j, k)];
          for (int q = 0; q < T->nq; q++) Q[q][c + 2] = T->list[q][IX(i, j, k)];
          L[c + 2] = Lz(m, j, k);
        }
        for (int f = -1; f <= n + 1; f++) h[f + 1] = hz(m, j, m->k0 + f);
        for (int f = 0; f <= n; f++) {
          w[f] = s->vz[IX(i, j, m->k0 + f)];
          S[f] = Sz(m, j, m->k0 + f);
        }
        for (int c = 0; c < n; c++) vi[c] = Vinv(m, j, m->k0 + c);
        sweep_line(n, T->nq, rho, Q, w, L, h, S, vi, dt, work);
        for (int c = 0; c < n; c++) {
          int k = m->k0 + c;
          T->a[T_RHO][IX(i, j, k)] = rho[c + 2];
          for (int q = 0; q < T->nq; q++) T->list[q][IX(i, j, k)] = Q[q][c + 2];
        }
      }
    free(buf);
  }
}

/* X transport of each active ring.  Without orbital advection: one van Leer
   sweep with v_x.  With it: a van Leer sweep with the residual velocity
   v_x - v0 (Eq. fargo1), the circular shift by N zones (Eq. 32), then the PPA
   fractional residual xi (Eq. 33). */
static void sweep_x(const mesh_t *m, const orc_state *s, tset_t *T, const double *v0, double dt) {
  int n = m->nx;
#pragma omp parallel
  {
    double *buf = malloc(sizeof(double) * ((size_t)(T_MAX + 5) * (n + 5) + 6 * (size_t)n + 4 * (n + 5)));
    double *rho = buf, *Q[T_MAX];
    for (int q = 0; q < T->nq; q++) Q[q] = buf + (size_t)(q + 1) * (n + 5);
    double *w = buf + (size_t)(T_MAX + 0) * (n + 5), *L = buf + (size_t)(T_MAX + 1) * (n + 5);
    double *h = buf + (size_t)(T_MAX + 2) * (n + 5), *S = buf + (size_t)(T_MAX + 3) * (n + 5);
    double *vi = buf + (size_t)(T_MAX + 4) * (n + 5);
    double *work = buf + (size_t)(T_MAX + 5) * (n + 5);
    double *pwork = work + 4 * (n + 5);
#pragma omp for collapse(2) schedule(static)
    for (int k = m->k0; k < m->kn; k++)
      for (int j = m->j0; j < m->jn; j++) {
        size_t r = (size_t)(k - m->k0) * m->ny + (j - m->j0);
        double vb = m->p->fargo ? v0[r] : 0.0;
        double dX = DXlen(m, j, k), sx = Sx(m, j, k), vinv = Vinv(m, j, k);
        for (int c = -2; c <= n + 1; c++) {
          size_t cc = IX(imod(c, n), j, k);
          rho[c + 2] = T->a[T_RHO][cc];
          for (int q = 0; q < T->nq; q++) Q[q][c + 2] = T->list[q][cc];
          L[c + 2] = dX;
        }
        for (int f = -1; f <= n + 1; f++) h[f + 1] = dX;
        for (int f = 0; f <= n; f++) {
          w[f] = s->vx[IX(imod(f, n), j, k)] - vb;
          S[f] = sx;
        }
        for (int c = 0; c < n; c++) vi[c] = vinv;
        sweep_line(n, T->nq, rho, Q, w, L, h, S, vi, dt, work);
        /* ring views on the active zones */
        double *rr = rho + 2, *QQ[T_MAX];
        for (int q = 0; q < T->nq; q++) QQ[q] = Q[q] + 2;
        if (m->p->fargo) {
          int32_t N;
          double xi;
          split_shift(v0[r], dt, dX, &N, &xi);
          shift_ring(n, rr, N, pwork);
          for (int q = 0; q < T->nq; q++) shift_ring(n, QQ[q], N, pwork);
          ppa_ring(n, T->nq, rr, QQ, xi, dX, sx, vinv, pwork);
        }
        for (int i = 0; i < n; i++) {
          T->a[T_RHO][IX(i, j, k)] = rr[i];
          for (int q = 0; q < T->nq; q++) T->list[q][IX(i, j, k)] = QQ[q][i];
        }
      }
    free(buf);
  }
}

/* Box 12d: velocities from the transported momenta and density (Eq. 18),
   on the owned faces; density and energy of the active zones. */
static void velocities(const mesh_t *m, orc_state *s, const tset_t *T) {
  double *const *a = T->a;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++)
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k), cm = IX(imod(i - 1, m->nx), j, k);
        double mom = (a[T_PXP][cm] + a[T_PXM][c]) / (a[T_RHO][cm] + a[T_RHO][c]);
        s->vx[c] = vx_of(m, j, k, mom);
      }
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = ylo_face(m); j < m->jn; j++) {
      int jm = jbelow(m, j);
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k), cm = IX(i, jm, k);
        s->vy[c] = (a[T_PYP][cm] + a[T_PYM][c]) / (a[T_RHO][cm] + a[T_RHO][c]);
      }
    }
  if (m->d3) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = zlo_face(m); k < m->kn; k++)
      for (int j = m->j0; j < m->jn; j++) {
        int km = kbelow(m, k);
        for (int i = 0; i < m->nx; i++) {
          size_t c = IX(i, j, k), cm = IX(i, j, km);
          double v = (a[T_PZP][cm] + a[T_PZM][c]) / (a[T_RHO][cm] + a[T_RHO][c]);
          s->vz[c] = (m->geo == GEO_SPH) ? v / m->ymed[j] : v;
        }
      }
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++)
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k);
        s->rho[c] = a[T_RHO][c];
        if (s->e) s->e[c] = a[T_E][c];
      }
}

static int state_ok(const mesh_t *m, const orc_state *s) {
  if (!s || !s->rho || !s->vx || !s->vy || !s->pot) return 0;
  if (m->d3 && !s->vz) return 0;
  if (m->p->eos == EOS_ISO && !s->cs) return 0;
  if (m->p->eos == EOS_ADI && !s->e) return 0;
  if (m->p->visc && !s->nu) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                      */
/* ------------------------------------------------------------------------ */

/* Boxes 2, 3, 4, 6: boundary fill of the state's ghosts, then the time step. */
int orc_cfl_dt(const orc_params *p, orc_state *s, double *dt_out) {
  mesh_t mm, *m = &mm;
  int rc = mesh_init(m, p);
  if (rc) return rc;
  if (!state_ok(m, s)) { mesh_free(m); return ORC_EINVAL; }
  double *v0 = malloc(sizeof(double) * (size_t)m->ny * m->nz);
  if (!v0) { mesh_free(m); return ORC_ENOMEM; }
  boundary_fill(m, s);
  ring_v0(m, s->vx, v0);
  int err = 0;
  double dt = cfl_dt(m, s, v0, &err);
  if (dt_out) *dt_out = dt;
  free(v0);
  mesh_free(m);
  return err;
}

/* One full update.  dt_in > 0 imposes the time step, otherwise Eq. cfl2 sets
   it; the step used is returned in *dt_out. */
int orc_step(const orc_params *p, orc_state *s, double dt_in, double *dt_out) {
  mesh_t mm, *m = &mm;
  int rc = mesh_init(m, p);
  if (rc) return rc;
  if (!state_ok(m, s)) { mesh_free(m); return ORC_EINVAL; }
  size_t nc = m->nc;
  int nring = m->ny * m->nz;
  double *v0 = malloc(sizeof(double) * nring);
  double *P = malloc(sizeof(double) * nc);
  double *v1[3] = {malloc(sizeof(double) * nc), malloc(sizeof(double) * nc), m->d3 ? malloc(sizeof(double) * nc) : NULL};
  double *q[3] = {calloc(nc, sizeof(double)), calloc(nc, sizeof(double)), m->d3 ? calloc(nc, sizeof(double)) : NULL};
  tset_t T;
  memset(&T, 0, sizeof(T));
  int ok = v0 && P && v1[0] && v1[1] && q[0] && q[1] && (!m->d3 || (v1[2] && q[2]));
  for (int t = 0; t < T_MAX && ok; t++) {
    int need = (t <= T_PYP) || (m->d3 && (t == T_PZM || t == T_PZP)) || (t == T_E && s->e);
    if (need) {
      T.a[t] = malloc(sizeof(double) * nc);
      if (!T.a[t]) ok = 0;
      else if (t != T_RHO) T.list[T.nq++] = T.a[t];
    }
  }
  int err = ok ? 0 : ORC_ENOMEM;
  double dt = dt_in;
  if (!err) {
    boundary_fill(m, s);                          /* box 2 */
    ring_v0(m, s->vx, v0);                        /* box 3 */
    int cerr = 0;
    double dtc = cfl_dt(m, s, v0, &cerr);         /* boxes 4, 6 */
    if (!(dt_in > 0.0)) { dt = dtc; err = cerr; }
    else if (cerr == ORC_ENONFINITE) err = cerr;
  }
  if (!err) {
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < nc; c++) P[c] = pressure(m, s, c); /* box 4 */
    memcpy(v1[0], s->vx, sizeof(double) * nc);
    memcpy(v1[1], s->vy, sizeof(double) * nc);
    if (m->d3) memcpy(v1[2], s->vz, sizeof(double) * nc);
    substep1(m, s, P, dt, v1[0], v1[1], v1[2]);   /* box 7a */
    substep2(m, s, v1[0], v1[1], v1[2], dt, q[0], q[1], q[2]); /* box 7b */
    if (p->visc) substep_visc(m, s, dt, q[0], q[1], P); /* box 7d (q and P reused as scratch) */
    if (p->eos == EOS_ADI) substep3(m, s, dt);    /* box 7c */
    boundary_fill(m, s);                          /* box 9 */
    momenta(m, s, &T);                            /* box 12a */
    sweep_y(m, s, &T, dt);                        /* box 12b/c */
    if (m->d3) sweep_z(m, s, &T, dt);
    sweep_x(m, s, &T, v0, dt);
    velocities(m, s, &T);                         /* box 12d */
  }
  if (dt_out) *dt_out = dt;
  free(v0); free(P);
  for (int d = 0; d < 3; d++) { free(v1[d]); free(q[d]); }
  for (int t = 0; t < T_MAX; t++) free(T.a[t]);
  mesh_free(m);
  return err;
}

/* Boxes 3 and the orbital-advection split on active rings: v0[r], N[r], xi[r]
   with r = (k-k0)*ny + (j-j0). */
int orc_ring_split(const orc_params *p, const double *vx, double dt, double *v0, int32_t *N, double *xi) {
  mesh_t mm, *m = &mm;
  int rc = mesh_init(m, p);
  if (rc) return rc;
  ring_v0(m, vx, v0);
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      size_t r = (size_t)(k - m->k0) * m->ny + (j - m->j0);
      split_shift(v0[r], dt, DXlen(m, j, k), &N[r], &xi[r]);
    }
  mesh_free(m);
  return ORC_OK;
}

/* Eq. 32 on every active ring of one field, in place. */
int orc_shift(const orc_params *p, double *field, const int32_t *N) {
  mesh_t mm, *m = &mm;
  int rc = mesh_init(m, p);
  if (rc) return rc;
  double *tmp = malloc(sizeof(double) * m->nx);
  if (!tmp) { mesh_free(m); return ORC_ENOMEM; }
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++)
      shift_ring(m->nx, field + IX(0, j, k), N[(size_t)(k - m->k0) * m->ny + (j - m->j0)], tmp);
  free(tmp);
  mesh_free(m);
  return ORC_OK;
}

/* Conserved sums over active zones, Neumaier-compensated, sequential (upper
   faces in a periodic direction are read through the wrap):
   out[0] = sum rho V, out[1] = sum rho mx(<v_x>) V with <v_x> the mean of the
   two X faces (Eq. 19), out[2] = sum rho <v_y> V, out[3] = sum rho mz(<v_z>) V,
   out[4] = sum e V.  abs_out (nullable) receives the sums of |term|. */
int orc_sums(const orc_params *p, const orc_state *s, double *out, double *abs_out) {
  mesh_t mm, *m = &mm;
  int rc = mesh_init(m, p);
  if (rc) return rc;
  double sum[5] = {0}, comp[5] = {0}, asum[5] = {0};
  for (int k = m->k0; k < m->kn; k++)
    for (int j = m->j0; j < m->jn; j++) {
      double V = Vol(m, j, k);
      int jp = jabove(m, j), kp = m->d3 ? kabove(m, k) : k;
      for (int i = 0; i < m->nx; i++) {
        size_t c = IX(i, j, k);
        double rho = s->rho[c];
        double t[5];
        t[0] = rho * V;
        t[1] = rho * 0.5 * (mx_of(m, j, k, s->vx[c]) + mx_of(m, j, k, s->vx[IX(imod(i + 1, m->nx), j, k)])) * V;
        t[2] = rho * 0.5 * (s->vy[c] + s->vy[IX(i, jp, k)]) * V;
        t[3] = m->d3 ? rho * 0.5 * (mz_of(m, j, s->vz[c]) + mz_of(m, j, s->vz[IX(i, j, kp)])) * V : 0.0;
        t[4] = s->e ? s->e[c] * V : 0.0;
        for (int q = 0; q < 5; q++) {
          double a = sum[q], b = t[q], x = a + b;
          comp[q] += (fabs(a) >= fabs(b)) ? (a - x) + b : (b - x) + a;
          sum[q] = x;
          asum[q] += fabs(b);
        }
      }
    }
  for (int q = 0; q < 5; q++) {
    out[q] = sum[q] + comp[q];
    if (abs_out) abs_out[q] = asum[q];
  }
  mesh_free(m);
  return ORC_OK;
}

/* Geometric tables for tests: per (k, j) with index k*nyg + j over the whole
   mesh, ghosts included.  Any output pointer may be NULL. */
int orc_geometry(const orc_params *p, double *vol, double *sx, double *sy, double *sz, double *dxlen) {
  mesh_t mm, *m = &mm;
  int rc = mesh_init(m, p);
  if (rc) return rc;
  for (int k = 0; k < m->nzg; k++)
    for (int j = 0; j < m->nyg; j++) {
      size_t r = (size_t)k * m->nyg + j;
      if (vol) vol[r] = Vol(m, j, k);
      if (sx) sx[r] = Sx(m, j, k);
      if (sy) sy[r] = Sy(m, j, k);
      if (sz) sz[r] = Sz(m, j, k);
      if (dxlen) dxlen[r] = DXlen(m, j, k);
    }
  mesh_free(m);
  return ORC_OK;
}

/* Unit-level access to the transport kernels, for pins against closed forms. */
void orc_sweep_line(int n, int nq, double *rho, double **Q, const double *w, const double *L, const double *h,
                    const double *S, const double *Vi, double dt) {
  double *work = malloc(sizeof(double) * 4 * (size_t)(n + 5));
  sweep_line(n, nq, rho, Q, w, L, h, S, Vi, dt, work);
  free(work);
}

void orc_ppa_faces(int n, const double *q, double xi, double *qstar) {
  double *w = malloc(sizeof(double) * 3 * (size_t)n);
  ppa_faces(n, q, xi, qstar, w, w + n, w + 2 * n);
  free(w);
}

void orc_ppa_ring(int n, int nq, double *rho, double **Q, double xi, double dX, double S, double vinv) {
  double *w = malloc(sizeof(double) * 6 * (size_t)n);
  ppa_ring(n, nq, rho, Q, xi, dX, S, vinv, w);
  free(w);
}

void orc_split_shift(double v0, double dt, double dX, int32_t *N, double *xi) { split_shift(v0, dt, dX, N, xi); }

/* Threads the oracle's parallel loops use. */
int orc_num_threads(void) { return omp_get_max_threads(); }
/* Thread count of later parallel regions (timing on a given number of cores);
   the arithmetic of a zone does not depend on it. */
void orc_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }
