// Internal definitions of libfargo: mesh description (passed by value as a
// kernel argument), device-side geometric accessors and launch helpers.
// gfx950 only: 64-wide wavefronts, FP64 state.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fargo.h"

namespace fargo {

constexpr int NGH = FARGO_NGH;
constexpr int WAVE = 64;

enum { T_RHO = 0, T_PXM, T_PXP, T_PYM, T_PYP, T_PZM, T_PZP, T_E, T_MAX };

// Device-resident geometric tables (FP64), computed on the host at init from
// Appendix A (Tab. "geom", Eqs. 70-71) and the face coordinates.
struct GeoTables {
  const double *ymin, *ymed, *zmin, *zmed, *sinz; // nyg+1, nyg, nzg+1, nzg, nzg
  const double *Ly, *hy;                           // nyg: zone width, centre distance at face j
  const double *sxj, *syj, *szj, *invVj;           // nyg, nyg+1, nyg, nyg
  const double *sxk, *syk, *szk;                   // nzg, nzg, nzg+1
  const double *dxlen;                             // nzg*nyg: azimuthal zone length
};

struct Mesh {
  int nx, ny, nz, pitch, nyg, nzg, j0, jn, k0, kn, d3;
  int geo, eos, fargo, v0_mean;
  int bc[4];
  int nring; // ny * nz active rings
  double dx, gamma, omega, courant, cvnr, shear_c0;
  GeoTables g;

  __host__ __device__ inline size_t idx(int i, int j, int k) const {
    return ((size_t)k * (size_t)nyg + (size_t)j) * (size_t)pitch + (size_t)i;
  }
  __host__ __device__ inline size_t plane() const { return (size_t)nyg * (size_t)pitch; }
  __host__ __device__ inline size_t cells() const { return (size_t)nzg * plane(); }
  __device__ inline bool yper() const { return bc[0] == FARGO_BC_PERIODIC; }
  __device__ inline bool zper() const { return bc[2] == FARGO_BC_PERIODIC; }
  // owned faces along Y/Z start here (boundary face included only if periodic)
  __device__ inline int ylo() const { return yper() ? j0 : j0 + 1; }
  __device__ inline int zlo() const { return zper() ? k0 : k0 + 1; }
  __device__ inline int jbelow(int j) const { return (yper() && j == j0) ? jn - 1 : j - 1; }
  __device__ inline int jabove(int j) const { return (yper() && j == jn - 1) ? j0 : j + 1; }
  __device__ inline int kbelow(int k) const { return (zper() && k == k0) ? kn - 1 : k - 1; }
  __device__ inline int kabove(int k) const { return (zper() && k == kn - 1) ? k0 : k + 1; }

  // Tab. "geom" products (Eqs. 70, 71); face areas are of the lower face.
  __device__ inline double Sx(int j, int k) const { return g.sxj[j] * g.sxk[k]; }
  __device__ inline double Sy(int j, int k) const { return g.syj[j] * g.syk[k]; }
  __device__ inline double Sz(int j, int k) const { return g.szj[j] * g.szk[k]; }
  __device__ inline double Vinv(int j, int k) const { return g.invVj[j] / g.syk[k]; }
  __device__ inline double Vol(int j, int k) const { return g.syk[k] / g.invVj[j]; }
  __device__ inline double DX(int j, int k) const { return g.dxlen[(size_t)k * nyg + j]; }
  __device__ inline double Lz(int j, int k) const {
    double d = g.zmin[k + 1] - g.zmin[k];
    return geo == FARGO_SPHERICAL ? d * g.ymed[j] : d;
  }
  __device__ inline double hz(int j, int k) const {
    double d = g.zmed[k] - g.zmed[k - 1];
    return geo == FARGO_SPHERICAL ? d * g.ymed[j] : d;
  }
  // distance of a v_phi face centre to the rotation axis
  __device__ inline double Rcyl(int j, int k) const {
    return geo == FARGO_SPHERICAL ? g.ymed[j] * g.sinz[k] : g.ymed[j];
  }
  // X-momentum factor of Tab. "momenta": Pi_x = rho * mx(v)
  __device__ inline double mx(int j, int k, double v) const {
    if (geo == FARGO_CARTESIAN) return v;
    double R = Rcyl(j, k);
    return R * (v + R * omega);
  }
  __device__ inline double vx_from(int j, int k, double m) const {
    if (geo == FARGO_CARTESIAN) return m;
    double R = Rcyl(j, k);
    return m / R - R * omega;
  }
  __device__ inline double mz(int j, double v) const { return geo == FARGO_SPHERICAL ? g.ymed[j] * v : v; }
};

__device__ inline int imod(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}
__device__ inline int iwrap1(int i, int n) { // i in [-n, 2n)
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// The set of transported quantities (box 12a): rho plus nq others.
struct TSet {
  double *a[T_MAX];   // indexed by T_* (NULL if absent)
  double *q[T_MAX];   // the non-density quantities, packed
  int nq;
};

// Order-preserving integer image of a non-negative double (for atomic min/max).
__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

// ------------------------------------------------------------------------
// Host-side launch API (one function per kernel family)
// ------------------------------------------------------------------------
struct Prof; // per-kernel event timing, defined in fargo_api.hip

struct Launch {
  hipStream_t s;
  Prof *prof;
};

void prof_begin(Launch &L, int kid);
void prof_end(Launch &L, int kid);

enum KernelId {
  K_SET_DT = 0, K_RESET, K_BC_FACES, K_BC_GHOSTS, K_RING_V0, K_CFL, K_DT_FINAL, K_SPLIT,
  K_SRC1, K_SRC2, K_SRC3, K_MOMENTA, K_SWEEP_Y, K_SWEEP_Z, K_RING_X, K_VEL, K_SHIFT, K_SUMS, K_SUMS_FINAL,
  K_COUNT
};
extern const char *kernel_names[K_COUNT];

// device words used by the step
struct DevWords {
  double *dt;                    // the step's time step
  unsigned long long *min_cell;  // bits of min cell dt
  unsigned long long *max_shear; // bits of max shear rate
  int *err;                      // error flags: 1 non-finite state, 2 bad dt
};

struct StateP {
  double *rho, *vx, *vy, *vz, *e;
  const double *cs, *pot;
};

// boundaries (boxes 2 and 9)
void launch_bc(Launch &L, const Mesh &m, double *rho, double *e, double *vx, double *vy, double *vz);
// box 3 / box 6
void launch_reset(Launch &L, const DevWords &w);
void launch_set_dt(Launch &L, const DevWords &w, double dt);
void launch_ring_v0(Launch &L, const Mesh &m, const double *vx, double *v0);
void launch_cfl(Launch &L, const Mesh &m, const StateP &s, const double *v0, const DevWords &w);
void launch_dt_final(Launch &L, const Mesh &m, const DevWords &w, int use_given);
// dt: device time step, or NULL to use dt_val
void launch_split(Launch &L, const Mesh &m, const double *v0, const double *dt, double dt_val, int32_t *N,
                  double *xi);
// box 7
void launch_source(Launch &L, const Mesh &m, const StateP &s, const double *dt, double *vx1, double *vy1, double *vz1);
// box 12
void launch_momenta(Launch &L, const Mesh &m, const StateP &s, const TSet &T);
void launch_sweep_y(Launch &L, const Mesh &m, const double *vy, const TSet &in, const TSet &out, const double *dt);
void launch_sweep_z(Launch &L, const Mesh &m, const double *vz, const TSet &in, const TSet &out, const double *dt);
void launch_ring_x(Launch &L, const Mesh &m, const double *vx, const TSet &T, const double *v0, const int32_t *N,
                   const double *xi, const double *dt);
void launch_vel(Launch &L, const Mesh &m, const StateP &s, const TSet &T);
// misc
void launch_shift(Launch &L, const Mesh &m, double *field, const int32_t *N);
void launch_sums(Launch &L, const Mesh &m, const StateP &s, double *partial, double *out);

} // namespace fargo
