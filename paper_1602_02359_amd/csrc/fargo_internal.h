// Internal definitions of libfargo: mesh description (passed by value as a
// kernel argument), device-side geometric accessors and launch helpers.
// gfx950 only: 64-wide wavefronts; the state is FP64, or FP32 in the
// FP32-bulk mode (kernels are templates on the field type).
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
  // reciprocals (1/dxlen, 1/hy, 1/Ly, 1/ymin, 1/ymed), cot(zmin) (spherical),
  // 1/(zmed[k] - zmed[k-1]) and 1/(zmin[k+1] - zmin[k])
  const double *inv_dxlen, *inv_hy, *inv_Ly, *inv_ymin, *inv_ymed, *cotz, *inv_dzmed, *inv_dz;
};

// The tables do not change while kernels run.  Device code reads them
// through the constant address space: with a wave-uniform index that is a
// scalar load, which neither waits behind nor holds up the vector memory
// counter of the field loads and stores around it.
using cdouble = const __attribute__((address_space(4))) double;
__device__ inline double gk(const double *p, size_t i) { return ((cdouble *)p)[i]; }

struct Mesh {
  int nx, ny, nz, pitch, nyg, nzg, j0, jn, k0, kn, d3;
  int geo, eos, fargo, v0_mean, visc;
  int bc[4];
  int nring; // ny * nz active rings
  int chunk; // zones per thread of the Y and Z column sweeps (a tuning parameter)
  double dx, gamma, omega, courant, cvnr, shear_c0;
  GeoTables g;

  __host__ __device__ inline size_t idx(int i, int j, int k) const {
    return ((size_t)k * (size_t)nyg + (size_t)j) * (size_t)pitch + (size_t)i;
  }
  // 32-bit element offset (the library requires every field to have fewer
  // than 2^31 elements), which lets loads use an SGPR base plus one VGPR
  __host__ __device__ inline unsigned o32(int i, int j, int k) const {
    return ((unsigned)k * (unsigned)nyg + (unsigned)j) * (unsigned)pitch + (unsigned)i;
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
  __device__ inline double Sx(int j, int k) const { return gk(g.sxj, j) * gk(g.sxk, k); }
  __device__ inline double Sy(int j, int k) const { return gk(g.syj, j) * gk(g.syk, k); }
  __device__ inline double Sz(int j, int k) const { return gk(g.szj, j) * gk(g.szk, k); }
  __device__ inline double Vinv(int j, int k) const { return gk(g.invVj, j) / gk(g.syk, k); }
  __device__ inline double Vol(int j, int k) const { return gk(g.syk, k) / gk(g.invVj, j); }
  __device__ inline double DX(int j, int k) const { return gk(g.dxlen, (size_t)k * nyg + j); }
  __device__ inline double Lz(int j, int k) const {
    double d = gk(g.zmin, k + 1) - gk(g.zmin, k);
    return geo == FARGO_SPHERICAL ? d * gk(g.ymed, j) : d;
  }
  __device__ inline double hz(int j, int k) const {
    double d = gk(g.zmed, k) - gk(g.zmed, k - 1);
    return geo == FARGO_SPHERICAL ? d * gk(g.ymed, j) : d;
  }
  // distance of a v_phi face centre to the rotation axis
  __device__ inline double Rcyl(int j, int k) const {
    return geo == FARGO_SPHERICAL ? gk(g.ymed, j) * gk(g.sinz, k) : gk(g.ymed, j);
  }
  // X-momentum factor of Tab. "momenta": Pi_x = rho * mx(v); evaluated in
  // the precision F of the field (geometric factors rounded to F)
  template <typename F>
  __device__ inline F mx(int j, int k, F v) const {
    if (geo == FARGO_CARTESIAN) return v;
    F R = (F)Rcyl(j, k);
    return R * (v + R * (F)omega);
  }
  template <typename F>
  __device__ inline F vx_from(int j, int k, F m) const {
    if (geo == FARGO_CARTESIAN) return m;
    F R = (F)Rcyl(j, k);
    return m / R - R * (F)omega;
  }
  template <typename F>
  __device__ inline F mz(int j, F v) const { return geo == FARGO_SPHERICAL ? (F)gk(g.ymed, j) * v : v; }
};

__device__ inline int imod(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}
__device__ inline int iwrap1(int i, int n) { // i in [-n, 2n)
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// The set of transported quantities (box 12a): rho plus nq others, stored
// with element type R (double, or float for the FP32-bulk state).
template <typename R>
struct TSetT {
  R *a[T_MAX]; // indexed by T_* (NULL if absent)
  R *q[T_MAX]; // the non-density quantities, packed
  int nq;
};

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each with
// its own L2.  This maps the hardware block id to a logical one so that every
// XCD works on a contiguous range of logical blocks (a bijection of [0, G)).
__device__ inline unsigned xcd_remap(unsigned b, unsigned G) {
  unsigned q = G >> 3, r = G & 7u, x = b & 7u, l = b >> 3;
  return x * q + (x < r ? x : r) + l;
}

// Blocks along an X row: nib blocks of bs threads (a multiple of 64, <= 256).
inline void row_blocks(int nx, int &nib, int &bs) {
  nib = (nx + 255) / 256;
  int per = (nx + nib - 1) / nib;
  bs = (per + 63) / 64 * 64;
}

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
  K_SET_DT = 0, K_BC_FACES, K_BC_GHOSTS, K_CFL, K_DT_FINAL, K_SPLIT, K_SRC, K_SRC_GHOSTS, K_VISC, K_SWEEP_Y,
  K_SWEEP_Z, K_RING_X, K_VEL, K_SHIFT, K_SUMS, K_SUMS_FINAL,
  K_COUNT
};
extern const char *kernel_names[K_COUNT];

// device words used by the step
struct DevWords {
  double *dt; // the step's time step
  int *err;   // error flags: 1 non-finite state, 2 bad dt
};

// Device pointers to the state (element type R); pointers the configuration
// does not use are NULL.  The static potential is FP64 in every mode: its
// gradient is the difference of two nearly equal values, which FP32 storage
// would turn into a relative force error of eps r / dr.
template <typename R>
struct StateT {
  R *rho, *vx, *vy, *vz, *e;
  const R *cs;
  const double *pot;
  const R *nu;
};

// Each launcher is defined once for R = double and R = float.
// boundaries (boxes 2 and 9)
template <typename R>
void launch_bc(Launch &L, const Mesh &m, R *rho, R *e, R *vx, R *vy, R *vz);
// boxes 3, 6 and the split of Eq. 29 (always FP64)
void launch_set_dt(Launch &L, const DevWords &w, double dt);
// per ring: v0 and (with_cfl) the largest squared rate 1/dt^2 of Eq. cfl2 and the maximum shear rate
template <typename R>
void launch_cfl(Launch &L, const Mesh &m, const StateT<R> &s, int with_cfl, double *v0, double *ringrate,
                double *ringshear, int *err);
// dt from the ring slots (unless imposed), then N and xi of every ring
void launch_dt_final(Launch &L, const Mesh &m, const DevWords &w, const double *ringrate, const double *ringshear,
                     int use_given, const double *v0, int32_t *N, double *xi);
void launch_split(Launch &L, const Mesh &m, const double *v0, double dt, int32_t *N, double *xi);
// box 7: post-source velocities and energy into vx2, vy2, vz2, e2
template <typename R>
void launch_source(Launch &L, const Mesh &m, const StateT<R> &s, const double *dt, R *vx2, R *vy2, R *vz2, R *e2);
// box 7d: viscous stress (cylindrical 2D) from vx2, vy2 into vx3, vy3
template <typename R>
void launch_visc(Launch &L, const Mesh &m, const StateT<R> &s, const R *vx2, const R *vy2, R *vx3, R *vy3,
                 const double *dt);
// box 12
template <typename R>
void launch_sweep_y(Launch &L, const Mesh &m, const StateT<R> &s, const TSetT<R> &out, const double *dt);
template <typename R>
void launch_sweep_z(Launch &L, const Mesh &m, const R *vz, const TSetT<R> &in, const TSetT<R> &out, const double *dt);
// X sweep, FARGO and 12d along X: reads T, writes rho, v_x, e of the state and
// the Y/Z momenta into Tout (out of place, shifted)
template <typename R>
void launch_ring_x(Launch &L, const Mesh &m, const R *vx2, const TSetT<R> &T, const TSetT<R> &Tout,
                   const StateT<R> &s, const double *v0, const int32_t *N, const double *xi, const double *dt);
template <typename R>
void launch_vel(Launch &L, const Mesh &m, const StateT<R> &s, const TSetT<R> &T);
// misc
template <typename R>
void launch_shift(Launch &L, const Mesh &m, R *field, const int32_t *N);
template <typename R>
void launch_sums(Launch &L, const Mesh &m, const StateT<R> &s, double *partial, double *out);

} // namespace fargo
