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

// The tables do not change while kernels run.  Device code reads them
// through the constant address space: with a wave-uniform index that is a
// scalar load, which neither waits behind nor holds up the vector memory
// counter of the field loads and stores around it.
using cdouble = const __attribute__((address_space(4))) double;
__device__ inline double gk(const double *p, size_t i) { return ((cdouble *)p)[i]; }

// Device-resident geometric tables (FP64), computed on the host at init from
// Appendix A (Tab. "geom", Eqs. 70-71) and the face coordinates, in one block:
// the per-row tables (sj = nyg + 1 entries apart), the per-plane tables
// (sk = nzg + 1 entries apart), then the two per-(plane, row) tables.  A
// kernel holds one base address and three sizes in scalar registers instead
// of a pointer per table.
enum GeoRow {
  GJ_YMIN,      // face radius (nyg + 1 entries)
  GJ_YMED,      // zone centre
  GJ_LY,        // zone width
  GJ_HY,        // centre distance at face j
  GJ_SXJ,       // Tab. "geom" factors (syj: nyg + 1 entries)
  GJ_SYJ,
  GJ_SZJ,
  GJ_INVVJ,
  GJ_INV_HY,    // reciprocals
  GJ_INV_LY,
  GJ_INV_YMIN,  // nyg + 1 entries
  GJ_INV_YMED,
  GJ_N
};
enum GeoPlane {
  GK_ZMIN,      // face coordinate (nzg + 1 entries)
  GK_ZMED,
  GK_SINZ,      // sin(zmed)
  GK_SXK,       // Tab. "geom" factors (szk: nzg + 1 entries)
  GK_SYK,
  GK_SZK,
  GK_COTZ,      // cot(zmin) in spherical geometry (nzg + 1 entries)
  GK_INV_DZMED, // 1 / (zmed[k] - zmed[k-1])
  GK_INV_DZ,    // 1 / (zmin[k+1] - zmin[k])
  GK_N
};
struct GeoTables {
  const double *base;
  int sj, sk, n2; // nyg + 1, nzg + 1, nzg * nyg

  __device__ inline double tj(int t, int j) const { return gk(base, (size_t)t * sj + j); }
  __device__ inline double tk(int t, int k) const { return gk(base, (size_t)GJ_N * sj + (size_t)t * sk + k); }
  __device__ inline double t2(int t, size_t i) const {
    return gk(base, (size_t)GJ_N * sj + (size_t)GK_N * sk + (size_t)t * n2 + i);
  }
  __device__ inline double ymin(int j) const { return tj(GJ_YMIN, j); }
  __device__ inline double ymed(int j) const { return tj(GJ_YMED, j); }
  __device__ inline double Ly(int j) const { return tj(GJ_LY, j); }
  __device__ inline double hy(int j) const { return tj(GJ_HY, j); }
  __device__ inline double sxj(int j) const { return tj(GJ_SXJ, j); }
  __device__ inline double syj(int j) const { return tj(GJ_SYJ, j); }
  __device__ inline double szj(int j) const { return tj(GJ_SZJ, j); }
  __device__ inline double invVj(int j) const { return tj(GJ_INVVJ, j); }
  __device__ inline double inv_hy(int j) const { return tj(GJ_INV_HY, j); }
  __device__ inline double inv_Ly(int j) const { return tj(GJ_INV_LY, j); }
  __device__ inline double inv_ymin(int j) const { return tj(GJ_INV_YMIN, j); }
  __device__ inline double inv_ymed(int j) const { return tj(GJ_INV_YMED, j); }
  __device__ inline double zmin(int k) const { return tk(GK_ZMIN, k); }
  __device__ inline double zmed(int k) const { return tk(GK_ZMED, k); }
  __device__ inline double sinz(int k) const { return tk(GK_SINZ, k); }
  __device__ inline double sxk(int k) const { return tk(GK_SXK, k); }
  __device__ inline double syk(int k) const { return tk(GK_SYK, k); }
  __device__ inline double szk(int k) const { return tk(GK_SZK, k); }
  __device__ inline double cotz(int k) const { return tk(GK_COTZ, k); }
  __device__ inline double inv_dzmed(int k) const { return tk(GK_INV_DZMED, k); }
  __device__ inline double inv_dz(int k) const { return tk(GK_INV_DZ, k); }
  // azimuthal zone length and its reciprocal at index k * nyg + j
  __device__ inline double dxlen(size_t i) const { return t2(0, i); }
  __device__ inline double inv_dxlen(size_t i) const { return t2(1, i); }
};

// Background of the azimuthal velocity (FP32-bulk state only): per-ring FP64
// tables, [nzg][nyg] each, one after the other from Mesh::bgt.  The FP32
// arrays of v_x (and of the X momenta in transport) hold deviations from it,
// so that their rounding is relative to the deviation, not to the orbital
// speed.  ell is the X-momentum factor of Tab. "momenta" applied to the
// background (R (vb + R Omega), or vb on a Cartesian mesh).
enum BgTable {
  BG_V,   // vb: the background of v_x
  BG_VT,  // vb + R Omega: the background of the inertial azimuthal velocity
  BG_DLY, // ell(j, k) - ell(j - 1, k) (0 for j = 0)
  BG_DLZ, // ell(j, k) - ell(j, k - 1) (0 for k = 0)
  BG_KV,  // viscous edge term of the background (cylindrical 2D):
          // (vb_j - vb_{j-1}) / h_j - (vb_j / r_j + vb_{j-1} / r_{j-1}) / 2
  BG_CY,  // centrifugal term of the background on Y face j: W^2 / ymin(j),
          // W = (VT(j, k) + VT(j - 1, k)) / 2 (cylindrical and spherical)
  BG_CZ,  // on spherical Z face k: W^2 cot(zmin(k)) / ymed(j),
          // W = (VT(j, k) + VT(j, k - 1)) / 2
  BG_N
};

struct Mesh {
  int nx, ny, nz, pitch, nyg, nzg, j0, jn, k0, kn, d3;
  int geo, eos, fargo, v0_mean, visc;
  int bc[4];
  int nring; // ny * nz active rings
  int chunk; // zones per thread of the Y and Z column sweeps (a tuning parameter)
  // rings longer than CFL_RING_MAX zones: the time-step pass splits each ring
  // into cseg segments of CFL_SEG zones (1 otherwise), with per-segment slots
  int cseg;
  double *segmm; // per-segment extrema (or sums) of v_x, 2 per segment (cseg > 1)
  double dx, gamma, omega, courant, cvnr, shear_c0;
  GeoTables g;
  const double *bgt; // background tables (FP32-bulk state), NULL for FP64

  // background table t of ring (j, k), read through the constant address space
  __device__ inline double bg(int t, int j, int k) const {
    return gk(bgt, (size_t)t * (size_t)g.n2 + (size_t)k * (size_t)nyg + (size_t)j);
  }

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
  __device__ inline double Sx(int j, int k) const { return g.sxj(j) * g.sxk(k); }
  __device__ inline double Sy(int j, int k) const { return g.syj(j) * g.syk(k); }
  __device__ inline double Sz(int j, int k) const { return g.szj(j) * g.szk(k); }
  __device__ inline double Vinv(int j, int k) const { return g.invVj(j) / g.syk(k); }
  __device__ inline double Vol(int j, int k) const { return g.syk(k) / g.invVj(j); }
  __device__ inline double DX(int j, int k) const { return g.dxlen((size_t)k * nyg + j); }
  __device__ inline double Lz(int j, int k) const {
    double d = g.zmin(k + 1) - g.zmin(k);
    return geo == FARGO_SPHERICAL ? d * g.ymed(j) : d;
  }
  __device__ inline double hz(int j, int k) const {
    double d = g.zmed(k) - g.zmed(k - 1);
    return geo == FARGO_SPHERICAL ? d * g.ymed(j) : d;
  }
  // distance of a v_phi face centre to the rotation axis
  __device__ inline double Rcyl(int j, int k) const {
    return geo == FARGO_SPHERICAL ? g.ymed(j) * g.sinz(k) : g.ymed(j);
  }
  // X-momentum factor of Tab. "momenta": Pi_x = rho * mx(v); evaluated in
  // the precision F of the field (geometric factors rounded to F)
  template <typename F>
  __device__ inline F mx(int j, int k, F v) const {
    if (geo == FARGO_CARTESIAN) return v;
    F R = (F)Rcyl(j, k);
    return R * (v + R * (F)omega);
  }
  // the same factor on a deviation from the background: R v (no frame term,
  // which the background carries)
  template <typename F>
  __device__ inline F mxd(int j, int k, F v) const {
    if (geo == FARGO_CARTESIAN) return v;
    return (F)Rcyl(j, k) * v;
  }
  template <typename F>
  __device__ inline F vx_from(int j, int k, F m) const {
    if (geo == FARGO_CARTESIAN) return m;
    F R = (F)Rcyl(j, k);
    return m / R - R * (F)omega;
  }
  template <typename F>
  __device__ inline F mz(int j, F v) const { return geo == FARGO_SPHERICAL ? (F)g.ymed(j) * v : v; }
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
  K_SWEEP_Z, K_RING_X, K_VEL, K_SHIFT, K_SUMS, K_SUMS_FINAL, K_ZX,
  // learned flux correction
  K_LFC_FEATURES, K_LFC_FWD1, K_LFC_FWD2, K_LFC_FWD3, K_LFC_DRHO, K_LFC_W3, K_LFC_ADJ3, K_LFC_W2, K_LFC_ADJ2,
  K_LFC_W1, K_LFC_REDUCE, K_LFC_ADAM, K_LFC_APPLY,
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

// ------------------------------------------------------------------------
// One launch over the blocks of several meshes (a batch of disks).  Block b
// of the launch runs block tab[b].y of mesh tab[b].x with that mesh's
// arguments args[tab[b].x] (the kernel's argument block, filled on the host
// by its *_args function); tab[b].x == MANY_NONE marks a padding block, which
// exits at once.  Every mesh's blocks start at a multiple of 8 in the launch,
// so that the XCD-contiguous block order of a single launch carries over.
// The kernels are the single-mesh kernels' bodies: every zone takes the same
// arithmetic as in its own launch.
// ------------------------------------------------------------------------
constexpr unsigned MANY_NONE = 0xFFFFFFFFu;
struct ManyGrid {
  const void *args;  // device: one argument block per mesh
  const uint2 *tab;  // device: nblk entries
  unsigned nblk;
};
// the blocks and tables do not change while the kernels run: read through
// the constant address space (scalar loads), word by word
using cuint = const __attribute__((address_space(4))) unsigned;
template <typename A>
__device__ inline A many_args(const void *args, unsigned d) {
  static_assert(sizeof(A) % 4 == 0, "argument blocks are whole words");
  const cuint *p = (const cuint *)((const char *)args + (size_t)d * sizeof(A));
  A a;
  unsigned *q = reinterpret_cast<unsigned *>(&a);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(A) / 4); i++) q[i] = p[i];
  return a;
}
__device__ inline uint2 many_block(const uint2 *tab) {
  const cuint *p = (const cuint *)(tab + blockIdx.x);
  return make_uint2(p[0], p[1]);
}

// Each launcher is defined once for R = double and R = float.
// boundaries (boxes 2 and 9)
template <typename R>
void launch_bc(Launch &L, const Mesh &m, R *rho, R *e, R *vx, R *vy, R *vz);
// boxes 3, 6 and the split of Eq. 29 (always FP64)
void launch_set_dt(Launch &L, const DevWords &w, double dt);
// per ring: v0 and (with_cfl) the largest squared rate 1/dt^2 of Eq. cfl2 and the maximum shear rate
// (per segment of a ring when m.cseg > 1: ringrate and ringshear hold nring * cseg slots)
constexpr int CFL_RING_MAX = 4096; // the longest ring one workgroup of the time-step kernel holds
constexpr int CFL_SEG = 1024;      // zones of a segment of a longer ring
template <typename R>
void launch_cfl(Launch &L, const Mesh &m, const StateT<R> &s, int with_cfl, double *v0, double *ringrate,
                double *ringshear, int *err);
// dt from the ring slots (unless imposed; the ring kernel splits each ring's
// displacement itself)
void launch_dt_final(Launch &L, const Mesh &m, const DevWords &w, const double *ringrate, const double *ringshear,
                     int use_given);
void launch_split(Launch &L, const Mesh &m, const double *v0, double dt, int32_t *N, double *xi);
// box 7: post-source velocities and energy into vx2, vy2, vz2, e2
template <typename R>
void launch_source(Launch &L, const Mesh &m, const StateT<R> &s, const double *dt, R *vx2, R *vy2, R *vz2, R *e2);
// box 7d: viscous stress (cylindrical 2D) from vx2, vy2 into vx3, vy3
template <typename R>
void launch_visc(Launch &L, const Mesh &m, const StateT<R> &s, const R *vx2, const R *vy2, R *vx3, R *vy3,
                 const double *dt, R *const tau[3]);
// box 12
template <typename R>
void launch_sweep_y(Launch &L, const Mesh &m, const StateT<R> &s, const TSetT<R> &out, const double *dt);
template <typename R>
void launch_sweep_z(Launch &L, const Mesh &m, const R *vz, const TSetT<R> &in, const TSetT<R> &out, const double *dt);
// X sweep, split of Eq. 29, FARGO and 12d along X: reads T, writes rho, v_x, e
// of the state and the Y/Z momenta into Tout (out of place, shifted)
template <typename R>
void launch_ring_x(Launch &L, const Mesh &m, const R *vx2, const TSetT<R> &T, const TSetT<R> &Tout,
                   const StateT<R> &s, const double *v0, const double *dt);
// 3D: the Z sweep of the Y-swept set T fused with the X transport of
// launch_ring_x (used for the FP32-bulk state)
template <typename R>
void launch_zx(Launch &L, const Mesh &m, const R *vx2, const R *vz, const TSetT<R> &T, const TSetT<R> &Tout,
               const StateT<R> &s, const double *v0, const double *dt);
template <typename R>
void launch_vel(Launch &L, const Mesh &m, const StateT<R> &s, const TSetT<R> &T);
// misc
template <typename R>
void launch_shift(Launch &L, const Mesh &m, R *field, const int32_t *N, R *scratch);
// Device scratch of the allocation-free sums (a file-scope device array):
// per-device address lookup, done once per device at context creation with
// that device current, and the address looked up (NULL before set-up).
constexpr int SUMS_STATIC_RINGS = 1 << 17;
constexpr int SCRATCH_MAX_DEVICES = 64;
int static_scratch_setup(int dev);
double *static_scratch(int dev);
// bandwidth probe: a plain streaming copy of `bytes` (a multiple of 16)
void launch_stream_copy(hipStream_t s, const void *src, void *dst, size_t bytes, int blocks);
constexpr int STREAMS_MAX = 9; // fields of the access-pattern probe
struct StreamPtrs {
  const double *in[STREAMS_MAX];
  double *out[STREAMS_MAX];
};
void launch_streams(hipStream_t s, const StreamPtrs &p, int nin, int nout, size_t ncol, int nz, int march);
template <typename R>
void launch_sums(Launch &L, const Mesh &m, const StateT<R> &s, double *partial, double *out);

// Multi-mesh forms of the step's kernels on 2D meshes (see ManyGrid): for
// each, the size of its argument block, a host function that writes one
// mesh's block to dst and returns that mesh's block count, and the launch.
template <typename R>
size_t cfl_args_bytes();
template <typename R>
unsigned cfl_args(const Mesh &m, const StateT<R> &s, double *v0, double *ringrate, double *ringshear, int *err,
                  void *dst);
template <typename R>
void launch_cfl_many(Launch &L, const ManyGrid &g, int nxmax);
size_t dt_final_args_bytes();
unsigned dt_final_args(const Mesh &m, const DevWords &w, const double *ringrate, const double *ringshear, void *dst);
void launch_dt_final_many(Launch &L, const ManyGrid &g);
template <typename F>
size_t source_args_bytes();
template <typename F>
unsigned source_args(const Mesh &m, const StateT<F> &s, const double *dt, F *vx2, F *vy2, F *vz2, F *e2, void *dst);
template <typename F>
unsigned source_ghosts_args(const Mesh &m, const StateT<F> &s, F *vx2, F *vy2, F *vz2, F *e2, void *dst);
template <typename F>
void launch_source_many(Launch &L, const Mesh &m0, const ManyGrid &g, const ManyGrid &ghosts);
template <typename F>
size_t visc_args_bytes();
template <typename F>
unsigned visc_args(const Mesh &m, const StateT<F> &s, const F *vx2, const F *vy2, F *vx3, F *vy3, const double *dt,
                   F *const tau[3], void *dst, unsigned *nb1);
template <typename F>
void launch_visc_many(Launch &L, const ManyGrid &g1, const ManyGrid &g);
template <typename F>
size_t sweep_y_args_bytes();
template <typename F>
unsigned sweep_y_args(const Mesh &m, const StateT<F> &s, const TSetT<F> &out, const double *dt, void *dst);
template <typename F>
void launch_sweep_y_many(Launch &L, const Mesh &m0, const ManyGrid &g);
template <typename F>
size_t ring_x_args_bytes();
template <typename F>
unsigned ring_x_args(const Mesh &m, const F *vx2, const TSetT<F> &T, const TSetT<F> &Tout, const StateT<F> &s,
                     const double *v0, const double *dt, void *dst);
template <typename F>
void launch_ring_x_many(Launch &L, int nq, const ManyGrid &g);
template <typename F>
size_t vel_args_bytes();
template <typename F>
unsigned vel_args(const Mesh &m, const StateT<F> &s, const TSetT<F> &T, void *dst);
template <typename F>
void launch_vel_many(Launch &L, const ManyGrid &g);

// ------------------------------------------------------------------------
// Learned flux correction (2D cylindrical FP64 state)
// ------------------------------------------------------------------------
// FP32 master parameters: W1 [32][9*4], b1 [32], W2 [32][9*32], b2 [32],
// W3 [2][9*32], b3 [2]; weights [co][tap][ci], tap = 3 ty + tx
constexpr int LFC_OFF_W1 = 0, LFC_OFF_B1 = 1152, LFC_OFF_W2 = 1184, LFC_OFF_B2 = 10400, LFC_OFF_W3 = 10432,
              LFC_OFF_B3 = 11008, LFC_NPARAM = 11010;
struct LfcScales {
  double rho_s, u_s, r_mid, r_span;
};
// bfloat16 weight matrices of the five convolutions (forward L1-L3, adjoint
// of L3 and of L2), packed as MFMA A operands (lane-major, 16 bytes a lane)
struct LfcWeights {
  unsigned short *wp1, *wp2, *wp3, *wpa3, *wpa2; // 2048, 9216, 4608, 2048, 9216 elements
};
struct LfcBufs {
  unsigned short *f, *h1, *h2;      // activations [sample][pixel][4 | 32 | 32]
  float *o;                         // net output [sample][pixel][2]
  unsigned short *g3, *g2, *g1;     // layer gradients [sample][pixel][4 | 32 | 32]
  double *drho, *gD, *lpart, *loss; // density change, dL/d(divergence), loss partials, loss
  float *w, *mo, *ve, *grad;        // master parameters, Adam moments, gradient [LFC_NPARAM]
  float *part;                      // weight-gradient partials, one row of LFC_NPARAM per block
  LfcWeights wt;
};
// samples of one training or forward batch (at most LFC_MAXB), passed by value
constexpr int LFC_MAXB = 32;
struct LfcFeed {
  const double *rho[LFC_MAXB], *vx[LFC_MAXB], *vy[LFC_MAXB];
};
struct LfcTargets {
  const double *t[LFC_MAXB];
};
// blocks of the weight-gradient kernels for nsamp samples (rows per block
// and row chunks per strip returned through rpc, nrc)
int lfc_wblocks(int nx, int ny, int nsamp, int *rpc, int *nrc);
void lfc_forward(Launch &L, const Mesh &m, const LfcFeed &in, int nsamp, const LfcScales &sc, const LfcBufs &B);
void lfc_drho(Launch &L, const Mesh &m, int nsamp, const LfcBufs &B, double sF, const LfcTargets *tg, double sigma);
void lfc_backward(Launch &L, const Mesh &m, int nsamp, const LfcBufs &B, double sF);
void lfc_adam(Launch &L, const LfcBufs &B, float lr, float c1, float c2);
void lfc_pack(Launch &L, const LfcBufs &B);
void lfc_apply(Launch &L, const Mesh &m, const LfcBufs &B, double *rho, double guard, int *flag);
void lfc_restrict(Launch &L, const Mesh &mf, const double *rf, const double *vxf, const double *vyf, const Mesh &mc,
                  double *rc, double *vxc, double *vyc);
void lfc_target(Launch &L, const Mesh &m, const double *ref, const double *plain, double *t);

} // namespace fargo
