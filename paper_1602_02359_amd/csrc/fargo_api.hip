// Host side of the C ABI declared in include/fargo.h: parameter checks, the
// FP64 geometric tables of Appendix A, workspace layout and the sequence of
// kernels of one full update (Sect. 3, Fig. "flowchart"), instantiated for
// the FP64 state and for the FP32-bulk state.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include <type_traits>

#include "fargo_internal.h"

using namespace fargo;

namespace fargo {

const char *kernel_names[K_COUNT] = {"set_dt", "bc_faces", "bc_ghosts", "cfl",    "dt_final", "split",
                                     "source", "source_ghosts", "visc", "sweep_y", "sweep_z",  "ring_x",
                                     "vel_yz", "shift",    "sums",      "sums_final", "zx_ring",
                                     "lfc_features", "lfc_fwd_l1", "lfc_fwd_l2", "lfc_fwd_l3", "lfc_drho",
                                     "lfc_wgrad_l3", "lfc_adj_l3", "lfc_wgrad_l2", "lfc_adj_l2",
                                     "lfc_wgrad_l1", "lfc_reduce", "lfc_adam", "lfc_apply"};

struct Prof {
  bool on = false;
  struct Pending {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t cur_a = nullptr;
  double total_ms[K_COUNT] = {};
  int64_t count[K_COUNT] = {};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~Prof() {
    for (auto &p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

void prof_begin(Launch &L, int kid) {
  (void)kid;
  if (!L.prof || !L.prof->on) return;
  L.prof->cur_a = L.prof->get();
  if (L.prof->cur_a) (void)hipEventRecord(L.prof->cur_a, L.s);
}

void prof_end(Launch &L, int kid) {
  if (!L.prof || !L.prof->on || !L.prof->cur_a) return;
  hipEvent_t b = L.prof->get();
  if (!b) return;
  (void)hipEventRecord(b, L.s);
  L.prof->pending.push_back({kid, L.prof->cur_a, b});
  L.prof->cur_a = nullptr;
}

} // namespace fargo

struct fargo_ctx {
  int dev = 0;
  fargo_params p{};
  Mesh m{};
  std::vector<double> ymin, zmin;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  // carved workspace
  DevWords w{};
  double *v0 = nullptr, *ringrate = nullptr, *ringshear = nullptr;
  double *partial = nullptr, *sums_out = nullptr;
  size_t esize = 8;                                    // bytes per state element
  void *v2[4] = {nullptr, nullptr, nullptr, nullptr}; // post-source vx, vy, vz, e
  void *v3[2] = {nullptr, nullptr};                   // after box 7d: vx, vy (viscosity only)
  // transport buffers (box 12): slot t of set A / B, and the packed order of
  // the non-density quantities
  void *TA[T_MAX] = {}, *TB[T_MAX] = {};
  int tq[T_MAX] = {}, nq = 0;
  Prof prof;
};

namespace {

int check_params(const fargo_params *p) {
  if (!p) return FARGO_EINVAL;
  if (p->abi_version != FARGO_ABI_VERSION) return FARGO_EINVAL;
  if (p->nx < 1 || p->ny < 3) return FARGO_EINVAL;
  if (p->nz != 1 && p->nz < 3) return FARGO_EINVAL;
  if (p->geometry < 0 || p->geometry > 2) return FARGO_EINVAL;
  if (p->geometry == FARGO_SPHERICAL && p->nz < 3) return FARGO_EINVAL;
  if (!p->ymin || !p->zmin || !(p->xmax > p->xmin)) return FARGO_EINVAL;
  if (p->eos != FARGO_ISOTHERMAL && p->eos != FARGO_ADIABATIC) return FARGO_EINVAL;
  if (p->eos == FARGO_ADIABATIC && !(p->gamma > 1.0)) return FARGO_EINVAL;
  if (p->v0_mode != FARGO_V0_MINMAX && p->v0_mode != FARGO_V0_MEAN) return FARGO_EINVAL;
  if (!(p->courant > 0.0) || !(p->cvnr >= 0.0)) return FARGO_EINVAL;
  for (int s = 0; s < 4; s++)
    if (p->bc[s] < 0 || p->bc[s] > 3) return FARGO_EINVAL;
  if ((p->bc[0] == FARGO_BC_PERIODIC) != (p->bc[1] == FARGO_BC_PERIODIC)) return FARGO_EINVAL;
  if (p->nz > 1 && (p->bc[2] == FARGO_BC_PERIODIC) != (p->bc[3] == FARGO_BC_PERIODIC)) return FARGO_EINVAL;
  if (p->geometry != FARGO_CARTESIAN && p->bc[0] == FARGO_BC_PERIODIC) return FARGO_EINVAL;
  if (p->geometry == FARGO_SPHERICAL && p->bc[2] == FARGO_BC_PERIODIC) return FARGO_EINVAL;
  if (p->precision != FARGO_FP64 && p->precision != FARGO_FP32_BULK) return FARGO_EINVAL;
  if (p->visc != 0 && p->visc != 1) return FARGO_EINVAL;
  if (p->visc && (p->geometry != FARGO_CYLINDRICAL || p->nz != 1 || p->eos != FARGO_ISOTHERMAL))
    return FARGO_EUNSUPPORTED;
  if (p->nx > (1 << 22)) return FARGO_EUNSUPPORTED; // segments of a ring in one launch dimension
  {
    // kernels address fields with 32-bit element offsets
    size_t pitch = (size_t)(p->nx + 63) / 64 * 64 + 64;
    size_t cells = pitch * (size_t)(p->ny + 2 * NGH) * (size_t)(p->nz > 1 ? p->nz + 2 * NGH : 1);
    if (cells >= ((size_t)1 << 31)) return FARGO_EUNSUPPORTED;
  }
  int nyg = p->ny + 2 * NGH, nzg = p->nz > 1 ? p->nz + 2 * NGH : 1;
  for (int j = 0; j < nyg; j++)
    if (!(p->ymin[j + 1] > p->ymin[j]) || !std::isfinite(p->ymin[j + 1])) return FARGO_EINVAL;
  for (int k = 0; k < nzg; k++)
    if (!(p->zmin[k + 1] > p->zmin[k]) || !std::isfinite(p->zmin[k + 1])) return FARGO_EINVAL;
  if (p->geometry != FARGO_CARTESIAN && !(p->ymin[0] > 0.0)) return FARGO_EINVAL;
  if (p->geometry == FARGO_SPHERICAL && !(p->zmin[0] > 0.0 && p->zmin[nzg] < M_PI)) return FARGO_EINVAL;
  return FARGO_OK;
}

void dims(const fargo_params *p, int &pitch, int &nyg, int &nzg) {
  pitch = (p->nx + 63) / 64 * 64;
  // rows whose length is a multiple of 8 KiB of doubles would put the
  // neighbours a column sweep reads on the same memory channels: one more
  // 64-element block of padding (never read or written)
  if (pitch % 1024 == 0) pitch += 64;
  nyg = p->ny + 2 * NGH;
  nzg = p->nz > 1 ? p->nz + 2 * NGH : 1;
}

// segments per ring of the time-step pass (1: one workgroup holds the ring)
int cfl_segments(int nx) { return nx <= CFL_RING_MAX ? 1 : (nx + CFL_SEG - 1) / CFL_SEG; }

int ntransported(const fargo_params *p) { return 5 + (p->nz > 1 ? 2 : 0) + (p->eos == FARGO_ADIABATIC ? 1 : 0); }

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

size_t elem_bytes(const fargo_params *p) { return p->precision == FARGO_FP32_BULK ? 4 : 8; }

// host tables, in the order of GeoTables
struct HostGeo {
  std::vector<double> ymin, ymed, zmin, zmed, sinz, Ly, hy, sxj, syj, szj, invVj, sxk, syk, szk, dxlen;
  std::vector<double> inv_dxlen, inv_hy, inv_Ly, inv_ymin, inv_ymed, cotz, inv_dzmed, inv_dz;
};

#pragma clang fp contract(off)
void make_geo(const fargo_params *p, HostGeo &G) {
  int pitch, nyg, nzg;
  dims(p, pitch, nyg, nzg);
  double dx = (p->xmax - p->xmin) / p->nx;
  G.ymin.assign(p->ymin, p->ymin + nyg + 1);
  G.zmin.assign(p->zmin, p->zmin + nzg + 1);
  G.ymed.resize(nyg);
  G.zmed.resize(nzg);
  G.sinz.resize(nzg);
  G.Ly.resize(nyg);
  G.hy.resize(nyg);
  for (int j = 0; j < nyg; j++) {
    G.ymed[j] = 0.5 * (G.ymin[j] + G.ymin[j + 1]);
    G.Ly[j] = G.ymin[j + 1] - G.ymin[j];
  }
  for (int j = 0; j < nyg; j++) G.hy[j] = j > 0 ? G.ymed[j] - G.ymed[j - 1] : G.Ly[0];
  for (int k = 0; k < nzg; k++) {
    G.zmed[k] = 0.5 * (G.zmin[k] + G.zmin[k + 1]);
    G.sinz[k] = std::sin(G.zmed[k]);
  }
  G.sxj.resize(nyg);
  G.szj.resize(nyg);
  G.invVj.resize(nyg);
  G.syj.resize(nyg + 1);
  for (int j = 0; j <= nyg; j++) {
    double a = G.ymin[j];
    if (j < nyg) {
      double b = G.ymin[j + 1];
      if (p->geometry == FARGO_CARTESIAN) {
        G.sxj[j] = b - a;
        G.szj[j] = dx * (b - a);
        G.invVj[j] = 1.0 / (b - a);
      } else if (p->geometry == FARGO_CYLINDRICAL) {
        G.sxj[j] = b - a;
        G.szj[j] = 0.5 * dx * (b * b - a * a);
        G.invVj[j] = 2.0 / ((b * b - a * a) * dx);
      } else {
        G.sxj[j] = 0.5 * (b * b - a * a);
        G.szj[j] = 0.5 * dx * (b * b - a * a);
        G.invVj[j] = 3.0 / ((b * b * b - a * a * a) * dx);
      }
    }
    G.syj[j] = p->geometry == FARGO_CARTESIAN ? 1.0 : (p->geometry == FARGO_CYLINDRICAL ? a * dx : a * a * dx);
  }
  G.sxk.resize(nzg);
  G.syk.resize(nzg);
  G.szk.resize(nzg + 1);
  for (int k = 0; k <= nzg; k++) {
    double a = G.zmin[k];
    if (k < nzg) {
      double b = G.zmin[k + 1];
      G.sxk[k] = b - a;
      if (p->geometry == FARGO_CARTESIAN) G.syk[k] = dx * (b - a);
      else if (p->geometry == FARGO_CYLINDRICAL) G.syk[k] = b - a;
      else G.syk[k] = std::cos(a) - std::cos(b);
    }
    G.szk[k] = p->geometry == FARGO_SPHERICAL ? std::sin(a) : 1.0;
  }
  G.dxlen.resize((size_t)nzg * nyg);
  for (int k = 0; k < nzg; k++)
    for (int j = 0; j < nyg; j++) {
      double v;
      if (p->geometry == FARGO_CARTESIAN) v = dx;
      else if (p->geometry == FARGO_CYLINDRICAL) v = G.ymed[j] * dx;
      else v = G.ymed[j] * G.sinz[k] * dx;
      G.dxlen[(size_t)k * nyg + j] = v;
    }
  // reciprocals and the cotangent of the face colatitudes, so that kernels
  // multiply instead of dividing by geometric lengths
  auto inv = [](const std::vector<double> &a) {
    std::vector<double> r(a.size());
    for (size_t t = 0; t < a.size(); t++) r[t] = 1.0 / a[t];
    return r;
  };
  G.inv_dxlen = inv(G.dxlen);
  G.inv_hy = inv(G.hy);
  G.inv_Ly = inv(G.Ly);
  G.inv_ymin.resize(nyg + 1);
  for (int j = 0; j <= nyg; j++) G.inv_ymin[j] = G.ymin[j] != 0.0 ? 1.0 / G.ymin[j] : 0.0;
  G.inv_ymed = inv(G.ymed);
  G.cotz.resize(nzg + 1);
  for (int k = 0; k <= nzg; k++)
    G.cotz[k] = p->geometry == FARGO_SPHERICAL ? std::cos(G.zmin[k]) / std::sin(G.zmin[k]) : 0.0;
  G.inv_dzmed.resize(nzg);
  G.inv_dz.resize(nzg);
  for (int k = 0; k < nzg; k++) {
    G.inv_dzmed[k] = 1.0 / (k > 0 ? G.zmed[k] - G.zmed[k - 1] : G.zmin[1] - G.zmin[0]);
    G.inv_dz[k] = 1.0 / (G.zmin[k + 1] - G.zmin[k]);
  }
}

// the block of GeoTables: GJ_N row tables of nyg + 1 entries, GK_N plane
// tables of nzg + 1 entries, dxlen and its reciprocal (nzg * nyg each)
size_t geo_doubles(int nyg, int nzg) {
  return (size_t)GJ_N * (nyg + 1) + (size_t)GK_N * (nzg + 1) + 2 * (size_t)nzg * nyg;
}

struct Layout {
  size_t geo, words, v0, ringrate, ringshear, segmm, partial, sums, bg, v2, T, total;
};

Layout layout(const fargo_params *p) {
  int pitch, nyg, nzg;
  dims(p, pitch, nyg, nzg);
  size_t nc = (size_t)pitch * nyg * nzg;
  size_t nring = (size_t)p->ny * p->nz;
  size_t eb = elem_bytes(p);
  Layout L{};
  size_t o = 0;
  L.geo = o;
  o += al(geo_doubles(nyg, nzg) * 8);
  L.words = o;
  o += 256;
  L.v0 = o;
  o += al(nring * 8);
  const size_t cseg = (size_t)cfl_segments(p->nx);
  L.ringrate = o;
  o += al(nring * cseg * 8);
  L.ringshear = o;
  o += al(nring * cseg * 8);
  L.segmm = o;
  if (cseg > 1) o += al(nring * cseg * 2 * 8);
  L.partial = o;
  o += al(nring * 10 * 8);
  L.sums = o;
  o += 256;
  L.bg = o; // background tables of v_x (FP32-bulk state only)
  if (p->precision == FARGO_FP32_BULK) o += al((size_t)BG_N * nyg * nzg * 8);
  L.v2 = o;
  o += al(nc * eb) * ((p->nz > 1 ? 3 : 2) + (p->eos == FARGO_ADIABATIC ? 1 : 0) + (p->visc ? 2 : 0));
  L.T = o;
  o += al(nc * eb) * 2 * ntransported(p);
  L.total = o;
  return L;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? FARGO_OK : FARGO_EHIP; }

// Pointers the configuration does not use are dropped, so that no kernel
// touches a field (or a transport buffer) that does not exist.
template <typename F>
StateT<F> state_of(const fargo_ctx *c, const fargo_state *s) {
  StateT<F> S;
  S.rho = (F *)s->rho;
  S.vx = (F *)s->vx;
  S.vy = (F *)s->vy;
  S.vz = c->m.d3 ? (F *)s->vz : nullptr;
  S.e = c->p.eos == FARGO_ADIABATIC ? (F *)s->e : nullptr;
  S.cs = c->p.eos == FARGO_ISOTHERMAL ? (const F *)s->cs : nullptr;
  S.pot = (const double *)s->pot;
  S.nu = c->p.visc ? (const F *)s->nu : nullptr;
  return S;
}

template <typename F>
TSetT<F> tset(const fargo_ctx *c, void *const *slots) {
  TSetT<F> T{};
  for (int t = 0; t < T_MAX; t++) T.a[t] = (F *)slots[t];
  for (int q = 0; q < c->nq; q++) T.q[q] = (F *)slots[c->tq[q]];
  T.nq = c->nq;
  return T;
}

bool fp32(const fargo_ctx *c) { return c->p.precision == FARGO_FP32_BULK; }

int check_state(const fargo_ctx *c, const fargo_state *s) {
  if (!s || !s->rho || !s->vx || !s->vy || !s->pot) return FARGO_EINVAL;
  if (c->m.d3 && !s->vz) return FARGO_EINVAL;
  if (c->p.eos == FARGO_ISOTHERMAL && !s->cs) return FARGO_EINVAL;
  if (c->p.eos == FARGO_ADIABATIC && !s->e) return FARGO_EINVAL;
  if (c->p.visc && !s->nu) return FARGO_EINVAL;
  return FARGO_OK;
}

// The background tables of an FP32-bulk context (enum BgTable) for the
// per-ring background vb [nzg][nyg], formed on the host in FP64 and copied
// to the device.
int upload_background(fargo_ctx *ctx, const double *vb) {
  const Mesh &m = ctx->m;
  const int nyg = m.nyg, nzg = m.nzg;
  const size_t n2 = (size_t)nyg * nzg;
  HostGeo G;
  make_geo(&ctx->p, G);
  const bool cart = ctx->p.geometry == FARGO_CARTESIAN, sph = ctx->p.geometry == FARGO_SPHERICAL;
  std::vector<double> tab((size_t)BG_N * n2, 0.0), ell(n2);
  for (int k = 0; k < nzg; k++)
    for (int j = 0; j < nyg; j++) {
      const size_t r = (size_t)k * nyg + j;
      const double R = cart ? 1.0 : (sph ? G.ymed[j] * G.sinz[k] : G.ymed[j]);
      const double Rw = cart ? 0.0 : R * ctx->p.omega;
      tab[BG_V * n2 + r] = vb[r];
      tab[BG_VT * n2 + r] = vb[r] + Rw;
      ell[r] = cart ? vb[r] : R * (vb[r] + Rw);
    }
  for (int k = 0; k < nzg; k++)
    for (int j = 0; j < nyg; j++) {
      const size_t r = (size_t)k * nyg + j;
      if (j > 0) {
        tab[BG_DLY * n2 + r] = ell[r] - ell[r - 1];
        tab[BG_KV * n2 + r] =
            (vb[r] - vb[r - 1]) / G.hy[j] - 0.5 * (vb[r] / G.ymed[j] + vb[r - 1] / G.ymed[j - 1]);
      }
      if (k > 0) tab[BG_DLZ * n2 + r] = ell[r] - ell[r - nyg];
      if (!cart && j > 0) {
        const double W = 0.5 * (tab[BG_VT * n2 + r] + tab[BG_VT * n2 + r - 1]);
        tab[BG_CY * n2 + r] = W * W * G.inv_ymin[j];
      }
      if (sph && k > 0) {
        const double W = 0.5 * (tab[BG_VT * n2 + r] + tab[BG_VT * n2 + r - nyg]);
        tab[BG_CZ * n2 + r] = W * W * G.cotz[k] * (1.0 / G.ymed[j]);
      }
    }
  return hip_ok(hipMemcpy((void *)m.bgt, tab.data(), tab.size() * 8, hipMemcpyHostToDevice));
}

// boxes 2, 3, 4, 6 and the split of Eq. 29 (dt > 0: imposed)
template <typename F>
void timestep_phase(fargo_ctx *c, Launch &L, const StateT<F> &S, double dt) {
  const Mesh &m = c->m;
  if (dt > 0.0) launch_set_dt(L, c->w, dt);
  launch_bc(L, m, S.rho, S.e, S.vx, S.vy, S.vz);
  launch_cfl(L, m, S, 1, c->v0, c->ringrate, c->ringshear, c->w.err);
  launch_dt_final(L, m, c->w, c->ringrate, c->ringshear, dt > 0.0);
}

} // namespace

extern "C" {

int fargo_abi_version(void) { return FARGO_ABI_VERSION; }

const char *fargo_strerror(int status) {
  switch (status) {
  case FARGO_OK: return "ok";
  case FARGO_EINVAL: return "invalid argument";
  case FARGO_ENOMEM: return "out of memory or workspace too small";
  case FARGO_EHIP: return "HIP runtime error";
  case FARGO_ENONFINITE: return "non-finite or non-positive state";
  case FARGO_ECFL: return "invalid time step";
  case FARGO_EUNSUPPORTED: return "unsupported configuration";
  default: return "unknown status";
  }
}

int fargo_layout(const fargo_params *params, int32_t *pitch, int32_t *ny_g, int32_t *nz_g) {
  int rc = check_params(params);
  if (rc) return rc;
  int a, b, c;
  dims(params, a, b, c);
  if (pitch) *pitch = a;
  if (ny_g) *ny_g = b;
  if (nz_g) *nz_g = c;
  return FARGO_OK;
}

int fargo_workspace_bytes(const fargo_params *params, size_t *bytes) {
  int rc = check_params(params);
  if (rc) return rc;
  if (!bytes) return FARGO_EINVAL;
  *bytes = layout(params).total;
  return FARGO_OK;
}

int fargo_init(const fargo_params *params, void *workspace, size_t ws_bytes, fargo_ctx **out) {
  if (!out) return FARGO_EINVAL;
  int rc = check_params(params);
  if (rc) return rc;
  fargo_ctx *c = new (std::nothrow) fargo_ctx();
  if (!c) return FARGO_ENOMEM;
  if (hipGetDevice(&c->dev) != hipSuccess) {
    delete c;
    return FARGO_EHIP;
  }
  // the device copy of the static scratch of fargo_conserved_sums_noalloc
  // (looked up once per device, with that device current)
  if (static_scratch_setup(c->dev) != FARGO_OK) {
    delete c;
    return FARGO_EHIP;
  }
  c->p = *params;
  int pitch, nyg, nzg;
  dims(params, pitch, nyg, nzg);
  c->ymin.assign(params->ymin, params->ymin + nyg + 1);
  c->zmin.assign(params->zmin, params->zmin + nzg + 1);
  c->p.ymin = c->ymin.data();
  c->p.zmin = c->zmin.data();
  Layout Lo = layout(params);
  if (workspace) {
    if (ws_bytes < Lo.total || ((uintptr_t)workspace & 255)) {
      delete c;
      return ws_bytes < Lo.total ? FARGO_ENOMEM : FARGO_EINVAL;
    }
    c->ws = workspace;
  } else {
    if (hipMalloc(&c->ws, Lo.total) != hipSuccess) {
      delete c;
      return FARGO_ENOMEM;
    }
    c->own_ws = true;
  }
  c->ws_bytes = Lo.total;
  char *base = (char *)c->ws;
  // geometry
  HostGeo G;
  make_geo(&c->p, G);
  // one block in the order of GeoRow, GeoPlane, then dxlen, 1/dxlen; each
  // row (plane) table padded to nyg + 1 (nzg + 1) entries
  std::vector<double> buf;
  buf.reserve(geo_doubles(nyg, nzg));
  const std::vector<double> *rows[GJ_N] = {&G.ymin, &G.ymed,  &G.Ly,     &G.hy,     &G.sxj,      &G.syj,
                                          &G.szj,  &G.invVj, &G.inv_hy, &G.inv_Ly, &G.inv_ymin, &G.inv_ymed};
  const std::vector<double> *planes[GK_N] = {&G.zmin, &G.zmed, &G.sinz, &G.sxk,      &G.syk,
                                            &G.szk,  &G.cotz, &G.inv_dzmed, &G.inv_dz};
  for (const std::vector<double> *v : rows) {
    buf.insert(buf.end(), v->begin(), v->end());
    buf.resize(buf.size() + (nyg + 1) - v->size(), 0.0);
  }
  for (const std::vector<double> *v : planes) {
    buf.insert(buf.end(), v->begin(), v->end());
    buf.resize(buf.size() + (nzg + 1) - v->size(), 0.0);
  }
  buf.insert(buf.end(), G.dxlen.begin(), G.dxlen.end());
  buf.insert(buf.end(), G.inv_dxlen.begin(), G.inv_dxlen.end());
  double *gd = (double *)(base + Lo.geo);
  if (buf.size() != geo_doubles(nyg, nzg)) { // the workspace slot is sized by geo_doubles
    fargo_destroy(c);
    return FARGO_EINVAL;
  }
  if (hipMemcpy(gd, buf.data(), buf.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    fargo_destroy(c);
    return FARGO_EHIP;
  }
  Mesh &m = c->m;
  m.nx = params->nx;
  m.ny = params->ny;
  m.nz = params->nz;
  m.pitch = pitch;
  m.nyg = nyg;
  m.nzg = nzg;
  m.j0 = NGH;
  m.jn = NGH + params->ny;
  m.d3 = params->nz > 1;
  m.k0 = m.d3 ? NGH : 0;
  m.kn = m.d3 ? NGH + params->nz : 1;
  m.geo = params->geometry;
  m.eos = params->eos;
  m.fargo = params->fargo ? 1 : 0;
  m.v0_mean = params->v0_mode == FARGO_V0_MEAN;
  m.visc = params->visc;
  for (int s = 0; s < 4; s++) m.bc[s] = params->bc[s];
  m.nring = params->ny * params->nz;
  m.chunk = 64;
  m.cseg = cfl_segments(params->nx);
  m.segmm = m.cseg > 1 ? (double *)(base + Lo.segmm) : nullptr;
  m.dx = (params->xmax - params->xmin) / params->nx;
  m.gamma = params->gamma;
  m.omega = params->omega;
  m.courant = params->courant;
  m.cvnr = params->cvnr;
  m.shear_c0 = params->shear_c0;
  m.g.base = gd;
  m.g.sj = nyg + 1;
  m.g.sk = nzg + 1;
  m.g.n2 = nzg * nyg;
  // words and per-ring arrays
  char *wd = base + Lo.words;
  c->w.dt = (double *)wd;
  c->w.err = (int *)(wd + 8);
  if (hipMemset(wd, 0, 256) != hipSuccess) {
    fargo_destroy(c);
    return FARGO_EHIP;
  }
  m.bgt = nullptr;
  if (params->precision == FARGO_FP32_BULK) { // zero background until set
    m.bgt = (const double *)(base + Lo.bg);
    std::vector<double> zero((size_t)nyg * nzg, 0.0);
    if (upload_background(c, zero.data()) != FARGO_OK) {
      fargo_destroy(c);
      return FARGO_EHIP;
    }
  }
  c->v0 = (double *)(base + Lo.v0);
  c->ringrate = (double *)(base + Lo.ringrate);
  c->ringshear = (double *)(base + Lo.ringshear);
  c->partial = (double *)(base + Lo.partial);
  c->sums_out = (double *)(base + Lo.sums);
  size_t nc = (size_t)pitch * nyg * nzg;
  c->esize = elem_bytes(params);
  size_t fb = al(nc * c->esize);
  {
    size_t o = Lo.v2;
    for (int d = 0; d < 4; d++) {
      bool need = d < 2 || (d == 2 && m.d3) || (d == 3 && params->eos == FARGO_ADIABATIC);
      if (!need) continue;
      c->v2[d] = base + o;
      o += fb;
    }
    if (params->visc) {
      c->v3[0] = base + o;
      c->v3[1] = base + o + fb;
    }
  }
  int nT = ntransported(params);
  int slot = 0;
  for (int t = 0; t < T_MAX; t++) {
    bool need = t <= T_PYP || (m.d3 && (t == T_PZM || t == T_PZP)) || (t == T_E && params->eos == FARGO_ADIABATIC);
    c->TA[t] = c->TB[t] = nullptr;
    if (!need) continue;
    c->TA[t] = base + Lo.T + (size_t)slot * fb;
    c->TB[t] = base + Lo.T + (size_t)(nT + slot) * fb;
    slot++;
    if (t != T_RHO) c->tq[c->nq++] = t;
  }
  *out = c;
  return FARGO_OK;
}

int fargo_set_vx_background(fargo_ctx *ctx, const double *vb) {
  if (!ctx || !vb) return FARGO_EINVAL;
  if (ctx->p.precision != FARGO_FP32_BULK) return FARGO_EINVAL;
  const size_t n2 = (size_t)ctx->m.nyg * ctx->m.nzg;
  for (size_t t = 0; t < n2; t++)
    if (!std::isfinite(vb[t])) return FARGO_EINVAL;
  return upload_background(ctx, vb);
}

void fargo_destroy(fargo_ctx *ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
  delete ctx;
}

int fargo_cfl_dt(fargo_ctx *ctx, fargo_state *state, double *dt_host, void *stream) {
  if (!ctx) return FARGO_EINVAL;
  int rc = check_state(ctx, state);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Launch L{s, &ctx->prof};
  if (fp32(ctx)) timestep_phase(ctx, L, state_of<float>(ctx, state), 0.0);
  else timestep_phase(ctx, L, state_of<double>(ctx, state), 0.0);
  if (hipGetLastError() != hipSuccess) return FARGO_EHIP;
  if (!dt_host) return FARGO_OK;
  double dt = 0.0;
  int err = 0;
  if (hipMemcpyAsync(&dt, ctx->w.dt, 8, hipMemcpyDeviceToHost, s) != hipSuccess) return FARGO_EHIP;
  if (hipMemcpyAsync(&err, ctx->w.err, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return FARGO_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return FARGO_EHIP;
  *dt_host = dt;
  if (err & 1) return FARGO_ENONFINITE;
  if (err & 2) return FARGO_ECFL;
  return FARGO_OK;
}

} // extern "C"

namespace {

// One full update (Sect. 3, Fig. "flowchart") on a state of element type F.
template <typename F>
void step_impl(fargo_ctx *ctx, const fargo_state *state, double dt, Launch &L) {
  const Mesh &m = ctx->m;
  StateT<F> S = state_of<F>(ctx, state);
  timestep_phase(ctx, L, S, dt > 0.0 ? dt : 0.0);                                  // boxes 2, 3, 4, 6
  const double *dtp = ctx->w.dt;
  F *v2[4] = {(F *)ctx->v2[0], (F *)ctx->v2[1], (F *)ctx->v2[2], (F *)ctx->v2[3]};
  launch_source(L, m, S, dtp, v2[0], v2[1], v2[2], v2[3]);                        // boxes 7a-7c
  StateT<F> P = S; // post-source fields: density of the state, v'' and e''
  P.vx = v2[0];
  P.vy = v2[1];
  if (m.visc) {                                                                    // box 7d
    // the stress components in transport set A, which holds nothing until the X sweep
    F *const tau[3] = {(F *)ctx->TA[T_RHO], (F *)ctx->TA[T_PXM], (F *)ctx->TA[T_PXP]};
    launch_visc(L, m, S, v2[0], v2[1], (F *)ctx->v3[0], (F *)ctx->v3[1], dtp, tau);
    P.vx = (F *)ctx->v3[0];
    P.vy = (F *)ctx->v3[1];
  }
  P.vz = v2[2];
  P.e = v2[3];
  launch_bc(L, m, P.rho, P.e, P.vx, P.vy, P.vz);                                   // box 9
  const TSetT<F> TA = tset<F>(ctx, ctx->TA), TB = tset<F>(ctx, ctx->TB);
  launch_sweep_y(L, m, P, TB, dtp);                                                // boxes 12a-c, Y
  const TSetT<F> *cur = &TB, *other = &TA;
  if constexpr (std::is_same<F, float>::value) {
    if (m.d3) { // FP32: Z, X, split, FARGO and 12d (v_x) in one pass
      launch_zx(L, m, (const F *)P.vx, (const F *)P.vz, TB, TA, S, ctx->v0, dtp);
      launch_vel(L, m, S, TA);                                                     // 12d (v_y, v_z)
      return;
    }
  }
  if (m.d3) {
    launch_sweep_z(L, m, (const F *)P.vz, TB, TA, dtp);                            // Z
    cur = &TA;
    other = &TB;
  }
  launch_ring_x(L, m, (const F *)P.vx, *cur, *other, S, ctx->v0, dtp);           // X, split, FARGO, 12d (v_x)
  launch_vel(L, m, S, *other);                                                     // 12d (v_y, v_z)
}

} // namespace

extern "C" {

int fargo_step(fargo_ctx *ctx, fargo_state *state, double dt, void *stream) {
  if (!ctx) return FARGO_EINVAL;
  int rc = check_state(ctx, state);
  if (rc) return rc;
  if (!(dt <= 0.0) && !std::isfinite(dt)) return FARGO_EINVAL;
  Launch L{(hipStream_t)stream, &ctx->prof};
  if (fp32(ctx)) step_impl<float>(ctx, state, dt, L);
  else step_impl<double>(ctx, state, dt, L);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_shift(fargo_ctx *ctx, void *field, const int32_t *nshift, void *stream) {
  if (!ctx || !field || !nshift) return FARGO_EINVAL;
  Launch L{(hipStream_t)stream, &ctx->prof};
  // a ring staged in LDS, or (longer rings) out of place through a transport
  // buffer of the workspace, which holds nothing between steps
  if (fp32(ctx)) launch_shift(L, ctx->m, (float *)field, nshift, (float *)ctx->TA[T_RHO]);
  else launch_shift(L, ctx->m, (double *)field, nshift, (double *)ctx->TA[T_RHO]);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_ring_split(fargo_ctx *ctx, const void *vx, double dt, double *v0, int32_t *nshift, double *xi,
                     void *stream) {
  if (!ctx || !vx || !v0 || !nshift || !xi || !(dt > 0.0) || !std::isfinite(dt)) return FARGO_EINVAL;
  Launch L{(hipStream_t)stream, &ctx->prof};
  if (fp32(ctx)) {
    StateT<float> S{};
    S.vx = (float *)const_cast<void *>(vx);
    launch_cfl(L, ctx->m, S, 0, v0, nullptr, nullptr, nullptr);
  } else {
    StateT<double> S{};
    S.vx = (double *)const_cast<void *>(vx);
    launch_cfl(L, ctx->m, S, 0, v0, nullptr, nullptr, nullptr);
  }
  launch_split(L, ctx->m, v0, dt, nshift, xi);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_conserved_sums(fargo_ctx *ctx, const fargo_state *state, double out[5], void *stream) {
  if (!ctx || !out) return FARGO_EINVAL;
  int rc = check_state(ctx, state);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Launch L{s, &ctx->prof};
  if (fp32(ctx)) launch_sums(L, ctx->m, state_of<float>(ctx, state), ctx->partial, ctx->sums_out);
  else launch_sums(L, ctx->m, state_of<double>(ctx, state), ctx->partial, ctx->sums_out);
  if (hipGetLastError() != hipSuccess) return FARGO_EHIP;
  if (hipMemcpyAsync(out, ctx->sums_out, 5 * 8, hipMemcpyDeviceToHost, s) != hipSuccess) return FARGO_EHIP;
  return hip_ok(hipStreamSynchronize(s));
}

int fargo_conserved_sums_noalloc(fargo_ctx *ctx, const fargo_state *state, double out[5], void *stream) {
  if (!ctx || !out) return FARGO_EINVAL;
  int rc = check_state(ctx, state);
  if (rc) return rc;
  if (ctx->m.nring > SUMS_STATIC_RINGS) return FARGO_ENOMEM;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return FARGO_EHIP;
  if (cur != ctx->dev) return FARGO_EINVAL;
  double *scr = static_scratch(cur); // device address of this device's copy
  if (!scr) return FARGO_EHIP;
  double *partial = scr, *res = scr + (size_t)SUMS_STATIC_RINGS * 10;
  hipStream_t s = (hipStream_t)stream;
  Launch L{s, &ctx->prof};
  if (fp32(ctx)) launch_sums(L, ctx->m, state_of<float>(ctx, state), partial, res);
  else launch_sums(L, ctx->m, state_of<double>(ctx, state), partial, res);
  if (hipGetLastError() != hipSuccess) return FARGO_EHIP;
  if (hipMemcpyAsync(out, res, 5 * 8, hipMemcpyDeviceToHost, s) != hipSuccess) return FARGO_EHIP;
  return hip_ok(hipStreamSynchronize(s));
}

int fargo_hbm_copy(const void *src, void *dst, size_t bytes, int blocks, void *stream) {
  if (!src || !dst || bytes == 0 || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
    return FARGO_EINVAL;
  if (blocks < 0 || blocks > (1 << 20) || bytes / 16 / 256 >= ((size_t)1 << 31)) return FARGO_EINVAL;
  const char *a = (const char *)src, *b = (const char *)dst;
  if (a < b + bytes && b < a + bytes) return FARGO_EINVAL; // overlapping ranges
  launch_stream_copy((hipStream_t)stream, src, dst, bytes, blocks);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_hbm_streams(const double *const *in, int nin, double *const *out, int nout, int nx, int ny, int nz,
                      int march, void *stream) {
  if (!in || !out || nin < 1 || nin > STREAMS_MAX || nout < 1 || nout > nin || nx < 1 || ny < 1 || nz < 1 ||
      (march != 0 && march != 1))
    return FARGO_EINVAL;
  const size_t ncol = (size_t)nx * (size_t)ny, n = ncol * (size_t)nz;
  if ((march ? ncol : n) / 256 >= ((size_t)1 << 31)) return FARGO_EINVAL;
  StreamPtrs p{};
  for (int q = 0; q < nin; q++) {
    if (!in[q] || ((uintptr_t)in[q] & 7)) return FARGO_EINVAL;
    p.in[q] = in[q];
  }
  for (int q = 0; q < nout; q++) {
    if (!out[q] || ((uintptr_t)out[q] & 7)) return FARGO_EINVAL;
    p.out[q] = out[q];
  }
  // no output may overlap another output or any input
  auto overlap = [&](const void *a, const void *b) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + n * 8 && y < x + n * 8;
  };
  for (int q = 0; q < nout; q++) {
    for (int r = 0; r < nin; r++)
      if (overlap(p.out[q], p.in[r])) return FARGO_EINVAL;
    for (int r = 0; r < q; r++)
      if (overlap(p.out[q], p.out[r])) return FARGO_EINVAL;
  }
  launch_streams((hipStream_t)stream, p, nin, nout, ncol, nz, march);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_get_dt(fargo_ctx *ctx, double *dt_host, void *stream) {
  if (!ctx || !dt_host) return FARGO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(dt_host, ctx->w.dt, 8, hipMemcpyDeviceToHost, s) != hipSuccess) return FARGO_EHIP;
  return hip_ok(hipStreamSynchronize(s));
}

int fargo_check(fargo_ctx *ctx) {
  if (!ctx) return FARGO_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return FARGO_EHIP;
  int err = 0;
  if (hipMemcpy(&err, ctx->w.err, 4, hipMemcpyDeviceToHost) != hipSuccess) return FARGO_EHIP;
  int zero = 0;
  if (hipMemcpy(ctx->w.err, &zero, 4, hipMemcpyHostToDevice) != hipSuccess) return FARGO_EHIP;
  if (err & 1) return FARGO_ENONFINITE;
  if (err & 2) return FARGO_ECFL;
  return FARGO_OK;
}

int fargo_profile_enable(fargo_ctx *ctx, int on) {
  if (!ctx) return FARGO_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return FARGO_EHIP;
  Prof &P = ctx->prof;
  for (auto &pd : P.pending) {
    P.pool.push_back(pd.a);
    P.pool.push_back(pd.b);
  }
  P.pending.clear();
  for (int k = 0; k < K_COUNT; k++) {
    P.total_ms[k] = 0.0;
    P.count[k] = 0;
  }
  P.on = on != 0;
  return FARGO_OK;
}

int fargo_timings(fargo_ctx *ctx, const char **names, int64_t *counts, double *total_ms, int cap, int *n_out,
                  void *stream) {
  if (!ctx) return FARGO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipStreamSynchronize(s) != hipSuccess) return FARGO_EHIP;
  Prof &P = ctx->prof;
  for (auto &pd : P.pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
      P.total_ms[pd.kid] += ms;
      P.count[pd.kid] += 1;
    }
    P.pool.push_back(pd.a);
    P.pool.push_back(pd.b);
  }
  P.pending.clear();
  int n = 0;
  for (int k = 0; k < K_COUNT && n < cap; k++) {
    if (names) names[n] = kernel_names[k];
    if (counts) counts[n] = P.count[k];
    if (total_ms) total_ms[n] = P.total_ms[k];
    n++;
  }
  if (n_out) *n_out = n;
  return FARGO_OK;
}

} // extern "C"

// ------------------------------------------------------------------------
// Batches of independent contexts (many disks of uneven sizes): one step of
// every context is captured once into a hipGraph, the disks spread over
// `lanes` capture streams that fork from and join into one origin stream, and
// replayed with a single graph launch per step.  Each context keeps its own
// device time step (box 6), so nothing synchronises the host.
// ------------------------------------------------------------------------
//
// Fused mode (lanes == 0): each kernel of the step runs once for all disks,
// its blocks mapped to (disk, block) through a table (ManyGrid), so that a
// step is seven or eight launches whatever the number of disks, captured into
// one graph.  Every zone takes the arithmetic of its disk's own step, so the
// results are those of fargo_step disk by disk, bit for bit.  It takes 2D
// meshes of one configuration (precision, geometry, equation of state,
// viscosity, orbital advection, v0 mode, boundary kinds) with FIXED radial
// sides (boxes 2 and 9 then launch nothing) and rings of at most 1792 zones.
struct fargo_batch {
  std::vector<fargo_ctx *> ctx;
  std::vector<fargo_state> st;
  int lanes = 1; // 0: fused
  hipStream_t origin = nullptr;
  std::vector<hipStream_t> ls;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // fused mode: the launches' argument blocks and tables in one allocation
  void *fmem = nullptr;
  ManyGrid g[9] = {};
  ManyGrid gcfl[8] = {}; // the time-step pass by zones per thread (ceil(nx / 256), 1..7)
  int nxmax = 0;
  std::vector<int> chunk; // per disk (the sweep's chunk length, tuned per size class)
};

namespace {

void batch_release_graph(fargo_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  for (hipStream_t s : b->ls) (void)hipStreamDestroy(s);
  b->ls.clear();
}

// capture one step of every context; lanes streams of default priority
int batch_capture(fargo_batch *b, int lanes) {
  batch_release_graph(b);
  b->lanes = lanes;
  for (int l = 0; l < lanes; l++) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return FARGO_EHIP;
    b->ls.push_back(s);
  }
  std::vector<bool> prof_on(b->ctx.size());
  for (size_t d = 0; d < b->ctx.size(); d++) { // no event records inside the graph
    prof_on[d] = b->ctx[d]->prof.on;
    b->ctx[d]->prof.on = false;
  }
  int rc = FARGO_OK;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join(lanes, nullptr);
  if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) rc = FARGO_EHIP;
  for (int l = 0; l < lanes && !rc; l++)
    if (hipEventCreateWithFlags(&join[l], hipEventDisableTiming) != hipSuccess) rc = FARGO_EHIP;
  bool capturing = false;
  if (!rc && hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = FARGO_EHIP;
  else if (!rc) capturing = true;
  if (!rc && hipEventRecord(fork, b->origin) != hipSuccess) rc = FARGO_EHIP;
  for (int l = 0; l < lanes && !rc; l++)
    if (hipStreamWaitEvent(b->ls[l], fork, 0) != hipSuccess) rc = FARGO_EHIP;
  for (size_t d = 0; d < b->ctx.size() && !rc; d++)
    rc = fargo_step(b->ctx[d], &b->st[d], 0.0, (void *)b->ls[d % lanes]);
  for (int l = 0; l < lanes && !rc; l++) {
    if (hipEventRecord(join[l], b->ls[l]) != hipSuccess) rc = FARGO_EHIP;
    else if (hipStreamWaitEvent(b->origin, join[l], 0) != hipSuccess) rc = FARGO_EHIP;
  }
  if (capturing) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->origin, &g);
    if (!rc && e != hipSuccess) rc = FARGO_EHIP;
    if (!rc) {
      b->graph = g;
      if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) rc = FARGO_EHIP;
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  if (fork) (void)hipEventDestroy(fork);
  for (hipEvent_t e : join)
    if (e) (void)hipEventDestroy(e);
  for (size_t d = 0; d < b->ctx.size(); d++) b->ctx[d]->prof.on = prof_on[d];
  (void)hipGetLastError();
  return rc;
}

size_t field_bytes(const fargo_ctx *c) { return (size_t)c->m.pitch * c->m.nyg * c->m.nzg * c->esize; }

// ---- fused mode ----
enum { FU_CFL, FU_DT, FU_SRC, FU_SRCG, FU_VISC1, FU_VISC, FU_SY, FU_RX, FU_VEL, FU_N };

bool fused_ok(fargo_ctx *const *c, int n) {
  const fargo_params &p0 = c[0]->p;
  for (int d = 0; d < n; d++) {
    const fargo_params &p = c[d]->p;
    const Mesh &m = c[d]->m;
    if (m.d3 || p.precision != p0.precision || p.geometry != p0.geometry || p.eos != p0.eos ||
        p.visc != p0.visc || p.fargo != p0.fargo || p.v0_mode != p0.v0_mode)
      return false;
    for (int k = 0; k < 4; k++)
      if (p.bc[k] != p0.bc[k]) return false;
    if (p.bc[0] != FARGO_BC_FIXED || p.bc[1] != FARGO_BC_FIXED) return false;
    if (m.cseg != 1 || m.nx > 1792) return false;
  }
  return true;
}

// argument blocks and block table of one launch over all disks
struct ManyHost {
  size_t asz = 0;
  std::vector<char> args;
  std::vector<uint2> tab;
  void *slot(size_t d) {
    if (args.size() < (d + 1) * asz) args.resize((d + 1) * asz);
    return args.data() + d * asz;
  }
  void blocks(unsigned d, unsigned nb) {
    while (tab.size() % 8) tab.push_back(make_uint2(MANY_NONE, 0u)); // each disk from a multiple of 8
    for (unsigned b = 0; b < nb; b++) tab.push_back(make_uint2(d, b));
  }
};

template <typename F>
int fused_build(fargo_batch *b) {
  const unsigned n = (unsigned)b->ctx.size();
  ManyHost H[FU_N], HC[8];
  // argument blocks packed at their exact size: the kernels index them so
  for (auto &h : HC) h.asz = cfl_args_bytes<F>();
  H[FU_CFL].asz = cfl_args_bytes<F>();
  H[FU_DT].asz = dt_final_args_bytes();
  H[FU_SRC].asz = H[FU_SRCG].asz = source_args_bytes<F>();
  H[FU_VISC].asz = H[FU_VISC1].asz = visc_args_bytes<F>();
  H[FU_SY].asz = sweep_y_args_bytes<F>();
  H[FU_RX].asz = ring_x_args_bytes<F>();
  H[FU_VEL].asz = vel_args_bytes<F>();
  b->nxmax = 0;
  for (unsigned d = 0; d < n; d++) {
    fargo_ctx *c = b->ctx[d];
    Mesh m = c->m;
    m.chunk = b->chunk[d];
    b->nxmax = std::max(b->nxmax, m.nx);
    const StateT<F> S = state_of<F>(c, &b->st[d]);
    const double *dtp = c->w.dt;
    F *v2[4] = {(F *)c->v2[0], (F *)c->v2[1], (F *)c->v2[2], (F *)c->v2[3]};
    // the time-step pass in one launch per class of ring length (zones per
    // thread), each with its own argument array indexed by disk
    ManyHost &hc = HC[(m.nx + 255) / 256];
    hc.blocks(d, cfl_args<F>(m, S, c->v0, c->ringrate, c->ringshear, c->w.err, hc.slot(d)));
    H[FU_DT].blocks(d, dt_final_args(m, c->w, c->ringrate, c->ringshear, H[FU_DT].slot(d)));
    H[FU_SRC].blocks(d, source_args<F>(m, S, dtp, v2[0], v2[1], v2[2], v2[3], H[FU_SRC].slot(d)));
    H[FU_SRCG].blocks(d, source_ghosts_args<F>(m, S, v2[0], v2[1], v2[2], v2[3], H[FU_SRCG].slot(d)));
    StateT<F> P = S; // post-source fields, as in the step
    P.vx = v2[0];
    P.vy = v2[1];
    if (m.visc) {
      F *const tau[3] = {(F *)c->TA[T_RHO], (F *)c->TA[T_PXM], (F *)c->TA[T_PXP]};
      unsigned nb1 = 0;
      H[FU_VISC].blocks(d, visc_args<F>(m, S, v2[0], v2[1], (F *)c->v3[0], (F *)c->v3[1], dtp, tau,
                                        H[FU_VISC].slot(d), &nb1));
      visc_args<F>(m, S, v2[0], v2[1], (F *)c->v3[0], (F *)c->v3[1], dtp, tau, H[FU_VISC1].slot(d), &nb1);
      H[FU_VISC1].blocks(d, nb1);
      P.vx = (F *)c->v3[0];
      P.vy = (F *)c->v3[1];
    }
    P.vz = v2[2];
    P.e = v2[3];
    const TSetT<F> TA = tset<F>(c, c->TA), TB = tset<F>(c, c->TB);
    H[FU_SY].blocks(d, sweep_y_args<F>(m, P, TB, dtp, H[FU_SY].slot(d)));
    H[FU_RX].blocks(d, ring_x_args<F>(m, (const F *)P.vx, TB, TA, S, c->v0, dtp, H[FU_RX].slot(d)));
    H[FU_VEL].blocks(d, vel_args<F>(m, S, TA, H[FU_VEL].slot(d)));
  }
  size_t total = 0;
  for (auto &h : H) total += al(h.args.size()) + al(h.tab.size() * sizeof(uint2));
  for (auto &h : HC) total += al(h.args.size()) + al(h.tab.size() * sizeof(uint2));
  if (b->fmem) (void)hipFree(b->fmem);
  b->fmem = nullptr;
  if (hipMalloc(&b->fmem, total) != hipSuccess) return FARGO_ENOMEM;
  char *base = (char *)b->fmem;
  size_t o = 0;
  auto upload = [&](ManyHost &h, ManyGrid &g) {
    g = ManyGrid{nullptr, nullptr, (unsigned)h.tab.size()};
    if (h.tab.empty()) return FARGO_OK;
    if (hipMemcpy(base + o, h.args.data(), h.args.size(), hipMemcpyHostToDevice) != hipSuccess) return FARGO_EHIP;
    g.args = base + o;
    o += al(h.args.size());
    if (hipMemcpy(base + o, h.tab.data(), h.tab.size() * sizeof(uint2), hipMemcpyHostToDevice) != hipSuccess)
      return FARGO_EHIP;
    g.tab = (const uint2 *)(base + o);
    o += al(h.tab.size() * sizeof(uint2));
    return FARGO_OK;
  };
  for (int k = 0; k < FU_N; k++) {
    const int rc = upload(H[k], b->g[k]);
    if (rc) return rc;
  }
  for (int k = 0; k < 8; k++) {
    const int rc = upload(HC[k], b->gcfl[k]);
    if (rc) return rc;
  }
  return FARGO_OK;
}

// one step of every disk: the step's kernels, each once over all disks
template <typename F>
void fused_step(fargo_batch *b, Launch &L) {
  const Mesh &m0 = b->ctx[0]->m;
  for (int k = 1; k < 8; k++)                                                      // boxes 3, 4, 6
    if (b->gcfl[k].nblk) launch_cfl_many<F>(L, b->gcfl[k], 256 * k);
  launch_dt_final_many(L, b->g[FU_DT]);
  launch_source_many<F>(L, m0, b->g[FU_SRC], b->g[FU_SRCG]);                        // boxes 7a-7c
  if (m0.visc) launch_visc_many<F>(L, b->g[FU_VISC1], b->g[FU_VISC]);              // box 7d
  launch_sweep_y_many<F>(L, m0, b->g[FU_SY]);                                       // boxes 12a-c, Y
  launch_ring_x_many<F>(L, b->ctx[0]->nq, b->g[FU_RX]);                              // X, split, FARGO, 12d
  launch_vel_many<F>(L, b->g[FU_VEL]);                                              // 12d (v_y)
}

int fused_capture(fargo_batch *b) {
  batch_release_graph(b);
  int rc = fp32(b->ctx[0]) ? fused_build<float>(b) : fused_build<double>(b);
  if (rc) return rc;
  if (hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal) != hipSuccess) return FARGO_EHIP;
  Launch L{b->origin, nullptr};
  if (fp32(b->ctx[0])) fused_step<float>(b, L);
  else fused_step<double>(b, L);
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(b->origin, &g) != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return FARGO_EHIP;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) return FARGO_EHIP;
  return FARGO_OK;
}

} // namespace

extern "C" {

int fargo_batch_create(fargo_ctx *const *ctxs, const fargo_state *states, int count, int lanes,
                       fargo_batch **out) {
  if (!ctxs || !states || !out || count < 1 || lanes < 0 || lanes > 64) return FARGO_EINVAL;
  for (int d = 0; d < count; d++) {
    if (!ctxs[d]) return FARGO_EINVAL;
    int rc = check_state(ctxs[d], &states[d]);
    if (rc) return rc;
    if (ctxs[d]->dev != ctxs[0]->dev) return FARGO_EINVAL;
  }
  if (lanes == 0 && !fused_ok(ctxs, count)) return FARGO_EUNSUPPORTED;
  fargo_batch *b = new (std::nothrow) fargo_batch();
  if (!b) return FARGO_ENOMEM;
  b->ctx.assign(ctxs, ctxs + count);
  b->st.assign(states, states + count);
  for (int d = 0; d < count; d++) b->chunk.push_back(ctxs[d]->m.chunk);
  if (hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return FARGO_EHIP;
  }
  b->lanes = lanes;
  int rc = lanes == 0 ? fused_capture(b) : batch_capture(b, lanes);
  if (rc) {
    fargo_batch_destroy(b);
    return rc;
  }
  *out = b;
  return FARGO_OK;
}

int fargo_batch_step(fargo_batch *b, void *stream) {
  if (!b || !b->exec) return FARGO_EINVAL;
  return hip_ok(hipGraphLaunch(b->exec, (hipStream_t)stream));
}

int fargo_batch_chunks(const fargo_batch *b, int32_t *chunk, int n) {
  if (!b || !chunk || n != (int)b->ctx.size()) return FARGO_EINVAL;
  for (int d = 0; d < n; d++) chunk[d] = b->lanes == 0 ? b->chunk[d] : b->ctx[d]->m.chunk;
  return FARGO_OK;
}

int fargo_batch_tune(fargo_batch *b, const int32_t *lanes, int nlanes, const int32_t *chunks, int nchunks,
                     int steps, void *stream, int32_t *best) {
  if (!b || !chunks || nchunks < 1 || steps < 1) return FARGO_EINVAL;
  if (b->lanes != 0) { // the fused form ignores lanes
    if (!lanes || nlanes < 1) return FARGO_EINVAL;
    for (int t = 0; t < nlanes; t++)
      if (lanes[t] < 1 || lanes[t] > 64) return FARGO_EINVAL;
  }
  for (int t = 0; t < nchunks; t++)
    if (chunks[t] < 1) return FARGO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipStreamSynchronize(s) != hipSuccess) return FARGO_EHIP;
  // the evolving fields are saved and restored: tuning leaves the states as found
  std::vector<std::pair<void *, size_t>> fields;
  for (size_t d = 0; d < b->ctx.size(); d++) {
    const fargo_state &st = b->st[d];
    void *f[5] = {st.rho, st.vx, st.vy, b->ctx[d]->m.d3 ? st.vz : nullptr,
                  b->ctx[d]->p.eos == FARGO_ADIABATIC ? st.e : nullptr};
    for (void *p : f)
      if (p) fields.push_back({p, field_bytes(b->ctx[d])});
  }
  size_t total = 0;
  for (auto &f : fields) total += f.second;
  void *save = nullptr;
  if (hipMalloc(&save, total) != hipSuccess) return FARGO_ENOMEM;
  int rc = FARGO_OK;
  {
    size_t o = 0;
    for (auto &f : fields) {
      if (hipMemcpyAsync((char *)save + o, f.first, f.second, hipMemcpyDeviceToDevice, s) != hipSuccess) rc = FARGO_EHIP;
      o += f.second;
    }
  }
  std::vector<int> chunk0(b->ctx.size());
  for (size_t d = 0; d < b->ctx.size(); d++) chunk0[d] = b->ctx[d]->m.chunk;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = FARGO_EHIP;
  auto restore = [&]() {
    size_t o = 0;
    for (auto &f : fields) {
      if (!rc && hipMemcpyAsync(f.first, (char *)save + o, f.second, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = FARGO_EHIP;
      o += f.second;
    }
  };
  auto timed = [&](float &ms) {
    if (hipGraphLaunch(b->exec, s) != hipSuccess) rc = FARGO_EHIP; // warm-up
    if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = FARGO_EHIP;
    for (int k = 0; k < steps && !rc; k++)
      if (hipGraphLaunch(b->exec, s) != hipSuccess) rc = FARGO_EHIP;
    if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = FARGO_EHIP;
    if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = FARGO_EHIP;
  };
  if (b->lanes == 0) {
    // fused: the sweep's chunk length per size class of disks (floor(log2 ny)),
    // one class after the other, the others held at their best so far
    std::vector<int> cls(b->ctx.size());
    int cmin = 99, cmax = -1;
    for (size_t d = 0; d < b->ctx.size(); d++) {
      int c = 0;
      while ((2 << c) <= b->ctx[d]->m.ny) c++;
      cls[d] = c;
      cmin = std::min(cmin, c);
      cmax = std::max(cmax, c);
    }
    for (int c = cmin; c <= cmax && !rc; c++) {
      bool any = false;
      for (int v : cls) any |= v == c;
      if (!any) continue;
      float best_ms = 0.0f;
      int best_chunk = -1;
      for (int ci = 0; ci < nchunks && !rc; ci++) {
        for (size_t d = 0; d < b->ctx.size(); d++)
          if (cls[d] == c) b->chunk[d] = chunks[ci];
        rc = fused_capture(b);
        float ms = 0.0f;
        if (!rc) timed(ms);
        restore();
        if (!rc && (best_chunk < 0 || ms < best_ms)) {
          best_ms = ms;
          best_chunk = chunks[ci];
        }
      }
      for (size_t d = 0; d < b->ctx.size(); d++)
        if (cls[d] == c && best_chunk > 0) b->chunk[d] = best_chunk;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = FARGO_EHIP;
    (void)hipFree(save);
    if (rc) b->chunk = chunk0;
    const int rc2 = fused_capture(b);
    if (!rc) rc = rc2;
    if (!rc && best) {
      best[0] = 0;
      best[1] = b->chunk.back();
    }
    return rc;
  }
  float best_ms = 0.0f;
  int best_l = b->lanes, best_c = chunk0[0];
  // the fastest candidate's graph is kept as timed: a graph captured again
  // with the same width does not always run as fast (its streams differ)
  hipGraph_t kept_graph = nullptr;
  hipGraphExec_t kept_exec = nullptr;
  std::vector<hipStream_t> kept_ls;
  auto drop_kept = [&]() {
    if (kept_exec) (void)hipGraphExecDestroy(kept_exec);
    if (kept_graph) (void)hipGraphDestroy(kept_graph);
    for (hipStream_t q : kept_ls) (void)hipStreamDestroy(q);
    kept_exec = nullptr;
    kept_graph = nullptr;
    kept_ls.clear();
  };
  for (int ci = 0; ci < nchunks && !rc; ci++)
    for (int li = 0; li < nlanes && !rc; li++) {
      for (auto *c : b->ctx) c->m.chunk = chunks[ci];
      rc = batch_capture(b, lanes[li]);
      if (rc) break;
      if (hipGraphLaunch(b->exec, s) != hipSuccess) rc = FARGO_EHIP; // warm-up
      if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = FARGO_EHIP;
      for (int k = 0; k < steps && !rc; k++)
        if (hipGraphLaunch(b->exec, s) != hipSuccess) rc = FARGO_EHIP;
      if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = FARGO_EHIP;
      float ms = 0.0f;
      if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = FARGO_EHIP;
      if (!rc && (best_ms == 0.0f || ms < best_ms)) {
        best_ms = ms;
        best_l = lanes[li];
        best_c = chunks[ci];
        drop_kept();
        kept_graph = b->graph;
        kept_exec = b->exec;
        kept_ls.swap(b->ls);
        b->graph = nullptr;
        b->exec = nullptr;
      }
      // back to the saved state before the next candidate
      size_t o = 0;
      for (auto &f : fields) {
        if (!rc && hipMemcpyAsync(f.first, (char *)save + o, f.second, hipMemcpyDeviceToDevice, s) != hipSuccess)
          rc = FARGO_EHIP;
        o += f.second;
      }
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = FARGO_EHIP;
  (void)hipFree(save);
  for (size_t d = 0; d < b->ctx.size(); d++) b->ctx[d]->m.chunk = rc ? chunk0[d] : best_c;
  if (!rc && kept_exec) {
    batch_release_graph(b);
    b->graph = kept_graph;
    b->exec = kept_exec;
    b->ls.swap(kept_ls);
    b->lanes = best_l;
    kept_graph = nullptr;
    kept_exec = nullptr;
  } else {
    drop_kept();
    int rc2 = batch_capture(b, rc ? b->lanes : best_l);
    if (!rc) rc = rc2;
  }
  if (!rc && best) {
    best[0] = best_l;
    best[1] = best_c;
  }
  return rc;
}

void fargo_batch_destroy(fargo_batch *b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  batch_release_graph(b);
  if (b->fmem) (void)hipFree(b->fmem);
  if (b->origin) (void)hipStreamDestroy(b->origin);
  delete b;
}

} // extern "C"

// ---------------------------------------------------------------------------
// Learned flux correction
// ---------------------------------------------------------------------------
struct fargo_lfc {
  fargo_ctx *ctx = nullptr;
  fargo_lfc_params p{};
  LfcScales sc{};
  LfcBufs B{};
  int maxb = 1;        // samples the buffers hold
  int *flag = nullptr; // guard: 1 if the last apply was rejected
  void *mem = nullptr;
  int step = 0; // Adam steps since the parameters were set
};

namespace {

bool lfc_mesh_ok(const fargo_ctx *c) {
  const Mesh &m = c->m;
  return c->p.geometry == FARGO_CYLINDRICAL && !m.d3 && !fp32(c) && m.nx % 64 == 0;
}

// the samples' density and velocities, checked against the context
int lfc_feed(const fargo_lfc *l, const fargo_state *states, int32_t n, LfcFeed &in) {
  if (!states || n < 1 || n > l->maxb) return FARGO_EINVAL;
  in = LfcFeed{};
  for (int s = 0; s < n; s++) {
    const int rc = check_state(l->ctx, &states[s]);
    if (rc) return rc;
    in.rho[s] = (const double *)states[s].rho;
    in.vx[s] = (const double *)states[s].vx;
    in.vy[s] = (const double *)states[s].vy;
  }
  return FARGO_OK;
}

} // namespace

extern "C" {

int fargo_lfc_create(fargo_ctx *ctx, const fargo_lfc_params *p, fargo_lfc **out) {
  if (!ctx || !p || !out) return FARGO_EINVAL;
  *out = nullptr;
  if (!lfc_mesh_ok(ctx)) return FARGO_EUNSUPPORTED;
  if (!(p->rho_s != 0.0) || !(p->u_s != 0.0) || !(p->r_span != 0.0) || !(p->sigma > 0.0) || !(p->guard > 0.0) ||
      !std::isfinite(p->flux_scale) || p->max_batch < 0 || p->max_batch > LFC_MAXB)
    return FARGO_EINVAL;
  const int maxb = p->max_batch > 0 ? p->max_batch : 1;
  const long npix = (long)ctx->m.nx * ctx->m.ny, ntot = npix * maxb;
  long nwb = 0; // weight-gradient blocks, the most any batch size up to maxb takes
  for (int n = 1; n <= maxb; n++) nwb = std::max(nwb, (long)lfc_wblocks(ctx->m.nx, ctx->m.ny, n, nullptr, nullptr));
  const long nlb = (ntot + 255) / 256;
  // one allocation, carved in 256-byte aligned slots
  size_t off = 0;
  auto slot = [&](size_t bytes) {
    size_t o = off;
    off += al(bytes);
    return o;
  };
  const size_t o_f = slot(ntot * 4 * 2), o_h1 = slot(ntot * 32 * 2), o_h2 = slot(ntot * 32 * 2),
               o_o = slot(ntot * 2 * 4), o_g3 = slot(ntot * 4 * 2), o_g2 = slot(ntot * 32 * 2),
               o_g1 = slot(ntot * 32 * 2), o_drho = slot(ntot * 8), o_gD = slot(ntot * 8), o_lp = slot(nlb * 8),
               o_loss = slot(8), o_flag = slot(4), o_w = slot(LFC_NPARAM * 4), o_mo = slot(LFC_NPARAM * 4),
               o_ve = slot(LFC_NPARAM * 4), o_gr = slot(LFC_NPARAM * 4), o_part = slot(nwb * LFC_NPARAM * 4), o_wp1 = slot(2048 * 2), o_wp2 = slot(9216 * 2), o_wp3 = slot(4608 * 2),
               o_wpa3 = slot(2048 * 2), o_wpa2 = slot(9216 * 2);
  fargo_lfc *l = new fargo_lfc;
  if (hipSetDevice(ctx->dev) != hipSuccess || hipMalloc(&l->mem, off) != hipSuccess) {
    delete l;
    return FARGO_ENOMEM;
  }
  if (hipMemset(l->mem, 0, off) != hipSuccess) {
    fargo_lfc_destroy(l);
    return FARGO_EHIP;
  }
  char *b = (char *)l->mem;
  LfcBufs &B = l->B;
  B.f = (unsigned short *)(b + o_f);
  B.h1 = (unsigned short *)(b + o_h1);
  B.h2 = (unsigned short *)(b + o_h2);
  B.o = (float *)(b + o_o);
  B.g3 = (unsigned short *)(b + o_g3);
  B.g2 = (unsigned short *)(b + o_g2);
  B.g1 = (unsigned short *)(b + o_g1);
  B.drho = (double *)(b + o_drho);
  B.gD = (double *)(b + o_gD);
  B.lpart = (double *)(b + o_lp);
  B.loss = (double *)(b + o_loss);
  l->flag = (int *)(b + o_flag);
  B.w = (float *)(b + o_w);
  B.mo = (float *)(b + o_mo);
  B.ve = (float *)(b + o_ve);
  B.grad = (float *)(b + o_gr);
  B.part = (float *)(b + o_part);
  B.wt.wp1 = (unsigned short *)(b + o_wp1);
  B.wt.wp2 = (unsigned short *)(b + o_wp2);
  B.wt.wp3 = (unsigned short *)(b + o_wp3);
  B.wt.wpa3 = (unsigned short *)(b + o_wpa3);
  B.wt.wpa2 = (unsigned short *)(b + o_wpa2);
  l->ctx = ctx;
  l->p = *p;
  l->maxb = maxb;
  l->sc = LfcScales{p->rho_s, p->u_s, p->r_mid, p->r_span};
  *out = l;
  return FARGO_OK;
}

void fargo_lfc_destroy(fargo_lfc *l) {
  if (!l) return;
  (void)hipDeviceSynchronize();
  if (l->mem) (void)hipFree(l->mem);
  delete l;
}

int fargo_lfc_set_params(fargo_lfc *l, const float *host, int32_t n) {
  if (!l || !host || n != LFC_NPARAM) return FARGO_EINVAL;
  for (int e = 0; e < n; e++)
    if (!std::isfinite(host[e])) return FARGO_EINVAL;
  if (hipMemcpy(l->B.w, host, (size_t)n * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(l->B.mo, 0, (size_t)n * 4) != hipSuccess || hipMemset(l->B.ve, 0, (size_t)n * 4) != hipSuccess)
    return FARGO_EHIP;
  Launch L{nullptr, nullptr};
  lfc_pack(L, l->B);
  l->step = 0;
  return hipDeviceSynchronize() == hipSuccess && hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

static int lfc_copy_out(const float *dev, float *host, int32_t n) {
  if (!host || n != LFC_NPARAM) return FARGO_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return FARGO_EHIP;
  return hipMemcpy(host, dev, (size_t)n * 4, hipMemcpyDeviceToHost) == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_lfc_get_params(fargo_lfc *l, float *host, int32_t n) { return l ? lfc_copy_out(l->B.w, host, n) : FARGO_EINVAL; }

int fargo_lfc_get_grad(fargo_lfc *l, float *host, int32_t n) {
  return l ? lfc_copy_out(l->B.grad, host, n) : FARGO_EINVAL;
}

int fargo_lfc_forward_batch(fargo_lfc *l, const fargo_state *states, int32_t n, void *stream) {
  if (!l) return FARGO_EINVAL;
  LfcFeed in;
  int rc = lfc_feed(l, states, n, in);
  if (rc) return rc;
  Launch L{(hipStream_t)stream, &l->ctx->prof};
  const Mesh &m = l->ctx->m;
  lfc_forward(L, m, in, n, l->sc, l->B);
  lfc_drho(L, m, n, l->B, l->p.flux_scale, nullptr, l->p.sigma);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_lfc_forward(fargo_lfc *l, const fargo_state *state, void *stream) {
  return fargo_lfc_forward_batch(l, state, 1, stream);
}

int fargo_lfc_train_batch(fargo_lfc *l, const fargo_state *states, const double *const *targets, int32_t n,
                          double lr, void *stream) {
  if (!l || !targets || !(lr > 0.0) || !std::isfinite(lr)) return FARGO_EINVAL;
  LfcFeed in;
  int rc = lfc_feed(l, states, n, in);
  if (rc) return rc;
  LfcTargets tg{};
  for (int s = 0; s < n; s++) {
    if (!targets[s]) return FARGO_EINVAL;
    tg.t[s] = targets[s];
  }
  Launch L{(hipStream_t)stream, &l->ctx->prof};
  const Mesh &m = l->ctx->m;
  lfc_forward(L, m, in, n, l->sc, l->B);
  lfc_drho(L, m, n, l->B, l->p.flux_scale, &tg, l->p.sigma);
  lfc_backward(L, m, n, l->B, l->p.flux_scale);
  l->step++;
  const double c1 = 1.0 - std::pow(0.9, l->step), c2 = 1.0 - std::pow(0.999, l->step);
  lfc_adam(L, l->B, (float)lr, (float)c1, (float)c2);
  lfc_pack(L, l->B);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_lfc_train_step(fargo_lfc *l, const fargo_state *state, const double *target, double lr, void *stream) {
  return fargo_lfc_train_batch(l, state, &target, 1, lr, stream);
}

int fargo_lfc_apply(fargo_lfc *l, fargo_state *state, void *stream) {
  int rc = fargo_lfc_forward(l, state, stream);
  if (rc) return rc;
  Launch L{(hipStream_t)stream, &l->ctx->prof};
  lfc_apply(L, l->ctx->m, l->B, (double *)state->rho, l->p.guard, l->flag);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_lfc_result(fargo_lfc *l, double *loss, int32_t *skipped, void *stream) {
  if (!l) return FARGO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipStreamSynchronize(s) != hipSuccess) return FARGO_EHIP;
  if (loss && hipMemcpy(loss, l->B.loss, 8, hipMemcpyDeviceToHost) != hipSuccess) return FARGO_EHIP;
  if (skipped) {
    int f = 0;
    if (hipMemcpy(&f, l->flag, 4, hipMemcpyDeviceToHost) != hipSuccess) return FARGO_EHIP;
    *skipped = f;
  }
  return FARGO_OK;
}

int fargo_lfc_get_views(fargo_lfc *l, fargo_lfc_views *v) {
  if (!l || !v) return FARGO_EINVAL;
  v->f = l->B.f;
  v->h1 = l->B.h1;
  v->h2 = l->B.h2;
  v->o = l->B.o;
  v->drho = l->B.drho;
  v->g3 = l->B.g3;
  v->g2 = l->B.g2;
  v->g1 = l->B.g1;
  return FARGO_OK;
}

int fargo_lfc_target(const fargo_ctx *ctx, const fargo_state *ref, const fargo_state *plain, double *target,
                     void *stream) {
  if (!ctx || !ref || !plain || !target || !ref->rho || !plain->rho) return FARGO_EINVAL;
  if (ctx->p.geometry != FARGO_CYLINDRICAL || ctx->m.d3 || fp32(ctx)) return FARGO_EUNSUPPORTED;
  Launch L{(hipStream_t)stream, nullptr};
  lfc_target(L, ctx->m, (const double *)ref->rho, (const double *)plain->rho, target);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

int fargo_lfc_restrict(const fargo_ctx *fine, const fargo_state *fs, const fargo_ctx *coarse, fargo_state *cs,
                       void *stream) {
  if (!fine || !coarse || !fs || !cs) return FARGO_EINVAL;
  const Mesh &mf = fine->m, &mc = coarse->m;
  for (const fargo_ctx *c : {fine, coarse})
    if (c->p.geometry != FARGO_CYLINDRICAL || c->m.d3 || fp32(c)) return FARGO_EUNSUPPORTED;
  const int R = mc.nx > 0 ? mf.nx / mc.nx : 0; // 2 or 4
  if ((R != 2 && R != 4) || mf.nx != R * mc.nx || mf.ny != R * mc.ny || fine->p.xmin != coarse->p.xmin ||
      fine->p.xmax != coarse->p.xmax)
    return FARGO_EINVAL;
  for (int J = 0; J <= mc.ny; J++) {
    const double yc = coarse->ymin[NGH + J], yf = fine->ymin[NGH + R * J];
    if (!(std::fabs(yc - yf) <= 1e-12 * std::fabs(yc))) return FARGO_EINVAL;
  }
  if (!fs->rho || !fs->vx || !fs->vy || !cs->rho || !cs->vx || !cs->vy) return FARGO_EINVAL;
  Launch L{(hipStream_t)stream, nullptr};
  lfc_restrict(L, mf, (const double *)fs->rho, (const double *)fs->vx, (const double *)fs->vy, mc, (double *)cs->rho,
               (double *)cs->vx, (double *)cs->vy);
  return hipGetLastError() == hipSuccess ? FARGO_OK : FARGO_EHIP;
}

} // extern "C"
