// Box 7d: kinematic viscosity, cylindrical 2D (phi, r), App. B: the stress
// components of Eq. 73 (tau_phiphi and tau_rr at zone centres, tau_rphi on
// the zone's lower edge in both X and Y, Fig. "stress") and their divergence
// (Eq. 76).  Every component comes from the velocities after box 7b (Jacobi);
// v_phi is updated on the X faces of active zones and v_r on the owned Y
// faces, with the face density of Eq. 20; ghost zones carry v'' over.  On an
// edge, rho and nu are the means of the four zones sharing it and v_phi / r
// is the mean of v_phi / r on the two X faces it joins.  Each thread forms
// the few components its two faces need; the field type F is double or float.
#include "fargo_internal.h"

namespace fargo {

namespace {

template <typename F>
struct Visc {
  Mesh m;
  StateT<F> s;
  const F *vx, *vy;

  __device__ inline unsigned at(int i, int j) const { return m.o32(i, j, 0); }
  __device__ inline int wrapx(int i) const { return i < 0 ? i + m.nx : (i >= m.nx ? i - m.nx : i); }
  // tau_phiphi and tau_rr of zone (a, b)
  __device__ inline void diag(int a, int b, F &tpp, F &trr) const {
    const unsigned c = at(a, b), cxp = at(wrapx(a + 1), b), cyp = c + (unsigned)m.pitch;
    const F dphi = (F)m.dx, r = (F)m.g.ymed(b);
    const F divv = (F)m.Vinv(b, 0) * ((F)m.Sx(b, 0) * (vx[cxp] - vx[c]) +
                                      ((F)m.Sy(b + 1, 0) * vy[cyp] - (F)m.Sy(b, 0) * vy[c]));
    const F rn = s.rho[c] * s.nu[c];
    const F ur = F(0.5) * (vy[c] + vy[cyp]);
    tpp = -rn * (F(2) * ((vx[cxp] - vx[c]) / (r * dphi) + ur / r) - F(2) / F(3) * divv);
    trr = -rn * (F(2) * (vy[cyp] - vy[c]) / (F)m.g.Ly(b) - F(2) / F(3) * divv);
  }
  // tau_rphi on the edge of zone (a, b) at its lower X and Y faces
  __device__ inline F edge(int a, int b) const {
    const int am = wrapx(a - 1);
    const unsigned c = at(a, b), cw = at(am, b), cs_ = c - (unsigned)m.pitch, csw = cw - (unsigned)m.pitch;
    const F rho4 = F(0.25) * (s.rho[c] + s.rho[cw] + s.rho[cs_] + s.rho[csw]);
    const F nu4 = F(0.25) * (s.nu[c] + s.nu[cw] + s.nu[cs_] + s.nu[csw]);
    const F dvphi_dr = (vx[c] - vx[cs_]) / (F)m.g.hy(b);
    const F vphi_r = F(0.5) * (vx[c] / (F)m.g.ymed(b) + vx[cs_] / (F)m.g.ymed(b - 1));
    const F dvr_dphi = (vy[c] - vy[cw]) / ((F)m.g.ymin(b) * (F)m.dx);
    F shear = dvphi_dr - vphi_r;
    // an FP32 v_phi is a deviation from its ring's background: the same two
    // terms of the background, formed in FP64 and rounded once
    if constexpr (sizeof(F) == 4) shear += (F)m.bg(BG_KV, b, 0);
    return -rho4 * nu4 * (shear + dvr_dphi);
  }
};

template <typename F>
__device__ __forceinline__ void visc_body(Visc<F> V, const double *__restrict__ dtp, F *__restrict__ vx3,
                                              F *__restrict__ vy3, unsigned bid_, unsigned nbk_) {
  const Mesh &m = V.m;
  const int nib = (m.nx + blockDim.x - 1) / blockDim.x;
  const unsigned Lb = xcd_remap(bid_, nbk_);
  const int j = (int)(Lb / (unsigned)nib);
  const int i = (int)(Lb % (unsigned)nib) * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx || j >= m.nyg) return;
  const unsigned c = V.at(i, j);
  if (j < m.j0 || j >= m.jn) {
    vx3[c] = V.vx[c];
    vy3[c] = V.vy[c];
    return;
  }
  const F dt = (F)*dtp, dphi = (F)m.dx;
  const F *rho = V.s.rho;
  // every stress component the zone's two faces need, each formed once
  // (the stores come last, so that no load waits behind them)
  const int im = V.wrapx(i - 1);
  const bool own_y = j >= m.ylo();
  F tpp0, trr0, tppw, trrw, tpps = F(0), trrs = F(0);
  V.diag(i, j, tpp0, trr0);
  V.diag(im, j, tppw, trrw);
  if (own_y) V.diag(i, j - 1, tpps, trrs);
  const F e0 = V.edge(i, j), en = V.edge(i, j + 1);
  const F ee = own_y ? V.edge(V.wrapx(i + 1), j) : F(0);
  // v_phi on the X face of zone (i, j)
  const F a = (F)m.g.ymin(j), b = (F)m.g.ymin(j + 1), r = (F)m.g.ymed(j);
  const F rx = F(0.5) * (rho[c] + rho[V.at(im, j)]);
  const F divx = (b * b * en - a * a * e0) / (r * r * (F)m.g.Ly(j)) + (tpp0 - tppw) / (r * dphi);
  const F vx3c = V.vx[c] - dt * divx / rx;
  // v_r on the Y face of zone (i, j), if the step owns it
  F vy3c = V.vy[c];
  if (own_y) {
    const F ry = F(0.5) * (rho[c] + rho[c - (unsigned)m.pitch]);
    const F divy = ((F)m.g.ymed(j) * trr0 - (F)m.g.ymed(j - 1) * trrs) / (a * (F)m.g.hy(j)) +
                   (ee - e0) / (a * dphi) - F(0.5) * (tpp0 + tpps) / a;
    vy3c = vy3c - dt * divy / ry;
  }
  vx3[c] = vx3c;
  vy3[c] = vy3c;
}
template <typename F>
__global__ __launch_bounds__(256) void k_visc(Visc<F> V, const double *__restrict__ dtp, F *__restrict__ vx3,
                                              F *__restrict__ vy3) {
  visc_body<F>(V, dtp, vx3, vy3, blockIdx.x, gridDim.x);
}

// multi-mesh form (ManyGrid)
template <typename F>
struct ViscArgs {
  Visc<F> V;
  const double *dt;
  F *vx3, *vy3;
  unsigned nb;
};
template <typename F>
__global__ __launch_bounds__(256) void k_visc_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const ViscArgs<F> a = many_args<ViscArgs<F>>(args, t.x);
  visc_body<F>(a.V, a.dt, a.vx3, a.vy3, t.y, a.nb);
}

} // namespace

template <typename F>
void launch_visc(Launch &L, const Mesh &m, const StateT<F> &s, const F *vx2, const F *vy2, F *vx3, F *vy3,
                 const double *dt) {
  const int bs = 256, nib = (m.nx + bs - 1) / bs;
  const unsigned nb = (unsigned)nib * (unsigned)m.nyg;
  prof_begin(L, K_VISC);
  k_visc<F><<<nb, bs, 0, L.s>>>(Visc<F>{m, s, vx2, vy2}, dt, vx3, vy3);
  prof_end(L, K_VISC);
}

template void launch_visc<double>(Launch &, const Mesh &, const StateT<double> &, const double *, const double *,
                                  double *, double *, const double *);
template void launch_visc<float>(Launch &, const Mesh &, const StateT<float> &, const float *, const float *,
                                 float *, float *, const double *);

template <typename F>
size_t visc_args_bytes() { return sizeof(ViscArgs<F>); }

template <typename F>
unsigned visc_args(const Mesh &m, const StateT<F> &s, const F *vx2, const F *vy2, F *vx3, F *vy3, const double *dt,
                   void *dst) {
  const int bs = 256, nib = (m.nx + bs - 1) / bs;
  const unsigned nb = (unsigned)nib * (unsigned)m.nyg;
  *(ViscArgs<F> *)dst = ViscArgs<F>{Visc<F>{m, s, vx2, vy2}, dt, vx3, vy3, nb};
  return nb;
}

template <typename F>
void launch_visc_many(Launch &L, const ManyGrid &g) {
  prof_begin(L, K_VISC);
  k_visc_many<F><<<g.nblk, 256, 0, L.s>>>(g.args, g.tab);
  prof_end(L, K_VISC);
}

#define FARGO_VISC_MANY(F)                                                                                          \
  template size_t visc_args_bytes<F>();                                                                            \
  template unsigned visc_args<F>(const Mesh &, const StateT<F> &, const F *, const F *, F *, F *, const double *,  \
                                 void *);                                                                          \
  template void launch_visc_many<F>(Launch &, const ManyGrid &);
FARGO_VISC_MANY(double)
FARGO_VISC_MANY(float)
#undef FARGO_VISC_MANY

} // namespace fargo
