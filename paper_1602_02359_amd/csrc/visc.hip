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

// Two passes.  1: the stress components, each formed once: tau_phiphi and
// tau_rr of every zone in rows j0 - 1 .. jn - 1, tau_rphi of every edge in
// rows j0 .. jn, into three scratch fields.  2: their divergence on the
// faces (ghost zones carry v'' over).
template <typename F>
__device__ __forceinline__ void visc_tau_body(Visc<F> V, F *__restrict__ tpp, F *__restrict__ trr,
                                              F *__restrict__ trp, unsigned bid_, unsigned nbk_) {
  const Mesh &m = V.m;
  const int nib = (m.nx + blockDim.x - 1) / blockDim.x;
  const unsigned Lb = xcd_remap(bid_, nbk_);
  const int j = m.j0 - 1 + (int)(Lb / (unsigned)nib);
  const int i = (int)(Lb % (unsigned)nib) * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx || j > m.jn) return;
  const unsigned c = V.at(i, j);
  if (j < m.jn) {
    F a, b;
    V.diag(i, j, a, b);
    tpp[c] = a;
    trr[c] = b;
  }
  if (j >= m.j0) trp[c] = V.edge(i, j);
}

template <typename F>
__device__ __forceinline__ void visc_div_body(Visc<F> V, const F *__restrict__ tpp, const F *__restrict__ trr,
                                              const F *__restrict__ trp, const double *__restrict__ dtp,
                                              F *__restrict__ vx3, F *__restrict__ vy3, unsigned bid_,
                                              unsigned nbk_) {
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
  const int im = V.wrapx(i - 1);
  const unsigned cw = V.at(im, j), cs_ = c - (unsigned)m.pitch;
  // v_phi on the X face of zone (i, j)
  const F a = (F)m.g.ymin(j), b = (F)m.g.ymin(j + 1), r = (F)m.g.ymed(j);
  const F rx = F(0.5) * (rho[c] + rho[cw]);
  const F e0 = trp[c], tpp0 = tpp[c];
  const F divx = (b * b * trp[c + (unsigned)m.pitch] - a * a * e0) / (r * r * (F)m.g.Ly(j)) + (tpp0 - tpp[cw]) / (r * dphi);
  vx3[c] = V.vx[c] - dt * divx / rx;
  // v_r on the Y face of zone (i, j), if the step owns it
  if (j >= m.ylo()) {
    const F ry = F(0.5) * (rho[c] + rho[cs_]);
    const F divy = ((F)m.g.ymed(j) * trr[c] - (F)m.g.ymed(j - 1) * trr[cs_]) / (a * (F)m.g.hy(j)) +
                   (trp[V.at(V.wrapx(i + 1), j)] - e0) / (a * dphi) - F(0.5) * (tpp0 + tpp[cs_]) / a;
    vy3[c] = V.vy[c] - dt * divy / ry;
  } else {
    vy3[c] = V.vy[c];
  }
}

template <typename F>
__global__ __launch_bounds__(256) void k_visc_tau(Visc<F> V, F *__restrict__ tpp, F *__restrict__ trr,
                                                  F *__restrict__ trp) {
  visc_tau_body<F>(V, tpp, trr, trp, blockIdx.x, gridDim.x);
}
template <typename F>
__global__ __launch_bounds__(256) void k_visc(Visc<F> V, const F *__restrict__ tpp, const F *__restrict__ trr,
                                              const F *__restrict__ trp, const double *__restrict__ dtp,
                                              F *__restrict__ vx3, F *__restrict__ vy3) {
  visc_div_body<F>(V, tpp, trr, trp, dtp, vx3, vy3, blockIdx.x, gridDim.x);
}

// multi-mesh forms (ManyGrid): one argument block serves both passes
template <typename F>
struct ViscArgs {
  Visc<F> V;
  F *tpp, *trr, *trp;
  const double *dt;
  F *vx3, *vy3;
  unsigned nb, nb1;
};
template <typename F>
__global__ __launch_bounds__(256) void k_visc_tau_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const ViscArgs<F> a = many_args<ViscArgs<F>>(args, t.x);
  visc_tau_body<F>(a.V, a.tpp, a.trr, a.trp, t.y, a.nb1);
}
template <typename F>
__global__ __launch_bounds__(256) void k_visc_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const ViscArgs<F> a = many_args<ViscArgs<F>>(args, t.x);
  visc_div_body<F>(a.V, a.tpp, a.trr, a.trp, a.dt, a.vx3, a.vy3, t.y, a.nb);
}

} // namespace

template <typename F>
void launch_visc(Launch &L, const Mesh &m, const StateT<F> &s, const F *vx2, const F *vy2, F *vx3, F *vy3,
                 const double *dt, F *const tau[3]) {
  const int bs = 256, nib = (m.nx + bs - 1) / bs;
  const Visc<F> V{m, s, vx2, vy2};
  prof_begin(L, K_VISC);
  k_visc_tau<F><<<(unsigned)nib * (unsigned)(m.ny + 2), bs, 0, L.s>>>(V, tau[0], tau[1], tau[2]);
  k_visc<F><<<(unsigned)nib * (unsigned)m.nyg, bs, 0, L.s>>>(V, tau[0], tau[1], tau[2], dt, vx3, vy3);
  prof_end(L, K_VISC);
}

template void launch_visc<double>(Launch &, const Mesh &, const StateT<double> &, const double *, const double *,
                                  double *, double *, const double *, double *const[3]);
template void launch_visc<float>(Launch &, const Mesh &, const StateT<float> &, const float *, const float *,
                                 float *, float *, const double *, float *const[3]);

template <typename F>
size_t visc_args_bytes() { return sizeof(ViscArgs<F>); }

// the blocks of the second pass; those of the first through *nb1
template <typename F>
unsigned visc_args(const Mesh &m, const StateT<F> &s, const F *vx2, const F *vy2, F *vx3, F *vy3, const double *dt,
                   F *const tau[3], void *dst, unsigned *nb1) {
  const int bs = 256, nib = (m.nx + bs - 1) / bs;
  const unsigned nb = (unsigned)nib * (unsigned)m.nyg, n1 = (unsigned)nib * (unsigned)(m.ny + 2);
  *(ViscArgs<F> *)dst = ViscArgs<F>{Visc<F>{m, s, vx2, vy2}, tau[0], tau[1], tau[2], dt, vx3, vy3, nb, n1};
  *nb1 = n1;
  return nb;
}

template <typename F>
void launch_visc_many(Launch &L, const ManyGrid &g1, const ManyGrid &g) {
  prof_begin(L, K_VISC);
  k_visc_tau_many<F><<<g1.nblk, 256, 0, L.s>>>(g1.args, g1.tab);
  k_visc_many<F><<<g.nblk, 256, 0, L.s>>>(g.args, g.tab);
  prof_end(L, K_VISC);
}

#define FARGO_VISC_MANY(F)                                                                                          \
  template size_t visc_args_bytes<F>();                                                                            \
  template unsigned visc_args<F>(const Mesh &, const StateT<F> &, const F *, const F *, F *, F *, const double *,  \
                                 F *const[3], void *, unsigned *);                                                 \
  template void launch_visc_many<F>(Launch &, const ManyGrid &, const ManyGrid &);
FARGO_VISC_MANY(double)
FARGO_VISC_MANY(float)
#undef FARGO_VISC_MANY

} // namespace fargo
