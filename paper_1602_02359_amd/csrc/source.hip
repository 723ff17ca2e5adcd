// Box 7: source step (Sect. 3.3), boxes 7a, 7b and 7c fused in one pass.
//   7a  pressure and potential gradients on the owned faces, centrifugal
//       terms as squares of four-point arithmetic averages (Eq. 12 and its
//       generalisation); Jacobi: every face reads only v^n.  The pressure
//       term uses the arithmetic mean of the two face densities (Eq. 20),
//       which makes it momentum conserving (Eqs. 21-25).
//   7b  von Neumann-Richtmyer artificial viscosity per direction,
//       q = C^2 rho dv^2 where dv < 0, its gradient in the same conservative
//       form, and the heating -q dv / L.
//   7c  compressional heating of a gamma-law gas, time-centred:
//       e <- e (1 - a)/(1 + a), a = dt (gamma - 1) div(v) / 2.
// A zone owns its lower X, Y and Z faces (the lower Y/Z boundary face only in
// a periodic direction).  Active zones recompute the few intermediate face
// values their stencil needs (v' on four faces and q in three zones per
// direction) instead of storing them.  Results go to separate arrays (v'',
// e''), so the pass reads the state while it writes.
#include "fargo_internal.h"

namespace fargo {

namespace {

// The field type F is double, or float for the FP32-bulk state; arithmetic is
// carried out in F, geometric factors are rounded to F where they are used.
template <typename F>
struct Src {
  Mesh m;
  StateT<F> s;
  F dt;

  __device__ inline F P(unsigned c) const {
    return m.eos == FARGO_ISOTHERMAL ? s.cs[c] * s.cs[c] * s.rho[c] : (F)(m.gamma - 1.0) * s.e[c];
  }
  __device__ inline bool yowned(int jj) const { return jj >= m.ylo() && jj < m.jn; }
  __device__ inline bool zowned(int kk) const { return kk >= m.zlo() && kk < m.kn; }
};

template <typename F>
__device__ inline F qvisc(F c2, F rho, F dv) { return dv < F(0) ? c2 * rho * dv * dv : F(0); }

// What a zone's Z stencil needs from one plane of its column.
template <typename F>
struct Plane {
  F rho, P, pot, vz, vx, vxp; // vxp: v_x on the next X face (spherical centrifugal term)
};

// X and Y parts of box 7 at zone (i, j, k): v''_x of face i and v''_y of face
// j (written), and the heating and divergence contributions.  The values of
// the five zones of each stencil are loaded once and the four face values
// v' per direction are formed from them.
template <typename F>
__device__ inline void xy_part(const Src<F> &S, int i, int j, int k, unsigned c, F *__restrict__ vx2,
                               F *__restrict__ vy2, F &heat, F &flux) {
  const Mesh &m = S.m;
  const StateT<F> &s = S.s;
  const F dt = S.dt, c2 = (F)(m.cvnr * m.cvnr), om = (F)m.omega;
  const unsigned row = c - (unsigned)i;
  // ---- X: zones i-2 .. i+2, faces i-1 .. i+2
  {
    int ix[5];
    ix[2] = i;
    ix[1] = i == 0 ? m.nx - 1 : i - 1;
    ix[0] = ix[1] == 0 ? m.nx - 1 : ix[1] - 1;
    ix[3] = i + 1 == m.nx ? 0 : i + 1;
    ix[4] = ix[3] + 1 == m.nx ? 0 : ix[3] + 1;
    F r[5], P[5], ph[5], a[4];
#pragma unroll
    for (int t = 0; t < 5; t++) {
      unsigned cc = row + (unsigned)ix[t];
      r[t] = s.rho[cc];
      P[t] = S.P(cc);
      ph[t] = s.pot[cc];
    }
    const F dX = (F)m.DX(j, k);
#pragma unroll
    for (int t = 0; t < 4; t++) {
      F gradP = F(2) * (P[t + 1] - P[t]) / ((r[t + 1] + r[t]) * dX);
      F gradPhi = (ph[t + 1] - ph[t]) / dX;
      a[t] = s.vx[row + (unsigned)ix[t + 1]] - dt * (gradP + gradPhi);
    }
    F dvx = a[2] - a[1];
    F qx = qvisc(c2, r[2], dvx);
    F qxm = qvisc(c2, r[1], a[1] - a[0]), qxp = qvisc(c2, r[3], a[3] - a[2]);
    F bx1 = a[1] - dt * F(2) * (qx - qxm) / ((r[2] + r[1]) * dX);
    F bx2 = a[2] - dt * F(2) * (qxp - qx) / ((r[3] + r[2]) * dX);
    vx2[c] = bx1;
    heat = qx * dvx / dX;
    flux = (F)m.Sx(j, k) * (bx2 - bx1);
  }
  // ---- Y: zones jy[0..4] = below(below(j)) .. above(above(j)); faces jy[1..4]
  {
    int jy[5];
    jy[2] = j;
    jy[1] = m.jbelow(j);
    jy[0] = m.jbelow(jy[1]);
    jy[3] = m.jabove(j);
    jy[4] = m.jabove(jy[3]);
    const int ip = i + 1 == m.nx ? 0 : i + 1;
    const int kp = m.d3 ? m.kabove(k) : k;
    const bool sph = m.geo == FARGO_SPHERICAL, cyl = m.geo == FARGO_CYLINDRICAL;
    const unsigned plane = (unsigned)m.plane();
    F r[5], P[5], ph[5], vt[5], vth[5], a[4];
#pragma unroll
    for (int t = 0; t < 5; t++) {
      unsigned cc = m.o32(i, jy[t], k);
      r[t] = s.rho[cc];
      P[t] = S.P(cc);
      ph[t] = s.pot[cc];
      // azimuthal velocity in the inertial frame on the two X faces of the zone
      F R = (F)(sph ? m.g.ymed[jy[t]] * m.g.sinz[k] : m.g.ymed[jy[t]]);
      vt[t] = (s.vx[cc] + R * om) + (s.vx[cc - (unsigned)i + (unsigned)ip] + R * om);
      vth[t] = sph ? s.vz[cc] + s.vz[cc + (kp - k) * plane] : F(0);
    }
#pragma unroll
    for (int t = 0; t < 4; t++) {
      int f = jy[t + 1];
      unsigned cf = m.o32(i, f, k);
      if (!S.yowned(f)) {
        a[t] = s.vy[cf];
        continue;
      }
      F h = (F)m.g.hy[f];
      F gradP = F(2) * (P[t + 1] - P[t]) / ((r[t + 1] + r[t]) * h);
      F gradPhi = (ph[t + 1] - ph[t]) / h;
      F src = F(0);
      if (cyl || sph) {
        F v = F(0.25) * (vt[t + 1] + vt[t]);
        src = v * v;
        if (sph) {
          F w = F(0.25) * (vth[t + 1] + vth[t]);
          src += w * w;
        }
        src /= (F)m.g.ymin[f];
      }
      a[t] = s.vy[cf] - dt * (gradP + gradPhi) + dt * src;
    }
    F dvy = a[2] - a[1];
    F qy = qvisc(c2, r[2], dvy);
    F by1 = a[1], by2 = a[2]; // v^n on faces that are not owned
    if (S.yowned(j)) {
      F qb = qvisc(c2, r[1], a[1] - a[0]);
      by1 = a[1] - dt * F(2) * (qy - qb) / ((r[2] + r[1]) * (F)m.g.hy[j]);
    }
    if (S.yowned(jy[3])) {
      F qa = qvisc(c2, r[3], a[3] - a[2]);
      by2 = a[2] - dt * F(2) * (qa - qy) / ((r[3] + r[2]) * (F)m.g.hy[jy[3]]);
    }
    vy2[c] = by1;
    heat += qy * dvy / (F)m.g.Ly[j];
    flux += (F)m.Sy(j + 1, k) * by2 - (F)m.Sy(j, k) * by1;
  }
}

// 7c: e'' of zone c from e, the heating and the face-flux divergence sum
template <typename F>
__device__ inline void energy(const Src<F> &S, int j, int k, unsigned c, F heat, F flux, F *__restrict__ e2) {
  const Mesh &m = S.m;
  F e1 = S.s.e[c] - S.dt * heat;
  F a = F(0.5) * S.dt * (F)(m.gamma - 1.0) * ((F)m.Vinv(j, k) * flux);
  e2[c] = e1 * (F(1) - a) / (F(1) + a);
}

// One thread per (i, j) column marching along Z: the Z stencil of a zone
// (planes k-2 .. k+2, in the periodic order when Z is periodic) lives in a
// register window, so each value of the column is loaded once; the Y
// neighbours come from the columns of co-scheduled blocks (j fastest) at the
// same plane.  Ghost zones copy v^n and e.
template <typename F>
__global__ __launch_bounds__(256, 3) void k_source(Mesh m, StateT<F> s, const double *__restrict__ dtp,
                                                F *__restrict__ vx2, F *__restrict__ vy2, F *__restrict__ vz2,
                                                F *__restrict__ e2) {
  unsigned L = xcd_remap(blockIdx.x, gridDim.x);
  int j = (int)(L % (unsigned)m.nyg);
  int ib = (int)(L / (unsigned)m.nyg);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  const bool adi = m.eos == FARGO_ADIABATIC;
  auto copy = [&](int k) {
    unsigned c = m.o32(i, j, k);
    vx2[c] = s.vx[c];
    vy2[c] = s.vy[c];
    if (m.d3) vz2[c] = s.vz[c];
    if (adi) e2[c] = s.e[c];
  };
  if (j < m.j0 || j >= m.jn) {
#pragma unroll 1
    for (int k = 0; k < m.nzg; k++) copy(k);
    return;
  }
#pragma unroll 1
  for (int k = 0; k < m.k0; k++) copy(k);
#pragma unroll 1
  for (int k = m.kn; k < m.nzg; k++) copy(k);
  const Src<F> S{m, s, (F)*dtp};
  const F dt = S.dt, c2 = (F)(m.cvnr * m.cvnr);
  if (!m.d3) {
    unsigned c = m.o32(i, j, 0);
    F heat, flux;
    xy_part(S, i, j, 0, c, vx2, vy2, heat, flux);
    if (adi) energy(S, j, 0, c, heat, flux, e2);
    return;
  }
  const int ip = i + 1 == m.nx ? 0 : i + 1;
  const bool per = m.zper();
  // plane p of the march, with periodic wrap over the active range if needed
  auto pl = [&](int p) { return per ? m.k0 + (p - m.k0 + 2 * m.nz) % m.nz : p; };
  auto load = [&](int p, Plane<F> &z) {
    unsigned c = m.o32(i, j, p);
    z.rho = s.rho[c];
    z.P = S.P(c);
    z.pot = s.pot[c];
    z.vz = s.vz[c];
    z.vx = s.vx[c];
    z.vxp = s.vx[c - i + ip];
  };
  // v'_z on face p (planes below(p) = zb and p = z0), v^n if not owned
  auto vz1 = [&](int p, const Plane<F> &zb, const Plane<F> &z0) {
    if (!S.zowned(p)) return z0.vz;
    F h = (F)m.hz(j, p);
    F gradP = F(2) * (z0.P - zb.P) / ((z0.rho + zb.rho) * h);
    F gradPhi = (z0.pot - zb.pot) / h;
    F src = F(0);
    if (m.geo == FARGO_SPHERICAL) {
      const F om = (F)m.omega;
      F R0 = (F)(m.g.ymed[j] * m.g.sinz[p]), R1 = (F)(m.g.ymed[j] * m.g.sinz[m.kbelow(p)]);
      F vt = F(0.25) * ((z0.vx + R0 * om) + (z0.vxp + R0 * om) + (zb.vx + R1 * om) + (zb.vxp + R1 * om));
      double zf = m.g.zmin[p];
      src = vt * vt * (F)(cos(zf) / sin(zf)) / (F)m.g.ymed[j];
    }
    return z0.vz - dt * (gradP + gradPhi) + dt * src;
  };
  // window: full records of the two newest planes (Pa = k+1, Pb = k+2), the
  // densities of planes k-1 .. k+2 (R[0..3]) and v^n_z on faces k, k+1;
  // v'_z on faces k-1 .. k+2 (A[0..3]); q_z in zones k-1 .. k+1 (Q[0..2])
  const int k = m.k0;
  Plane<F> Pa, Pb;
  F R[4], A[4], Q[3], V0, V1;
  load(pl(k - 2), Pa);
  load(pl(k - 1), Pb);
  A[0] = vz1(pl(k - 1), Pa, Pb);
  R[0] = Pb.rho;
  load(k, Pa);
  A[1] = vz1(k, Pb, Pa);
  R[1] = Pa.rho;
  V0 = Pa.vz;
  load(pl(k + 1), Pb);
  A[2] = vz1(pl(k + 1), Pa, Pb);
  R[2] = Pb.rho;
  V1 = Pb.vz;
  Q[0] = qvisc(c2, R[0], A[1] - A[0]);
  Q[1] = qvisc(c2, R[1], A[2] - A[1]);
  Pa = Pb; // plane k+1
#pragma unroll 1
  for (int kk = m.k0; kk < m.kn; kk++) {
    const int ka = pl(kk + 1), kaa = pl(kk + 2);
    load(kaa, Pb);
    A[3] = vz1(kaa, Pa, Pb);
    R[3] = Pb.rho;
    Q[2] = qvisc(c2, R[2], A[3] - A[2]);
    unsigned c = m.o32(i, j, kk);
    F heat, flux;
    xy_part(S, i, j, kk, c, vx2, vy2, heat, flux);
    F bz1 = V0, bz2 = V1;
    if (S.zowned(kk)) bz1 = A[1] - dt * F(2) * (Q[1] - Q[0]) / ((R[1] + R[0]) * (F)m.hz(j, kk));
    if (S.zowned(ka)) bz2 = A[2] - dt * F(2) * (Q[2] - Q[1]) / ((R[2] + R[1]) * (F)m.hz(j, ka));
    vz2[c] = bz1;
    heat += Q[1] * (A[2] - A[1]) / (F)m.Lz(j, kk);
    flux += (F)m.Sz(j, kk + 1) * bz2 - (F)m.Sz(j, kk) * bz1;
    if (adi) energy(S, j, kk, c, heat, flux, e2);
    R[0] = R[1];
    R[1] = R[2];
    R[2] = R[3];
    A[0] = A[1];
    A[1] = A[2];
    A[2] = A[3];
    Q[0] = Q[1];
    Q[1] = Q[2];
    V0 = V1;
    V1 = Pb.vz;
    Pa = Pb;
  }
}

} // namespace

template <typename F>
void launch_source(Launch &L, const Mesh &m, const StateT<F> &s, const double *dt, F *vx2, F *vy2, F *vz2, F *e2) {
  int nib, bs;
  row_blocks(m.nx, nib, bs);
  unsigned nb = (unsigned)nib * (unsigned)m.nyg;
  prof_begin(L, K_SRC);
  k_source<F><<<nb, bs, 0, L.s>>>(m, s, dt, vx2, vy2, vz2, e2);
  prof_end(L, K_SRC);
}

template void launch_source<double>(Launch &, const Mesh &, const StateT<double> &, const double *, double *, double *,
                                    double *, double *);
template void launch_source<float>(Launch &, const Mesh &, const StateT<float> &, const double *, float *, float *,
                                   float *, float *);

} // namespace fargo
