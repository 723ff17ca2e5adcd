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
// One thread per zone of the whole mesh.  A zone owns its lower X, Y and Z
// faces (the lower Y/Z boundary face only in a periodic direction).  Active
// zones recompute the few intermediate face values their stencil needs
// (v' on four faces and q in three zones per direction) instead of storing
// them; ghost zones copy v^n and e.  Results go to separate arrays (v'', e''),
// so the pass reads the state while it writes.
#include "fargo_internal.h"

namespace fargo {

namespace {

struct Src {
  Mesh m;
  StateP s;
  double dt;

  __device__ inline double P(size_t c) const {
    return m.eos == FARGO_ISOTHERMAL ? s.cs[c] * s.cs[c] * s.rho[c] : (m.gamma - 1.0) * s.e[c];
  }
  // 7a on X face ii of row (j, k)
  __device__ inline double vx1(int ii, int j, int k) const {
    int im = ii == 0 ? m.nx - 1 : ii - 1;
    size_t c = m.idx(ii, j, k), cm = m.idx(im, j, k);
    double dX = m.DX(j, k);
    double gradP = 2.0 * (P(c) - P(cm)) / ((s.rho[c] + s.rho[cm]) * dX);
    double gradPhi = (s.pot[c] - s.pot[cm]) / dX;
    return s.vx[c] - dt * (gradP + gradPhi);
  }
  __device__ inline bool yowned(int jj) const { return jj >= m.ylo() && jj < m.jn; }
  __device__ inline bool zowned(int kk) const { return kk >= m.zlo() && kk < m.kn; }
  // 7a on Y face jj of column (i, k); v^n if the face is not owned
  __device__ inline double vy1(int i, int jj, int k) const {
    size_t c = m.idx(i, jj, k);
    if (!yowned(jj)) return s.vy[c];
    int jm = m.jbelow(jj);
    int ip = i + 1 == m.nx ? 0 : i + 1;
    size_t cm = m.idx(i, jm, k);
    double h = m.g.hy[jj];
    double gradP = 2.0 * (P(c) - P(cm)) / ((s.rho[c] + s.rho[cm]) * h);
    double gradPhi = (s.pot[c] - s.pot[cm]) / h;
    double src = 0.0;
    const double om = m.omega;
    if (m.geo == FARGO_CYLINDRICAL) {
      double r0 = m.g.ymed[jj], r1 = m.g.ymed[jm];
      double vt = 0.25 * ((s.vx[c] + r0 * om) + (s.vx[m.idx(ip, jj, k)] + r0 * om) + (s.vx[cm] + r1 * om) +
                          (s.vx[m.idx(ip, jm, k)] + r1 * om));
      src = vt * vt / m.g.ymin[jj];
    } else if (m.geo == FARGO_SPHERICAL) {
      double R0 = m.g.ymed[jj] * m.g.sinz[k], R1 = m.g.ymed[jm] * m.g.sinz[k];
      double vt = 0.25 * ((s.vx[c] + R0 * om) + (s.vx[m.idx(ip, jj, k)] + R0 * om) + (s.vx[cm] + R1 * om) +
                          (s.vx[m.idx(ip, jm, k)] + R1 * om));
      int kp = m.kabove(k);
      double vth = 0.25 * (s.vz[c] + s.vz[m.idx(i, jj, kp)] + s.vz[cm] + s.vz[m.idx(i, jm, kp)]);
      src = (vt * vt + vth * vth) / m.g.ymin[jj];
    }
    return s.vy[c] - dt * (gradP + gradPhi) + dt * src;
  }
  // 7a on Z face kk of column (i, j); v^n if the face is not owned
  __device__ inline double vz1(int i, int j, int kk) const {
    size_t c = m.idx(i, j, kk);
    if (!zowned(kk)) return s.vz[c];
    int km = m.kbelow(kk);
    size_t cm = m.idx(i, j, km);
    double h = m.hz(j, kk);
    double gradP = 2.0 * (P(c) - P(cm)) / ((s.rho[c] + s.rho[cm]) * h);
    double gradPhi = (s.pot[c] - s.pot[cm]) / h;
    double src = 0.0;
    if (m.geo == FARGO_SPHERICAL) {
      const double om = m.omega;
      int ip = i + 1 == m.nx ? 0 : i + 1;
      double R0 = m.g.ymed[j] * m.g.sinz[kk], R1 = m.g.ymed[j] * m.g.sinz[km];
      double vt = 0.25 * ((s.vx[c] + R0 * om) + (s.vx[m.idx(ip, j, kk)] + R0 * om) + (s.vx[cm] + R1 * om) +
                          (s.vx[m.idx(ip, j, km)] + R1 * om));
      double zf = m.g.zmin[kk];
      src = vt * vt * (cos(zf) / sin(zf)) / m.g.ymed[j];
    }
    return s.vz[c] - dt * (gradP + gradPhi) + dt * src;
  }
};

__device__ inline double qvisc(double c2, double rho, double dv) { return dv < 0.0 ? c2 * rho * dv * dv : 0.0; }

// Grid: blocks of `bs` threads along X; logical block = (k fastest, then j,
// then the X block), dispatched XCD-contiguously so that the neighbouring
// rows and planes a zone reads are being read by blocks on the same XCD.
__global__ __launch_bounds__(256) void k_source(Mesh m, StateP s, const double *__restrict__ dtp,
                                                double *__restrict__ vx2, double *__restrict__ vy2,
                                                double *__restrict__ vz2, double *__restrict__ e2) {
  unsigned L = xcd_remap(blockIdx.x, gridDim.x);
  int k = (int)(L % (unsigned)m.nzg);
  unsigned r = L / (unsigned)m.nzg;
  int j = (int)(r % (unsigned)m.nyg);
  int ib = (int)(r / (unsigned)m.nyg);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  size_t c = m.idx(i, j, k);
  bool act = j >= m.j0 && j < m.jn && k >= m.k0 && k < m.kn;
  if (!act) {
    vx2[c] = s.vx[c];
    vy2[c] = s.vy[c];
    if (m.d3) vz2[c] = s.vz[c];
    if (e2) e2[c] = s.e[c];
    return;
  }
  const Src S{m, s, *dtp};
  const double dt = S.dt;
  const double c2 = m.cvnr * m.cvnr;
  const double rc = s.rho[c];
  // ---- X: faces i-1, i, i+1, i+2; zones i-1, i, i+1
  int im = i == 0 ? m.nx - 1 : i - 1;
  int ip = i + 1 == m.nx ? 0 : i + 1;
  int ip2 = ip + 1 == m.nx ? 0 : ip + 1;
  double dX = m.DX(j, k);
  double ax0 = S.vx1(im, j, k), ax1 = S.vx1(i, j, k), ax2 = S.vx1(ip, j, k), ax3 = S.vx1(ip2, j, k);
  double rxm = s.rho[m.idx(im, j, k)], rxp = s.rho[m.idx(ip, j, k)];
  double dvx = ax2 - ax1;
  double qx = qvisc(c2, rc, dvx);
  double qxm = qvisc(c2, rxm, ax1 - ax0), qxp = qvisc(c2, rxp, ax3 - ax2);
  double bx1 = ax1 - dt * 2.0 * (qx - qxm) / ((rc + rxm) * dX);
  double bx2 = ax2 - dt * 2.0 * (qxp - qx) / ((rxp + rc) * dX);
  vx2[c] = bx1;
  // ---- Y: zones jb, j, ja; faces jb, j, ja, above(ja)
  int jb = m.jbelow(j), ja = m.jabove(j);
  double ay1 = S.vy1(i, j, k), ay2 = S.vy1(i, ja, k);
  double dvy = ay2 - ay1;
  double qy = qvisc(c2, rc, dvy);
  double by1 = s.vy[c], by2 = s.vy[m.idx(i, ja, k)];
  if (S.yowned(j)) {
    double ay0 = S.vy1(i, jb, k);
    double rb = s.rho[m.idx(i, jb, k)];
    double qb = qvisc(c2, rb, ay1 - ay0);
    by1 = ay1 - dt * 2.0 * (qy - qb) / ((rc + rb) * m.g.hy[j]);
  }
  if (S.yowned(ja)) {
    double ay3 = S.vy1(i, m.jabove(ja), k);
    double ra = s.rho[m.idx(i, ja, k)];
    double qa = qvisc(c2, ra, ay3 - ay2);
    by2 = ay2 - dt * 2.0 * (qa - qy) / ((ra + rc) * m.g.hy[ja]);
  }
  vy2[c] = by1;
  double heat = qx * dvx / dX + qy * dvy / m.g.Ly[j];
  double flux = m.Sx(j, k) * (bx2 - bx1) + (m.Sy(j + 1, k) * by2 - m.Sy(j, k) * by1);
  // ---- Z
  if (m.d3) {
    int kb = m.kbelow(k), ka = m.kabove(k);
    double az1 = S.vz1(i, j, k), az2 = S.vz1(i, j, ka);
    double dvz = az2 - az1;
    double qz = qvisc(c2, rc, dvz);
    double bz1 = s.vz[c], bz2 = s.vz[m.idx(i, j, ka)];
    if (S.zowned(k)) {
      double az0 = S.vz1(i, j, kb);
      double rb = s.rho[m.idx(i, j, kb)];
      double qb = qvisc(c2, rb, az1 - az0);
      bz1 = az1 - dt * 2.0 * (qz - qb) / ((rc + rb) * m.hz(j, k));
    }
    if (S.zowned(ka)) {
      double az3 = S.vz1(i, j, m.kabove(ka));
      double ra = s.rho[m.idx(i, j, ka)];
      double qa = qvisc(c2, ra, az3 - az2);
      bz2 = az2 - dt * 2.0 * (qa - qz) / ((ra + rc) * m.hz(j, ka));
    }
    vz2[c] = bz1;
    heat += qz * dvz / m.Lz(j, k);
    flux += m.Sz(j, k + 1) * bz2 - m.Sz(j, k) * bz1;
  }
  if (m.eos == FARGO_ADIABATIC) {
    double e1 = s.e[c] - dt * heat;
    double a = 0.5 * dt * (m.gamma - 1.0) * (m.Vinv(j, k) * flux);
    e2[c] = e1 * (1.0 - a) / (1.0 + a);
  }
}

} // namespace

void launch_source(Launch &L, const Mesh &m, const StateP &s, const double *dt, double *vx2, double *vy2,
                   double *vz2, double *e2) {
  int nib, bs;
  row_blocks(m.nx, nib, bs);
  unsigned nb = (unsigned)nib * (unsigned)m.nyg * (unsigned)m.nzg;
  prof_begin(L, K_SRC);
  k_source<<<nb, bs, 0, L.s>>>(m, s, dt, vx2, vy2, vz2, e2);
  prof_end(L, K_SRC);
}

} // namespace fargo
