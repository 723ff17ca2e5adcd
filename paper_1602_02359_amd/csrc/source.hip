// Box 7: source step (Sect. 3.3).
//   7a  pressure and potential gradients on the owned faces, centrifugal
//       terms as squares of four-point arithmetic averages (Eq. 12 and its
//       generalisation); Jacobi: every face reads only v^n.  The pressure
//       term uses the arithmetic mean of the two face densities (Eq. 20),
//       which makes it momentum conserving (Eqs. 21-25).
//   7b  von Neumann-Richtmyer artificial viscosity, per direction:
//       q = C^2 rho dv^2 where dv < 0, its gradient in the same conservative
//       form, and the heating -q dv / L.
//   7c  compressional heating of a gamma-law gas, time-centred:
//       e <- e (1 - a)/(1 + a), a = dt (gamma - 1) div(v) / 2.
// One thread per active zone; a zone owns its lower X, Y and Z faces (the
// lower Y/Z boundary face only in a periodic direction).
#include "fargo_internal.h"

namespace fargo {

namespace {

__device__ inline double pressure(const Mesh &m, const StateP &s, size_t c) {
  return m.eos == FARGO_ISOTHERMAL ? s.cs[c] * s.cs[c] * s.rho[c] : (m.gamma - 1.0) * s.e[c];
}

__device__ inline void zone_of(const Mesh &m, long t, int &i, int &j, int &k) {
  i = (int)(t % m.nx);
  long r = t / m.nx;
  j = m.j0 + (int)(r % m.ny);
  k = m.k0 + (int)(r / m.ny);
}

// 7a: v' from v^n
__global__ __launch_bounds__(256) void k_src1(Mesh m, StateP s, const double *__restrict__ dtp,
                                              double *__restrict__ vx1, double *__restrict__ vy1,
                                              double *__restrict__ vz1) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)m.nx * m.ny * m.nz) return;
  int i, j, k;
  zone_of(m, t, i, j, k);
  const double dt = *dtp;
  const double om = m.omega;
  int im = i == 0 ? m.nx - 1 : i - 1, ip = i + 1 == m.nx ? 0 : i + 1;
  size_t c = m.idx(i, j, k);
  double Pc = pressure(m, s, c), rc = s.rho[c], phc = s.pot[c];
  {
    size_t cm = m.idx(im, j, k);
    double dX = m.DX(j, k);
    double gradP = 2.0 * (Pc - pressure(m, s, cm)) / ((rc + s.rho[cm]) * dX);
    double gradPhi = (phc - s.pot[cm]) / dX;
    vx1[c] = s.vx[c] - dt * (gradP + gradPhi);
  }
  if (j >= m.ylo()) {
    int jm = m.jbelow(j);
    size_t cm = m.idx(i, jm, k);
    double h = m.g.hy[j];
    double gradP = 2.0 * (Pc - pressure(m, s, cm)) / ((rc + s.rho[cm]) * h);
    double gradPhi = (phc - s.pot[cm]) / h;
    double src = 0.0;
    if (m.geo == FARGO_CYLINDRICAL) {
      double r0 = m.g.ymed[j], r1 = m.g.ymed[jm];
      double vt = 0.25 * ((s.vx[c] + r0 * om) + (s.vx[m.idx(ip, j, k)] + r0 * om) + (s.vx[cm] + r1 * om) +
                          (s.vx[m.idx(ip, jm, k)] + r1 * om));
      src = vt * vt / m.g.ymin[j];
    } else if (m.geo == FARGO_SPHERICAL) {
      double R0 = m.g.ymed[j] * m.g.sinz[k], R1 = m.g.ymed[jm] * m.g.sinz[k];
      double vt = 0.25 * ((s.vx[c] + R0 * om) + (s.vx[m.idx(ip, j, k)] + R0 * om) + (s.vx[cm] + R1 * om) +
                          (s.vx[m.idx(ip, jm, k)] + R1 * om));
      int kp = m.kabove(k);
      double vth = 0.25 * (s.vz[c] + s.vz[m.idx(i, j, kp)] + s.vz[cm] + s.vz[m.idx(i, jm, kp)]);
      src = (vt * vt + vth * vth) / m.g.ymin[j];
    }
    vy1[c] = s.vy[c] - dt * (gradP + gradPhi) + dt * src;
  } else {
    vy1[c] = s.vy[c];
  }
  if (!m.yper() && j == m.jn - 1) vy1[m.idx(i, m.jn, k)] = s.vy[m.idx(i, m.jn, k)];
  if (!m.d3) return;
  if (k >= m.zlo()) {
    int km = m.kbelow(k);
    size_t cm = m.idx(i, j, km);
    double h = m.hz(j, k);
    double gradP = 2.0 * (Pc - pressure(m, s, cm)) / ((rc + s.rho[cm]) * h);
    double gradPhi = (phc - s.pot[cm]) / h;
    double src = 0.0;
    if (m.geo == FARGO_SPHERICAL) {
      double R0 = m.g.ymed[j] * m.g.sinz[k], R1 = m.g.ymed[j] * m.g.sinz[km];
      double vt = 0.25 * ((s.vx[c] + R0 * om) + (s.vx[m.idx(ip, j, k)] + R0 * om) + (s.vx[cm] + R1 * om) +
                          (s.vx[m.idx(ip, j, km)] + R1 * om));
      double zf = m.g.zmin[k];
      src = vt * vt * (cos(zf) / sin(zf)) / m.g.ymed[j];
    }
    vz1[c] = s.vz[c] - dt * (gradP + gradPhi) + dt * src;
  } else {
    vz1[c] = s.vz[c];
  }
  if (!m.zper() && k == m.kn - 1) vz1[m.idx(i, j, m.kn)] = s.vz[m.idx(i, j, m.kn)];
}

__device__ inline double qvisc(double c2, double rho, double dv) { return dv < 0.0 ? c2 * rho * dv * dv : 0.0; }

// 7b: v'' (into the state) and e - dt * heating (adiabatic)
__global__ __launch_bounds__(256) void k_src2(Mesh m, StateP s, const double *__restrict__ dtp,
                                              const double *__restrict__ vx1, const double *__restrict__ vy1,
                                              const double *__restrict__ vz1) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)m.nx * m.ny * m.nz) return;
  int i, j, k;
  zone_of(m, t, i, j, k);
  const double dt = *dtp;
  const double c2 = m.cvnr * m.cvnr;
  int im = i == 0 ? m.nx - 1 : i - 1, ip = i + 1 == m.nx ? 0 : i + 1;
  size_t c = m.idx(i, j, k);
  double rc = s.rho[c];
  double dX = m.DX(j, k);
  // X
  double dvx = vx1[m.idx(ip, j, k)] - vx1[c];
  double qx = qvisc(c2, rc, dvx);
  {
    size_t cm = m.idx(im, j, k);
    double rm = s.rho[cm];
    double qm = qvisc(c2, rm, vx1[c] - vx1[cm]);
    s.vx[c] = vx1[c] - dt * 2.0 * (qx - qm) / ((rc + rm) * dX);
  }
  // Y
  double dvy = vy1[m.idx(i, m.jabove(j), k)] - vy1[c];
  double qy = qvisc(c2, rc, dvy);
  if (j >= m.ylo()) {
    int jm = m.jbelow(j);
    size_t cm = m.idx(i, jm, k);
    double rm = s.rho[cm];
    double qm = qvisc(c2, rm, vy1[c] - vy1[cm]);
    s.vy[c] = vy1[c] - dt * 2.0 * (qy - qm) / ((rc + rm) * m.g.hy[j]);
  }
  double heat = qx * dvx / dX + qy * dvy / m.g.Ly[j];
  if (m.d3) {
    double dvz = vz1[m.idx(i, j, m.kabove(k))] - vz1[c];
    double qz = qvisc(c2, rc, dvz);
    if (k >= m.zlo()) {
      int km = m.kbelow(k);
      size_t cm = m.idx(i, j, km);
      double rm = s.rho[cm];
      double qm = qvisc(c2, rm, vz1[c] - vz1[cm]);
      s.vz[c] = vz1[c] - dt * 2.0 * (qz - qm) / ((rc + rm) * m.hz(j, k));
    }
    heat += qz * dvz / m.Lz(j, k);
  }
  if (m.eos == FARGO_ADIABATIC) s.e[c] = s.e[c] - dt * heat;
}

// 7c: e'' from the divergence of v''
__global__ __launch_bounds__(256) void k_src3(Mesh m, StateP s, const double *__restrict__ dtp) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)m.nx * m.ny * m.nz) return;
  int i, j, k;
  zone_of(m, t, i, j, k);
  const double dt = *dtp;
  int ip = i + 1 == m.nx ? 0 : i + 1;
  size_t c = m.idx(i, j, k);
  double flux = m.Sx(j, k) * (s.vx[m.idx(ip, j, k)] - s.vx[c]) +
                (m.Sy(j + 1, k) * s.vy[m.idx(i, m.jabove(j), k)] - m.Sy(j, k) * s.vy[c]);
  if (m.d3) flux += m.Sz(j, k + 1) * s.vz[m.idx(i, j, m.kabove(k))] - m.Sz(j, k) * s.vz[c];
  double divv = m.Vinv(j, k) * flux;
  double a = 0.5 * dt * (m.gamma - 1.0) * divv;
  s.e[c] = s.e[c] * (1.0 - a) / (1.0 + a);
}

} // namespace

void launch_source(Launch &L, const Mesh &m, const StateP &s, const double *dt, double *vx1, double *vy1,
                   double *vz1) {
  long total = (long)m.nx * m.ny * m.nz;
  unsigned nb = (unsigned)((total + 255) / 256);
  prof_begin(L, K_SRC1);
  k_src1<<<nb, 256, 0, L.s>>>(m, s, dt, vx1, vy1, vz1);
  prof_end(L, K_SRC1);
  prof_begin(L, K_SRC2);
  k_src2<<<nb, 256, 0, L.s>>>(m, s, dt, vx1, vy1, vz1);
  prof_end(L, K_SRC2);
  if (m.eos == FARGO_ADIABATIC) {
    prof_begin(L, K_SRC3);
    k_src3<<<nb, 256, 0, L.s>>>(m, s, dt);
    prof_end(L, K_SRC3);
  }
}

} // namespace fargo
