// Box 12: transport (Sect. 3.4, 3.5.1).
//   12a  left/right momenta Pi- = rho m(v_{i-1/2}), Pi+ = rho m(v_{i+1/2})
//        with the factors m of Tab. "momenta" (Eqs. 16, 17), in every zone
//        whose faces exist (ghosts included).
//   12b/c directional finite-volume updates, in the order Y, Z, X:
//        van Leer slopes (harmonic mean of one-sided differences per unit
//        length, zero unless of equal sign), interface value at half step
//        upwinded on the face velocity (Eqs. 14, 15), mass flux w rho* S dt
//        (Eq. flux), consistent transport (Q/rho interpolated, flux q* F_rho).
//        The Y sweep also runs on the two nearest ghost rows of each Z side,
//        which the Z sweep reads next.  The X sweep of each ring uses the
//        residual velocity v_x - v0 (Eq. fargo1) and is followed by the
//        circular shift by N zones (Eq. 32) and the PPA fractional residual
//        (Eqs. 33-36); both act identically on every zone of a ring, so the
//        shift is applied when the ring is stored.
//   12d  velocities from the transported momenta (Eq. 18).
#include "fargo_internal.h"

namespace fargo {

namespace {

__device__ inline double vanleer(double qm, double q0, double qp, double hm, double hp) {
  double dl = (q0 - qm) / hm, dr = (qp - q0) / hp;
  double pr = dl * dr;
  return pr > 0.0 ? 2.0 * pr / (dl + dr) : 0.0;
}

// ------------------------------------------------------------------------
// 12a
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_momenta(Mesh m, StateP s, TSet T) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)m.nx * m.nyg * m.nzg) return;
  int i = (int)(t % m.nx);
  long r = t / m.nx;
  int j = (int)(r % m.nyg), k = (int)(r / m.nyg);
  int ip = i + 1 == m.nx ? 0 : i + 1;
  size_t c = m.idx(i, j, k);
  double rho = s.rho[c];
  T.a[T_RHO][c] = rho;
  T.a[T_PXM][c] = rho * m.mx(j, k, s.vx[c]);
  T.a[T_PXP][c] = rho * m.mx(j, k, s.vx[m.idx(ip, j, k)]);
  T.a[T_PYM][c] = rho * s.vy[c];
  T.a[T_PYP][c] = j + 1 < m.nyg ? rho * s.vy[m.idx(i, j + 1, k)] : 0.0;
  if (m.d3) {
    T.a[T_PZM][c] = rho * m.mz(j, s.vz[c]);
    T.a[T_PZP][c] = k + 1 < m.nzg ? rho * m.mz(j, s.vz[m.idx(i, j, k + 1)]) : 0.0;
  }
  if (s.e) T.a[T_E][c] = s.e[c];
}

// ------------------------------------------------------------------------
// 12b/c along Y (DIR = 1) or Z (DIR = 2): one thread per zone, both faces of
// the zone evaluated from the five zones around it.
// ------------------------------------------------------------------------
template <int DIR>
__global__ __launch_bounds__(256) void k_sweep(Mesh m, const double *__restrict__ w, TSet in, TSet out,
                                               const double *__restrict__ dtp, int kbase, int nrows) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)m.nx * m.ny * nrows) return;
  int i = (int)(t % m.nx);
  long r = t / m.nx;
  int j = m.j0 + (int)(r % m.ny), k = kbase + (int)(r / m.ny);
  const double dt = *dtp;
  const size_t c = m.idx(i, j, k);
  const size_t st = DIR == 1 ? (size_t)m.pitch : m.plane();
  const int a = DIR == 1 ? j : k;
  double L[3], h[4];
  for (int d = 0; d < 3; d++) L[d] = DIR == 1 ? m.g.Ly[a - 1 + d] : m.Lz(j, a - 1 + d);
  for (int d = 0; d < 4; d++) h[d] = DIR == 1 ? m.g.hy[a - 1 + d] : m.hz(j, a - 1 + d);
  double S0 = DIR == 1 ? m.Sy(a, k) : m.Sz(j, a);
  double S1 = DIR == 1 ? m.Sy(a + 1, k) : m.Sz(j, a + 1);
  double vinv = m.Vinv(j, k);
  double w0 = w[c], w1 = w[c + st];
  const double *R = in.a[T_RHO];
  double r5[5];
  for (int d = 0; d < 5; d++) r5[d] = R[c + (long)(d - 2) * (long)st];
  double s3[3];
  for (int d = 0; d < 3; d++) s3[d] = vanleer(r5[d], r5[d + 1], r5[d + 2], h[d], h[d + 1]);
  double st0 = w0 >= 0.0 ? r5[1] + s3[0] * (L[0] - w0 * dt) * 0.5 : r5[2] - s3[1] * (L[1] + w0 * dt) * 0.5;
  double st1 = w1 >= 0.0 ? r5[2] + s3[1] * (L[1] - w1 * dt) * 0.5 : r5[3] - s3[2] * (L[2] + w1 * dt) * 0.5;
  double F0 = w0 * st0 * S0 * dt, F1 = w1 * st1 * S1 * dt;
  out.a[T_RHO][c] = r5[2] - vinv * (F1 - F0);
  for (int q = 0; q < in.nq; q++) {
    const double *Q = in.q[q];
    double q5[5];
    for (int d = 0; d < 5; d++) q5[d] = Q[c + (long)(d - 2) * (long)st] / r5[d];
    for (int d = 0; d < 3; d++) s3[d] = vanleer(q5[d], q5[d + 1], q5[d + 2], h[d], h[d + 1]);
    double a0 = w0 >= 0.0 ? q5[1] + s3[0] * (L[0] - w0 * dt) * 0.5 : q5[2] - s3[1] * (L[1] + w0 * dt) * 0.5;
    double a1 = w1 >= 0.0 ? q5[2] + s3[1] * (L[1] - w1 * dt) * 0.5 : q5[3] - s3[2] * (L[2] + w1 * dt) * 0.5;
    out.q[q][c] = Q[c] - vinv * (a1 * F1 - a0 * F0);
  }
}

// ------------------------------------------------------------------------
// 12c along X with orbital advection: one workgroup per ring, M zones per
// thread (zone i = tid + 256 m), LDS for neighbour exchange.
// ------------------------------------------------------------------------
__device__ inline double mc_slope(double qm, double q0, double qp) {
  double dq = 0.5 * (qp - qm);
  if ((qp - q0) * (q0 - qm) <= 0.0) return 0.0;
  double mag = fmin(fmin(2.0 * fabs(q0 - qm), 2.0 * fabs(qp - q0)), fabs(dq));
  return dq > 0.0 ? mag : -mag;
}

// PPA interface value supplied by zone i for xi >= 0 (its right face) or
// xi < 0 (its left face): Eqs. 35, 36 and the interface formula with |xi|.
__device__ inline double ppa_star(double qm, double q0, double qp, double dmm, double dm0, double dmp, double xi) {
  double l = qm + 0.5 * (q0 - qm) - (dm0 - dmm) / 6.0;
  double r = q0 + 0.5 * (qp - q0) - (dmp - dm0) / 6.0;
  double D = r - l, C = q0 - 0.5 * (l + r);
  if ((qp - q0) * (q0 - qm) <= 0.0) {
    l = q0;
    r = q0;
  } else if (D * C > D * D / 6.0) {
    l = 3.0 * q0 - 2.0 * r;
  } else if (-D * D / 6.0 > D * C) {
    r = 3.0 * q0 - 2.0 * l;
  }
  double x = fabs(xi);
  if (xi >= 0.0) return r + x * (q0 - r) + x * (1.0 - x) * (2.0 * q0 - r - l);
  return l + x * (q0 - l) + x * (1.0 - x) * (2.0 * q0 - r - l);
}

template <int M>
__global__ __launch_bounds__(256) void k_ring_x(Mesh m, const double *__restrict__ vx, TSet T,
                                                const double *__restrict__ v0, const int32_t *__restrict__ Nsh,
                                                const double *__restrict__ xis, const double *__restrict__ dtp) {
  extern __shared__ double lds[];
  const int n = m.nx;
  double *B = lds, *A = lds + n, *D = lds + 2 * n, *E = lds + 3 * n;
  const int r = blockIdx.x;
  const int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  const int tid = threadIdx.x;
  const double dt = *dtp;
  const double dX = m.DX(j, k), S = m.Sx(j, k), vinv = m.Vinv(j, k);
  const double vb = m.fargo ? v0[r] : 0.0;
  const int N = m.fargo ? Nsh[r] : 0;
  const double xi = m.fargo ? xis[r] : 0.0;
  const size_t base = m.idx(0, j, k);
  double r0[M], r1[M], r2[M], fr[M], wv[M];
#define FOR_ZONES(...)                                 \
  _Pragma("unroll") for (int mm = 0; mm < M; mm++) {   \
    int i = tid + 256 * mm;                            \
    if (i < n) {                                       \
      int im = i == 0 ? n - 1 : i - 1;                 \
      int ip = i + 1 == n ? 0 : i + 1;                 \
      (void)im;                                        \
      (void)ip;                                        \
      __VA_ARGS__                                      \
    }                                                  \
  }
  FOR_ZONES(r0[mm] = T.a[T_RHO][base + i]; B[i] = r0[mm]; wv[mm] = vx[base + i] - vb;)
  __syncthreads();
  FOR_ZONES(A[i] = vanleer(B[im], B[i], B[ip], dX, dX);)
  __syncthreads();
  FOR_ZONES(double w = wv[mm];
            double st = w >= 0.0 ? B[im] + A[im] * (dX - w * dt) * 0.5 : B[i] - A[i] * (dX + w * dt) * 0.5;
            fr[mm] = w * st * S * dt; D[i] = fr[mm];)
  __syncthreads();
  FOR_ZONES(r1[mm] = r0[mm] - vinv * (D[ip] - D[i]);)
  __syncthreads();
  if (m.fargo) {
    FOR_ZONES(B[i] = r1[mm];)
    __syncthreads();
    FOR_ZONES(A[i] = mc_slope(B[im], B[i], B[ip]);)
    __syncthreads();
    FOR_ZONES(double st = ppa_star(B[im], B[i], B[ip], A[im], A[i], A[ip], xi);
              E[xi >= 0.0 ? ip : i] = xi * dX * S * st;)
    __syncthreads();
    FOR_ZONES(r2[mm] = r1[mm] - vinv * (E[ip] - E[i]);)
    __syncthreads();
  }
  for (int q = 0; q < T.nq; q++) {
    double *Q = T.q[q] + base;
    double qv[M];
    FOR_ZONES(qv[mm] = Q[i]; B[i] = qv[mm] / r0[mm];)
    __syncthreads();
    FOR_ZONES(A[i] = vanleer(B[im], B[i], B[ip], dX, dX);)
    __syncthreads();
    FOR_ZONES(double w = wv[mm];
              double st = w >= 0.0 ? B[im] + A[im] * (dX - w * dt) * 0.5 : B[i] - A[i] * (dX + w * dt) * 0.5;
              D[i] = st * fr[mm];)
    __syncthreads();
    FOR_ZONES(qv[mm] = qv[mm] - vinv * (D[ip] - D[i]);)
    __syncthreads();
    if (m.fargo) {
      FOR_ZONES(B[i] = qv[mm] / r1[mm];)
      __syncthreads();
      FOR_ZONES(A[i] = mc_slope(B[im], B[i], B[ip]);)
      __syncthreads();
      FOR_ZONES(double st = ppa_star(B[im], B[i], B[ip], A[im], A[i], A[ip], xi);
                int f = xi >= 0.0 ? ip : i;
                D[f] = st * E[f];)
      __syncthreads();
      FOR_ZONES(qv[mm] = qv[mm] - vinv * (D[ip] - D[i]);)
    }
    FOR_ZONES(int o = i + N; o %= n; if (o < 0) o += n; Q[o] = qv[mm];)
    __syncthreads();
  }
  FOR_ZONES(int o = i + N; o %= n; if (o < 0) o += n; T.a[T_RHO][base + o] = m.fargo ? r2[mm] : r1[mm];)
#undef FOR_ZONES
}

// ------------------------------------------------------------------------
// 12d
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vel(Mesh m, StateP s, TSet T) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)m.nx * m.ny * m.nz) return;
  int i = (int)(t % m.nx);
  long r = t / m.nx;
  int j = m.j0 + (int)(r % m.ny), k = m.k0 + (int)(r / m.ny);
  int im = i == 0 ? m.nx - 1 : i - 1;
  size_t c = m.idx(i, j, k);
  const double *R = T.a[T_RHO];
  {
    size_t cm = m.idx(im, j, k);
    double mom = (T.a[T_PXP][cm] + T.a[T_PXM][c]) / (R[cm] + R[c]);
    s.vx[c] = m.vx_from(j, k, mom);
  }
  if (j >= m.ylo()) {
    size_t cm = m.idx(i, m.jbelow(j), k);
    s.vy[c] = (T.a[T_PYP][cm] + T.a[T_PYM][c]) / (R[cm] + R[c]);
  }
  if (m.d3 && k >= m.zlo()) {
    size_t cm = m.idx(i, j, m.kbelow(k));
    double v = (T.a[T_PZP][cm] + T.a[T_PZM][c]) / (R[cm] + R[c]);
    s.vz[c] = m.geo == FARGO_SPHERICAL ? v / m.g.ymed[j] : v;
  }
  s.rho[c] = R[c];
  if (s.e) s.e[c] = T.a[T_E][c];
}

} // namespace

void launch_momenta(Launch &L, const Mesh &m, const StateP &s, const TSet &T) {
  long total = (long)m.nx * m.nyg * m.nzg;
  prof_begin(L, K_MOMENTA);
  k_momenta<<<(unsigned)((total + 255) / 256), 256, 0, L.s>>>(m, s, T);
  prof_end(L, K_MOMENTA);
}

void launch_sweep_y(Launch &L, const Mesh &m, const double *vy, const TSet &in, const TSet &out, const double *dt) {
  int kbase = m.d3 ? m.k0 - 2 : 0, nrows = m.d3 ? m.nz + 4 : 1;
  long total = (long)m.nx * m.ny * nrows;
  prof_begin(L, K_SWEEP_Y);
  k_sweep<1><<<(unsigned)((total + 255) / 256), 256, 0, L.s>>>(m, vy, in, out, dt, kbase, nrows);
  prof_end(L, K_SWEEP_Y);
}

void launch_sweep_z(Launch &L, const Mesh &m, const double *vz, const TSet &in, const TSet &out, const double *dt) {
  long total = (long)m.nx * m.ny * m.nz;
  prof_begin(L, K_SWEEP_Z);
  k_sweep<2><<<(unsigned)((total + 255) / 256), 256, 0, L.s>>>(m, vz, in, out, dt, m.k0, m.nz);
  prof_end(L, K_SWEEP_Z);
}

void launch_ring_x(Launch &L, const Mesh &m, const double *vx, const TSet &T, const double *v0, const int32_t *N,
                   const double *xi, const double *dt) {
  size_t lds = 4 * (size_t)m.nx * sizeof(double);
  prof_begin(L, K_RING_X);
  if (m.nx <= 256)
    k_ring_x<1><<<m.nring, 256, lds, L.s>>>(m, vx, T, v0, N, xi, dt);
  else if (m.nx <= 512)
    k_ring_x<2><<<m.nring, 256, lds, L.s>>>(m, vx, T, v0, N, xi, dt);
  else if (m.nx <= 1024)
    k_ring_x<4><<<m.nring, 256, lds, L.s>>>(m, vx, T, v0, N, xi, dt);
  else
    k_ring_x<8><<<m.nring, 256, lds, L.s>>>(m, vx, T, v0, N, xi, dt);
  prof_end(L, K_RING_X);
}

void launch_vel(Launch &L, const Mesh &m, const StateP &s, const TSet &T) {
  long total = (long)m.nx * m.ny * m.nz;
  prof_begin(L, K_VEL);
  k_vel<<<(unsigned)((total + 255) / 256), 256, 0, L.s>>>(m, s, T);
  prof_end(L, K_VEL);
}

} // namespace fargo
