// Box 12: transport (Sect. 3.4, 3.5.1).
//   12a  left/right momenta Pi- = rho m(v_{i-1/2}), Pi+ = rho m(v_{i+1/2})
//        with the factors m of Tab. "momenta" (Eqs. 16, 17).  They are formed
//        on the fly by the Y sweep, which reads the state directly.
//   12b/c directional finite-volume updates in the order Y, Z, X: van Leer
//        slopes (harmonic mean of the one-sided differences per unit length,
//        zero unless of equal sign), interface value at half step upwinded on
//        the face velocity (Eqs. 14, 15), mass flux w rho* S dt (Eq. flux),
//        consistent transport (Q/rho interpolated, flux q* F_rho).  The Y
//        sweep also covers the two nearest ghost rows of each Z side, which
//        the Z sweep reads next.  The X sweep of each ring uses the residual
//        velocity v_x - v0 (Eq. fargo1); it is followed by the circular shift
//        by N zones (Eq. 32) and the PPA fractional residual (Eqs. 33-36);
//        both act identically on every zone of a ring, so the shift is applied
//        when the ring is stored.
//   12d  velocities from the transported momenta (Eq. 18): v_x by the ring
//        kernel, v_y and v_z by a final pass.
//
// Y and Z sweeps are column sweeps: a thread walks a chunk of one column with
// a sliding window of three zones in registers, so that every value is loaded
// once and every face flux and slope is computed once.
#include "fargo_internal.h"

namespace fargo {

namespace {

constexpr int CHUNK = 64; // zones per thread along the sweep direction

// van Leer slope per unit length from the one-sided differences and the
// centre distances below (hm) and above (hp): 2 dl dr/(dl + dr) with
// dl = dm/hm, dr = dp/hp, zero unless dl dr > 0.
__device__ inline double vl_slope(double qm, double q0, double qp, double hm, double hp) {
  double dm = q0 - qm, dp = qp - q0;
  double pr = dm * dp;
  return pr > 0.0 ? 2.0 * pr / (dm * hp + dp * hm) : 0.0;
}

// half-step interface value at a face, upwinded on w (Eq. 15)
__device__ inline double vl_star(double w, double dt, double ql, double al, double Ll, double qr, double ar,
                                 double Lr) {
  return w >= 0.0 ? ql + al * (Ll - w * dt) * 0.5 : qr - ar * (Lr + w * dt) * 0.5;
}

template <int NQ>
struct Zone {
  double rho, q[NQ], T[NQ]; // density, Q/rho, conserved Q
};

// Column sweep over zones [a0, a1) of one column; `ld(a, Zone&)` loads zone a,
// `geo` gives L(a) (zone width), h(f) (centre distance at face f), S(f),
// Vi(a), w(f); `st(a, rho, T[])` stores the updated zone.
template <int NQ, class LD, class GEO, class ST>
__device__ inline void column_sweep(int a0, int a1, double dt, const LD &ld, const GEO &geo, const ST &st) {
  Zone<NQ> zm, z0, zp;
  ld(a0 - 2, zp); // used only for the first slope
  ld(a0 - 1, zm);
  ld(a0, z0);
  double sm[NQ + 1], s0[NQ + 1];
  {
    double hm = geo.h(a0 - 1), hp = geo.h(a0);
    sm[NQ] = vl_slope(zp.rho, zm.rho, z0.rho, hm, hp);
#pragma unroll
    for (int q = 0; q < NQ; q++) sm[q] = vl_slope(zp.q[q], zm.q[q], z0.q[q], hm, hp);
  }
  double Fp = 0.0, FQp[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) FQp[q] = 0.0;
  double Lm = geo.L(a0 - 1);
  for (int f = a0; f <= a1; f++) {
    ld(f + 1, zp);
    double hm = geo.h(f), hp = geo.h(f + 1);
    s0[NQ] = vl_slope(zm.rho, z0.rho, zp.rho, hm, hp);
#pragma unroll
    for (int q = 0; q < NQ; q++) s0[q] = vl_slope(zm.q[q], z0.q[q], zp.q[q], hm, hp);
    double L0 = geo.L(f);
    double w = geo.w(f);
    double F = w * vl_star(w, dt, zm.rho, sm[NQ], Lm, z0.rho, s0[NQ], L0) * geo.S(f) * dt;
    double FQ[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) FQ[q] = vl_star(w, dt, zm.q[q], sm[q], Lm, z0.q[q], s0[q], L0) * F;
    if (f > a0) {
      double vi = geo.Vi(f - 1);
      double Tn[NQ];
#pragma unroll
      for (int q = 0; q < NQ; q++) Tn[q] = zm.T[q] - vi * (FQ[q] - FQp[q]);
      st(f - 1, zm.rho - vi * (F - Fp), Tn);
    }
    Fp = F;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      FQp[q] = FQ[q];
      sm[q] = s0[q];
    }
    sm[NQ] = s0[NQ];
    zm = z0;
    z0 = zp;
    Lm = L0;
  }
}

// ------------------------------------------------------------------------
// Y sweep, forming the momenta from the post-source state (box 12a fused).
// Quantities: Pi-_x, Pi+_x, Pi-_y, Pi+_y [, Pi-_z, Pi+_z] [, e].
// ------------------------------------------------------------------------
template <int NQ, bool D3, bool ADI>
__global__ __launch_bounds__(256) void k_sweep_y(Mesh m, const double *__restrict__ rho,
                                                 const double *__restrict__ vx, const double *__restrict__ vy,
                                                 const double *__restrict__ vz, const double *__restrict__ e,
                                                 TSet out, const double *__restrict__ dtp, int nchunk) {
  const int nrows = D3 ? m.nz + 4 : 1, kbase = D3 ? m.k0 - 2 : 0;
  unsigned Lb = xcd_remap(blockIdx.x, gridDim.x);
  int kr = (int)(Lb % (unsigned)nrows);
  unsigned rest = Lb / (unsigned)nrows;
  int ch = (int)(rest % (unsigned)nchunk), ib = (int)(rest / (unsigned)nchunk);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  const int k = kbase + kr;
  const int a0 = m.j0 + ch * CHUNK, a1 = min(a0 + CHUNK, m.jn);
  const double dt = *dtp;
  const int ip = i + 1 == m.nx ? 0 : i + 1;
  const size_t pitch = m.pitch, plane = m.plane();
  auto ld = [&](int a, Zone<NQ> &z) {
    size_t c = m.idx(i, a, k);
    double r = rho[c];
    z.rho = r;
    z.q[0] = m.mx(a, k, vx[c]);
    z.q[1] = m.mx(a, k, vx[c - i + ip]);
    z.q[2] = vy[c];
    z.q[3] = vy[c + pitch];
    if (D3) {
      z.q[4] = m.mz(a, vz[c]);
      z.q[5] = m.mz(a, vz[c + plane]);
    }
#pragma unroll
    for (int q = 0; q < (ADI ? NQ - 1 : NQ); q++) z.T[q] = r * z.q[q];
    if (ADI) {
      z.T[NQ - 1] = e[c];
      z.q[NQ - 1] = e[c] / r;
    }
  };
  struct Geo {
    const Mesh &m;
    const double *vy;
    size_t base;
    int k;
    __device__ double L(int a) const { return m.g.Ly[a]; }
    __device__ double h(int f) const { return m.g.hy[f]; }
    __device__ double S(int f) const { return m.Sy(f, k); }
    __device__ double Vi(int a) const { return m.Vinv(a, k); }
    __device__ double w(int f) const { return vy[base + (size_t)f * m.pitch]; }
  } geo{m, vy, m.idx(i, 0, k), k};
  auto st = [&](int a, double r, const double (&T)[NQ]) {
    size_t c = m.idx(i, a, k);
    out.a[T_RHO][c] = r;
#pragma unroll
    for (int q = 0; q < NQ; q++) out.q[q][c] = T[q];
  };
  column_sweep<NQ>(a0, a1, dt, ld, geo, st);
}

// ------------------------------------------------------------------------
// Z sweep on the Y-swept quantities.
// ------------------------------------------------------------------------
template <int NQ>
__global__ __launch_bounds__(256) void k_sweep_z(Mesh m, const double *__restrict__ vz, TSet in, TSet out,
                                                 const double *__restrict__ dtp, int nchunk) {
  unsigned Lb = xcd_remap(blockIdx.x, gridDim.x);
  int jr = (int)(Lb % (unsigned)m.ny);
  unsigned rest = Lb / (unsigned)m.ny;
  int ch = (int)(rest % (unsigned)nchunk), ib = (int)(rest / (unsigned)nchunk);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  const int j = m.j0 + jr;
  const int a0 = m.k0 + ch * CHUNK, a1 = min(a0 + CHUNK, m.kn);
  const double dt = *dtp;
  auto ld = [&](int a, Zone<NQ> &z) {
    size_t c = m.idx(i, j, a);
    double r = in.a[T_RHO][c];
    double ri = 1.0 / r;
    z.rho = r;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      z.T[q] = in.q[q][c];
      z.q[q] = z.T[q] * ri;
    }
  };
  struct Geo {
    const Mesh &m;
    const double *vz;
    size_t base;
    int j;
    __device__ double L(int a) const { return m.Lz(j, a); }
    __device__ double h(int f) const { return m.hz(j, f); }
    __device__ double S(int f) const { return m.Sz(j, f); }
    __device__ double Vi(int a) const { return m.Vinv(j, a); }
    __device__ double w(int f) const { return vz[base + (size_t)f * m.plane()]; }
  } geo{m, vz, m.idx(i, j, 0), j};
  auto st = [&](int a, double r, const double (&T)[NQ]) {
    size_t c = m.idx(i, j, a);
    out.a[T_RHO][c] = r;
#pragma unroll
    for (int q = 0; q < NQ; q++) out.q[q][c] = T[q];
  };
  column_sweep<NQ>(a0, a1, dt, ld, geo, st);
}

// ------------------------------------------------------------------------
// X: one workgroup per ring, M zones per thread (zone i = tid + B m), three
// LDS arrays for neighbour exchange.
// ------------------------------------------------------------------------
__device__ inline double mc_slope(double qm, double q0, double qp) {
  double dq = 0.5 * (qp - qm);
  if ((qp - q0) * (q0 - qm) <= 0.0) return 0.0;
  double mag = fmin(fmin(2.0 * fabs(q0 - qm), 2.0 * fabs(qp - q0)), fabs(dq));
  return dq > 0.0 ? mag : -mag;
}

// PPA interface value supplied by zone 0 (right face for xi >= 0, left face
// for xi < 0): Eqs. 34, 35, 36 and the interface formula with |xi|.
__device__ inline double ppa_star(double q2m, double qm, double q0, double qp, double q2p, double xi) {
  const double sixth = 1.0 / 6.0;
  double dmm = mc_slope(q2m, qm, q0), dm0 = mc_slope(qm, q0, qp), dmp = mc_slope(q0, qp, q2p);
  double l = qm + 0.5 * (q0 - qm) - (dm0 - dmm) * sixth;
  double r = q0 + 0.5 * (qp - q0) - (dmp - dm0) * sixth;
  double D = r - l, C = q0 - 0.5 * (l + r);
  if ((qp - q0) * (q0 - qm) <= 0.0) {
    l = q0;
    r = q0;
  } else if (D * C > D * D * sixth) {
    l = 3.0 * q0 - 2.0 * r;
  } else if (-D * D * sixth > D * C) {
    r = 3.0 * q0 - 2.0 * l;
  }
  double x = fabs(xi);
  if (xi >= 0.0) return r + x * (q0 - r) + x * (1.0 - x) * (2.0 * q0 - r - l);
  return l + x * (q0 - l) + x * (1.0 - x) * (2.0 * q0 - r - l);
}

// van Leer interface value with a uniform zone width: slopes in units of
// the zone (harmonic mean of the raw differences), cw = w dt / dX.
__device__ inline double vlx_star(double q2m, double qm, double q0, double qp, double w, double cw) {
  if (w >= 0.0) {
    double dm = qm - q2m, dp = q0 - qm, pr = dm * dp;
    double a = pr > 0.0 ? 2.0 * pr / (dm + dp) : 0.0;
    return qm + a * (1.0 - cw) * 0.5;
  }
  double dm = q0 - qm, dp = qp - q0, pr = dm * dp;
  double a = pr > 0.0 ? 2.0 * pr / (dm + dp) : 0.0;
  return q0 - a * (1.0 + cw) * 0.5;
}

template <int M>
__global__ __launch_bounds__(512) void k_ring_x(Mesh m, const double *__restrict__ vx2, TSet T, StateP s,
                                                const double *__restrict__ v0, const int32_t *__restrict__ Nsh,
                                                const double *__restrict__ xis, const double *__restrict__ dtp) {
  extern __shared__ double lds[];
  const int n = m.nx, B = blockDim.x, tid = threadIdx.x;
  double *Qs = lds, *Fs = lds + n, *Es = lds + 2 * n;
  const int r = blockIdx.x;
  const int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  const double dt = *dtp;
  const double dX = m.DX(j, k), S = m.Sx(j, k), vinv = m.Vinv(j, k);
  const bool fg = m.fargo != 0;
  const double vb = fg ? v0[r] : 0.0;
  const int N = fg ? Nsh[r] : 0;
  const double xi = fg ? xis[r] : 0.0;
  const size_t base = m.idx(0, j, k);
  const double cdt = dt / dX, pfac = xi * dX * S;
  int im2[M], im1[M], ip1[M], ip2[M], out[M];
  double r0[M], r1[M], rf[M], ri0[M], ri1[M], fr[M], wv[M], pxm[M], pxp[M];
#pragma unroll
  for (int mm = 0; mm < M; mm++) {
    int i = tid + B * mm;
    int ii = i < n ? i : 0;
    im1[mm] = (ii - 1 + n) % n;
    im2[mm] = (ii - 2 + 2 * n) % n;
    ip1[mm] = (ii + 1) % n;
    ip2[mm] = (ii + 2) % n;
    int o = (ii + N) % n;
    out[mm] = o < 0 ? o + n : o;
  }
#define ZONES(...)                                     \
  _Pragma("unroll") for (int mm = 0; mm < M; mm++) {   \
    const int i = tid + B * mm;                        \
    if (i < n) {                                       \
      __VA_ARGS__                                      \
    }                                                  \
  }
  // density: van Leer sweep with the residual velocity
  ZONES(r0[mm] = T.a[T_RHO][base + i]; wv[mm] = vx2[base + i] - vb; Qs[i] = r0[mm]; ri0[mm] = 1.0 / r0[mm];)
  __syncthreads();
  ZONES(double w = wv[mm];
        double st = vlx_star(Qs[im2[mm]], Qs[im1[mm]], Qs[i], Qs[ip1[mm]], w, w * cdt);
        fr[mm] = w * st * S * dt; Fs[i] = fr[mm];)
  __syncthreads();
  ZONES(r1[mm] = r0[mm] - vinv * (Fs[ip1[mm]] - fr[mm]); ri1[mm] = 1.0 / r1[mm]; Qs[i] = r1[mm]; rf[mm] = r1[mm];)
  if (fg) {
    __syncthreads();
    ZONES(double st = ppa_star(Qs[im2[mm]], Qs[im1[mm]], Qs[i], Qs[ip1[mm]], Qs[ip2[mm]], xi);
          Es[xi >= 0.0 ? ip1[mm] : i] = pfac * st;)
    __syncthreads();
    ZONES(rf[mm] = r1[mm] - vinv * (Es[ip1[mm]] - Es[i]);)
  }
  // the other quantities, in the order Pi-_x, Pi+_x, Pi-_y, Pi+_y [, Pi-_z, Pi+_z] [, e]
  for (int q = 0; q < T.nq; q++) {
    double *Tq = T.q[q] + base;
    double qv[M];
    __syncthreads();
    ZONES(qv[mm] = Tq[i]; Qs[i] = qv[mm] * ri0[mm];)
    __syncthreads();
    ZONES(double w = wv[mm];
          Fs[i] = vlx_star(Qs[im2[mm]], Qs[im1[mm]], Qs[i], Qs[ip1[mm]], w, w * cdt) * fr[mm];)
    __syncthreads();
    ZONES(qv[mm] = qv[mm] - vinv * (Fs[ip1[mm]] - Fs[i]);)
    if (fg) {
      ZONES(Qs[i] = qv[mm] * ri1[mm];)
      __syncthreads();
      ZONES(double st = ppa_star(Qs[im2[mm]], Qs[im1[mm]], Qs[i], Qs[ip1[mm]], Qs[ip2[mm]], xi);
            int f = xi >= 0.0 ? ip1[mm] : i; Fs[f] = st * Es[f];)
      __syncthreads();
      ZONES(qv[mm] = qv[mm] - vinv * (Fs[ip1[mm]] - Fs[i]);)
    }
    if (q == 0) {
      ZONES(pxm[mm] = qv[mm];)
    } else if (q == 1) {
      ZONES(pxp[mm] = qv[mm];)
    } else if (T.a[T_E] && q == T.nq - 1) {
      ZONES(s.e[base + out[mm]] = qv[mm];)
    } else {
      ZONES(Tq[out[mm]] = qv[mm];)
    }
  }
  // box 12d along X (Eq. 18) on the shifted ring: face i + N takes zones i - 1, i
  __syncthreads();
  ZONES(Fs[i] = pxp[mm]; Qs[i] = rf[mm];)
  __syncthreads();
  ZONES(double mom = (Fs[im1[mm]] + pxm[mm]) / (Qs[im1[mm]] + rf[mm]);
        s.vx[base + out[mm]] = m.vx_from(j, k, mom); s.rho[base + out[mm]] = rf[mm];)
#undef ZONES
}

// ------------------------------------------------------------------------
// 12d along Y and Z on the owned faces (Eq. 18 with Tab. "momenta").
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_vel(Mesh m, StateP s, TSet T) {
  unsigned Lb = xcd_remap(blockIdx.x, gridDim.x);
  int kk = (int)(Lb % (unsigned)m.nz);
  unsigned rest = Lb / (unsigned)m.nz;
  int jj = (int)(rest % (unsigned)m.ny), ib = (int)(rest / (unsigned)m.ny);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  int j = m.j0 + jj, k = m.k0 + kk;
  size_t c = m.idx(i, j, k);
  double rc = s.rho[c];
  if (j >= m.ylo()) {
    size_t cm = m.idx(i, m.jbelow(j), k);
    s.vy[c] = (T.a[T_PYP][cm] + T.a[T_PYM][c]) / (s.rho[cm] + rc);
  }
  if (m.d3 && k >= m.zlo()) {
    size_t cm = m.idx(i, j, m.kbelow(k));
    double v = (T.a[T_PZP][cm] + T.a[T_PZM][c]) / (s.rho[cm] + rc);
    s.vz[c] = m.geo == FARGO_SPHERICAL ? v / m.g.ymed[j] : v;
  }
}

template <int NQ, bool D3, bool ADI>
void sweep_y_launch(Launch &L, const Mesh &m, const StateP &s, const TSet &out, const double *dt) {
  int nib, bs;
  row_blocks(m.nx, nib, bs);
  int nchunk = (m.ny + CHUNK - 1) / CHUNK;
  int nrows = D3 ? m.nz + 4 : 1;
  unsigned nb = (unsigned)nib * (unsigned)nchunk * (unsigned)nrows;
  k_sweep_y<NQ, D3, ADI><<<nb, bs, 0, L.s>>>(m, s.rho, s.vx, s.vy, s.vz, s.e, out, dt, nchunk);
}

template <int NQ>
void sweep_z_launch(Launch &L, const Mesh &m, const double *vz, const TSet &in, const TSet &out, const double *dt) {
  int nib, bs;
  row_blocks(m.nx, nib, bs);
  int nchunk = (m.nz + CHUNK - 1) / CHUNK;
  unsigned nb = (unsigned)nib * (unsigned)nchunk * (unsigned)m.ny;
  k_sweep_z<NQ><<<nb, bs, 0, L.s>>>(m, vz, in, out, dt, nchunk);
}

template <int M>
void ring_launch(Launch &L, const Mesh &m, int B, const double *vx2, const TSet &T, const StateP &s,
                 const double *v0, const int32_t *N, const double *xi, const double *dt) {
  k_ring_x<M><<<m.nring, B, 3 * (size_t)m.nx * sizeof(double), L.s>>>(m, vx2, T, s, v0, N, xi, dt);
}

} // namespace

// s: rho of the state, post-source velocities and energy (box 9 filled)
void launch_sweep_y(Launch &L, const Mesh &m, const StateP &s, const TSet &out, const double *dt) {
  prof_begin(L, K_SWEEP_Y);
  bool adi = m.eos == FARGO_ADIABATIC;
  if (m.d3) {
    if (adi) sweep_y_launch<7, true, true>(L, m, s, out, dt);
    else sweep_y_launch<6, true, false>(L, m, s, out, dt);
  } else {
    if (adi) sweep_y_launch<5, false, true>(L, m, s, out, dt);
    else sweep_y_launch<4, false, false>(L, m, s, out, dt);
  }
  prof_end(L, K_SWEEP_Y);
}

void launch_sweep_z(Launch &L, const Mesh &m, const double *vz, const TSet &in, const TSet &out, const double *dt) {
  prof_begin(L, K_SWEEP_Z);
  if (in.nq == 7) sweep_z_launch<7>(L, m, vz, in, out, dt);
  else sweep_z_launch<6>(L, m, vz, in, out, dt);
  prof_end(L, K_SWEEP_Z);
}

// Block of B <= 512 threads with M = ceil(nx / B) zones each.
void launch_ring_x(Launch &L, const Mesh &m, const double *vx2, const TSet &T, const StateP &s, const double *v0,
                   const int32_t *N, const double *xi, const double *dt) {
  int B = m.nx < 512 ? (m.nx + 63) / 64 * 64 : 512;
  int M = (m.nx + B - 1) / B;
  prof_begin(L, K_RING_X);
  if (M == 1) ring_launch<1>(L, m, B, vx2, T, s, v0, N, xi, dt);
  else if (M == 2) ring_launch<2>(L, m, B, vx2, T, s, v0, N, xi, dt);
  else if (M == 3) ring_launch<3>(L, m, B, vx2, T, s, v0, N, xi, dt);
  else ring_launch<4>(L, m, B, vx2, T, s, v0, N, xi, dt);
  prof_end(L, K_RING_X);
}

void launch_vel(Launch &L, const Mesh &m, const StateP &s, const TSet &T) {
  int nib, bs;
  row_blocks(m.nx, nib, bs);
  unsigned nb = (unsigned)nib * (unsigned)m.ny * (unsigned)m.nz;
  prof_begin(L, K_VEL);
  k_vel<<<nb, bs, 0, L.s>>>(m, s, T);
  prof_end(L, K_VEL);
}

} // namespace fargo
