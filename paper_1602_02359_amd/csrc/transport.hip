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
//
// The field type F is double, or float for the FP32-bulk state; the arithmetic
// of a kernel is carried out in F (per-ring constants such as dt/dX and the
// PPA residual xi are formed in FP64 and rounded to F).
#include "fargo_internal.h"

namespace fargo {

namespace {

constexpr int CHUNK = 64; // zones per thread along the sweep direction

// van Leer slope per unit length from the one-sided differences and the
// centre distances below (hm) and above (hp): 2 dl dr/(dl + dr) with
// dl = dm/hm, dr = dp/hp, zero unless dl dr > 0.
template <typename F>
__device__ inline F vl_slope(F qm, F q0, F qp, F hm, F hp) {
  F dm = q0 - qm, dp = qp - q0;
  F pr = dm * dp;
  return pr > F(0) ? F(2) * pr / (dm * hp + dp * hm) : F(0);
}

// half-step interface value at a face, upwinded on w (Eq. 15)
template <typename F>
__device__ inline F vl_star(F w, F dt, F ql, F al, F Ll, F qr, F ar, F Lr) {
  return w >= F(0) ? ql + al * (Ll - w * dt) * F(0.5) : qr - ar * (Lr + w * dt) * F(0.5);
}

template <typename F, int NQ>
struct Zone {
  F rho, q[NQ], T[NQ]; // density, Q/rho, conserved Q
};

// Column sweep over zones [a0, a1) of one column; `ld(a, Zone&)` loads zone a,
// `geo` gives L(a) (zone width), h(f) (centre distance at face f), S(f),
// Vi(a), w(f); `st(a, rho, T[])` stores the updated zone.
template <typename F, int NQ, class LD, class GEO, class ST>
__device__ inline void column_sweep(int a0, int a1, F dt, const LD &ld, const GEO &geo, const ST &st) {
  Zone<F, NQ> zm, z0, zp;
  ld(a0 - 2, zp); // used only for the first slope
  ld(a0 - 1, zm);
  ld(a0, z0);
  F sm[NQ + 1], s0[NQ + 1];
  {
    F hm = geo.h(a0 - 1), hp = geo.h(a0);
    sm[NQ] = vl_slope(zp.rho, zm.rho, z0.rho, hm, hp);
#pragma unroll
    for (int q = 0; q < NQ; q++) sm[q] = vl_slope(zp.q[q], zm.q[q], z0.q[q], hm, hp);
  }
  F Fp = F(0), FQp[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) FQp[q] = F(0);
  F Lm = geo.L(a0 - 1);
  for (int f = a0; f <= a1; f++) {
    ld(f + 1, zp);
    F hm = geo.h(f), hp = geo.h(f + 1);
    s0[NQ] = vl_slope(zm.rho, z0.rho, zp.rho, hm, hp);
#pragma unroll
    for (int q = 0; q < NQ; q++) s0[q] = vl_slope(zm.q[q], z0.q[q], zp.q[q], hm, hp);
    F L0 = geo.L(f);
    F w = geo.w(f);
    F Fr = w * vl_star(w, dt, zm.rho, sm[NQ], Lm, z0.rho, s0[NQ], L0) * geo.S(f) * dt;
    F FQ[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) FQ[q] = vl_star(w, dt, zm.q[q], sm[q], Lm, z0.q[q], s0[q], L0) * Fr;
    if (f > a0) {
      F vi = geo.Vi(f - 1);
      F Tn[NQ];
#pragma unroll
      for (int q = 0; q < NQ; q++) Tn[q] = zm.T[q] - vi * (FQ[q] - FQp[q]);
      st(f - 1, zm.rho - vi * (Fr - Fp), Tn);
    }
    Fp = Fr;
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
template <typename F, int NQ, bool D3, bool ADI>
__global__ __launch_bounds__(256) void k_sweep_y(Mesh m, const F *__restrict__ rho, const F *__restrict__ vx,
                                                 const F *__restrict__ vy, const F *__restrict__ vz,
                                                 const F *__restrict__ e, TSetT<F> out,
                                                 const double *__restrict__ dtp, int nchunk) {
  const int nrows = D3 ? m.nz + 4 : 1, kbase = D3 ? m.k0 - 2 : 0;
  unsigned Lb = xcd_remap(blockIdx.x, gridDim.x);
  int kr = (int)(Lb % (unsigned)nrows);
  unsigned rest = Lb / (unsigned)nrows;
  int ch = (int)(rest % (unsigned)nchunk), ib = (int)(rest / (unsigned)nchunk);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  const int k = kbase + kr;
  const int a0 = m.j0 + ch * CHUNK, a1 = min(a0 + CHUNK, m.jn);
  const F dt = (F)*dtp;
  const int ip = i + 1 == m.nx ? 0 : i + 1;
  const unsigned pitch = m.pitch, plane = (unsigned)m.plane();
  auto ld = [&](int a, Zone<F, NQ> &z) {
    unsigned c = m.o32(i, a, k);
    F r = rho[c];
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
    const F *vy;
    unsigned base;
    int k;
    __device__ F L(int a) const { return (F)m.g.Ly[a]; }
    __device__ F h(int f) const { return (F)m.g.hy[f]; }
    __device__ F S(int f) const { return (F)m.Sy(f, k); }
    __device__ F Vi(int a) const { return (F)m.Vinv(a, k); }
    __device__ F w(int f) const { return vy[base + (unsigned)f * (unsigned)m.pitch]; }
  } geo{m, vy, m.o32(i, 0, k), k};
  auto st = [&](int a, F r, const F (&T)[NQ]) {
    unsigned c = m.o32(i, a, k);
    out.a[T_RHO][c] = r;
#pragma unroll
    for (int q = 0; q < NQ; q++) out.q[q][c] = T[q];
  };
  column_sweep<F, NQ>(a0, a1, dt, ld, geo, st);
}

// ------------------------------------------------------------------------
// Z sweep on the Y-swept quantities.
// ------------------------------------------------------------------------
template <typename F, int NQ>
__global__ __launch_bounds__(256) void k_sweep_z(Mesh m, const F *__restrict__ vz, TSetT<F> in, TSetT<F> out,
                                                 const double *__restrict__ dtp, int nchunk) {
  unsigned Lb = xcd_remap(blockIdx.x, gridDim.x);
  int jr = (int)(Lb % (unsigned)m.ny);
  unsigned rest = Lb / (unsigned)m.ny;
  int ch = (int)(rest % (unsigned)nchunk), ib = (int)(rest / (unsigned)nchunk);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  const int j = m.j0 + jr;
  const int a0 = m.k0 + ch * CHUNK, a1 = min(a0 + CHUNK, m.kn);
  const F dt = (F)*dtp;
  auto ld = [&](int a, Zone<F, NQ> &z) {
    unsigned c = m.o32(i, j, a);
    F r = in.a[T_RHO][c];
    F ri = F(1) / r;
    z.rho = r;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      z.T[q] = in.q[q][c];
      z.q[q] = z.T[q] * ri;
    }
  };
  struct Geo {
    const Mesh &m;
    const F *vz;
    unsigned base;
    int j;
    __device__ F L(int a) const { return (F)m.Lz(j, a); }
    __device__ F h(int f) const { return (F)m.hz(j, f); }
    __device__ F S(int f) const { return (F)m.Sz(j, f); }
    __device__ F Vi(int a) const { return (F)m.Vinv(j, a); }
    __device__ F w(int f) const { return vz[base + (unsigned)f * (unsigned)m.plane()]; }
  } geo{m, vz, m.o32(i, j, 0), j};
  auto st = [&](int a, F r, const F (&T)[NQ]) {
    unsigned c = m.o32(i, j, a);
    out.a[T_RHO][c] = r;
#pragma unroll
    for (int q = 0; q < NQ; q++) out.q[q][c] = T[q];
  };
  column_sweep<F, NQ>(a0, a1, dt, ld, geo, st);
}

// ------------------------------------------------------------------------
// X: one workgroup per ring, M zones per thread (zone i = tid + B m), three
// LDS arrays for neighbour exchange.
// ------------------------------------------------------------------------
template <typename F>
__device__ inline F mc_slope(F qm, F q0, F qp) {
  F dq = F(0.5) * (qp - qm);
  if ((qp - q0) * (q0 - qm) <= F(0)) return F(0);
  F mag = fmin(fmin(F(2) * fabs(q0 - qm), F(2) * fabs(qp - q0)), fabs(dq));
  return dq > F(0) ? mag : -mag;
}

// PPA interface value supplied by zone 0 (right face for xi >= 0, left face
// for xi < 0): Eqs. 34, 35, 36 and the interface formula with |xi|.
template <typename F>
__device__ inline F ppa_star(F q2m, F qm, F q0, F qp, F q2p, F xi) {
  const F sixth = F(1) / F(6);
  F dmm = mc_slope(q2m, qm, q0), dm0 = mc_slope(qm, q0, qp), dmp = mc_slope(q0, qp, q2p);
  F l = qm + F(0.5) * (q0 - qm) - (dm0 - dmm) * sixth;
  F r = q0 + F(0.5) * (qp - q0) - (dmp - dm0) * sixth;
  F D = r - l, C = q0 - F(0.5) * (l + r);
  if ((qp - q0) * (q0 - qm) <= F(0)) {
    l = q0;
    r = q0;
  } else if (D * C > D * D * sixth) {
    l = F(3) * q0 - F(2) * r;
  } else if (-D * D * sixth > D * C) {
    r = F(3) * q0 - F(2) * l;
  }
  F x = fabs(xi);
  if (xi >= F(0)) return r + x * (q0 - r) + x * (F(1) - x) * (F(2) * q0 - r - l);
  return l + x * (q0 - l) + x * (F(1) - x) * (F(2) * q0 - r - l);
}

// van Leer interface value with a uniform zone width: slopes in units of
// the zone (harmonic mean of the raw differences), cw = w dt / dX.
template <typename F>
__device__ inline F vlx_star(F q2m, F qm, F q0, F qp, F w, F cw) {
  if (w >= F(0)) {
    F dm = qm - q2m, dp = q0 - qm, pr = dm * dp;
    F a = pr > F(0) ? F(2) * pr / (dm + dp) : F(0);
    return qm + a * (F(1) - cw) * F(0.5);
  }
  F dm = q0 - qm, dp = qp - q0, pr = dm * dp;
  F a = pr > F(0) ? F(2) * pr / (dm + dp) : F(0);
  return q0 - a * (F(1) + cw) * F(0.5);
}

// neighbour index i + d (|d| <= 2) on a ring of n zones
__device__ inline int ringnb(int i, int d, int n) {
  int x = i + d;
  if (n >= 3) return x < 0 ? x + n : (x >= n ? x - n : x);
  x %= n;
  return x < 0 ? x + n : x;
}

template <typename F, int M>
__global__ __launch_bounds__(512, 4) void k_ring_x(Mesh m, const F *__restrict__ vx2, TSetT<F> T, StateT<F> s,
                                                const double *__restrict__ v0, const int32_t *__restrict__ Nsh,
                                                const double *__restrict__ xis, const double *__restrict__ dtp) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  F *lds = reinterpret_cast<F *>(lds_raw);
  const int n = m.nx, B = blockDim.x, tid = threadIdx.x;
  F *Qs = lds, *Fs = lds + n, *Es = lds + 2 * n, *Px = lds + 3 * n;
  const int r = blockIdx.x;
  const int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  const double dtd = *dtp;
  const F dt = (F)dtd;
  const double dXd = m.DX(j, k), Sd = m.Sx(j, k);
  const F S = (F)Sd, vinv = (F)m.Vinv(j, k);
  const bool fg = m.fargo != 0;
  const F vb = fg ? (F)v0[r] : F(0);
  const int N = fg ? Nsh[r] : 0;
  const int Nm = ((N % n) + n) % n; // shift on store: zone i goes to (i + Nm) mod n
  const double xid = fg ? xis[r] : 0.0;
  const F xi = (F)xid;
  const unsigned base = m.o32(0, j, k);
  const F cdt = (F)(dtd / dXd), pfac = (F)(xid * dXd * Sd);
  F r0[M], r1[M], rf[M], ri0[M], ri1[M], fr[M], wv[M], pxm[M], qn[M];
#define ZONES(...)                                     \
  _Pragma("unroll") for (int mm = 0; mm < M; mm++) {   \
    const int i = tid + B * mm;                        \
    if (i < n) {                                       \
      const int im1 = ringnb(i, -1, n), ip1 = ringnb(i, 1, n); \
      (void)im1;                                       \
      (void)ip1;                                       \
      __VA_ARGS__                                      \
    }                                                  \
  }
#define NB5(A) A[ringnb(i, -2, n)], A[im1], A[i], A[ip1], A[ringnb(i, 2, n)]
#define OUT() (i + Nm >= n ? i + Nm - n : i + Nm)
  // the next quantity is always loaded one quantity ahead: a barrier does not
  // wait for global loads, so their latency hides behind the LDS phases
  ZONES(qn[mm] = T.q[0][base + i];)
  // density: van Leer sweep with the residual velocity
  ZONES(r0[mm] = T.a[T_RHO][base + i]; wv[mm] = vx2[base + i] - vb; Qs[i] = r0[mm]; ri0[mm] = F(1) / r0[mm];)
  __syncthreads();
  ZONES(F w = wv[mm];
        F st = vlx_star(Qs[ringnb(i, -2, n)], Qs[im1], Qs[i], Qs[ip1], w, w * cdt);
        fr[mm] = w * st * S * dt; Fs[i] = fr[mm];)
  __syncthreads();
  ZONES(r1[mm] = r0[mm] - vinv * (Fs[ip1] - fr[mm]); ri1[mm] = F(1) / r1[mm]; Qs[i] = r1[mm]; rf[mm] = r1[mm];)
  if (fg) {
    __syncthreads();
    ZONES(F st = ppa_star(NB5(Qs), xi); Es[xi >= F(0) ? ip1 : i] = pfac * st;)
    __syncthreads();
    ZONES(rf[mm] = r1[mm] - vinv * (Es[ip1] - Es[i]);)
  }
  // the other quantities, in the order Pi-_x, Pi+_x, Pi-_y, Pi+_y [, Pi-_z, Pi+_z] [, e]
  for (int q = 0; q < T.nq; q++) {
    F *Tq = T.q[q] + base;
    F qv[M];
    ZONES(qv[mm] = qn[mm];)
    if (q + 1 < T.nq) {
      const F *Tn = T.q[q + 1] + base;
      ZONES(qn[mm] = Tn[i];)
    }
    __syncthreads();
    ZONES(Qs[i] = qv[mm] * ri0[mm];)
    __syncthreads();
    ZONES(F w = wv[mm];
          Fs[i] = vlx_star(Qs[ringnb(i, -2, n)], Qs[im1], Qs[i], Qs[ip1], w, w * cdt) * fr[mm];)
    __syncthreads();
    ZONES(qv[mm] = qv[mm] - vinv * (Fs[ip1] - Fs[i]);)
    if (fg) {
      ZONES(Qs[i] = qv[mm] * ri1[mm];)
      __syncthreads();
      ZONES(F st = ppa_star(NB5(Qs), xi); int f = xi >= F(0) ? ip1 : i; Fs[f] = st * Es[f];)
      __syncthreads();
      ZONES(qv[mm] = qv[mm] - vinv * (Fs[ip1] - Fs[i]);)
    }
    if (q == 0) {
      ZONES(pxm[mm] = qv[mm];)
    } else if (q == 1) {
      ZONES(Px[i] = qv[mm];)
    } else if (T.a[T_E] && q == T.nq - 1) {
      ZONES(s.e[base + OUT()] = qv[mm];)
    } else {
      ZONES(Tq[OUT()] = qv[mm];)
    }
  }
  // box 12d along X (Eq. 18) on the shifted ring: face i + N takes zones i - 1, i
  __syncthreads();
  ZONES(Qs[i] = rf[mm];)
  __syncthreads();
  ZONES(F mom = (Px[im1] + pxm[mm]) / (Qs[im1] + rf[mm]); const int o = OUT();
        s.vx[base + o] = m.vx_from(j, k, mom); s.rho[base + o] = rf[mm];)
#undef ZONES
#undef NB5
#undef OUT
}

// ------------------------------------------------------------------------
// 12d along Y and Z on the owned faces (Eq. 18 with Tab. "momenta").
// ------------------------------------------------------------------------
template <typename F>
__global__ __launch_bounds__(256) void k_vel(Mesh m, StateT<F> s, TSetT<F> T) {
  unsigned Lb = xcd_remap(blockIdx.x, gridDim.x);
  int kk = (int)(Lb % (unsigned)m.nz);
  unsigned rest = Lb / (unsigned)m.nz;
  int jj = (int)(rest % (unsigned)m.ny), ib = (int)(rest / (unsigned)m.ny);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  int j = m.j0 + jj, k = m.k0 + kk;
  unsigned c = m.o32(i, j, k);
  F rc = s.rho[c];
  if (j >= m.ylo()) {
    unsigned cm = m.o32(i, m.jbelow(j), k);
    s.vy[c] = (T.a[T_PYP][cm] + T.a[T_PYM][c]) / (s.rho[cm] + rc);
  }
  if (m.d3 && k >= m.zlo()) {
    unsigned cm = m.o32(i, j, m.kbelow(k));
    F v = (T.a[T_PZP][cm] + T.a[T_PZM][c]) / (s.rho[cm] + rc);
    s.vz[c] = m.geo == FARGO_SPHERICAL ? v / (F)m.g.ymed[j] : v;
  }
}

template <typename F, int NQ, bool D3, bool ADI>
void sweep_y_launch(Launch &L, const Mesh &m, const StateT<F> &s, const TSetT<F> &out, const double *dt) {
  int nib, bs;
  row_blocks(m.nx, nib, bs);
  int nchunk = (m.ny + CHUNK - 1) / CHUNK;
  int nrows = D3 ? m.nz + 4 : 1;
  unsigned nb = (unsigned)nib * (unsigned)nchunk * (unsigned)nrows;
  k_sweep_y<F, NQ, D3, ADI><<<nb, bs, 0, L.s>>>(m, s.rho, s.vx, s.vy, s.vz, s.e, out, dt, nchunk);
}

template <typename F, int NQ>
void sweep_z_launch(Launch &L, const Mesh &m, const F *vz, const TSetT<F> &in, const TSetT<F> &out, const double *dt) {
  int nib, bs;
  row_blocks(m.nx, nib, bs);
  int nchunk = (m.nz + CHUNK - 1) / CHUNK;
  unsigned nb = (unsigned)nib * (unsigned)nchunk * (unsigned)m.ny;
  k_sweep_z<F, NQ><<<nb, bs, 0, L.s>>>(m, vz, in, out, dt, nchunk);
}

template <typename F, int M>
void ring_launch(Launch &L, const Mesh &m, int B, const F *vx2, const TSetT<F> &T, const StateT<F> &s,
                 const double *v0, const int32_t *N, const double *xi, const double *dt) {
  k_ring_x<F, M><<<m.nring, B, 4 * (size_t)m.nx * sizeof(F), L.s>>>(m, vx2, T, s, v0, N, xi, dt);
}

} // namespace

// s: rho of the state, post-source velocities and energy (box 9 filled)
template <typename F>
void launch_sweep_y(Launch &L, const Mesh &m, const StateT<F> &s, const TSetT<F> &out, const double *dt) {
  prof_begin(L, K_SWEEP_Y);
  bool adi = m.eos == FARGO_ADIABATIC;
  if (m.d3) {
    if (adi) sweep_y_launch<F, 7, true, true>(L, m, s, out, dt);
    else sweep_y_launch<F, 6, true, false>(L, m, s, out, dt);
  } else {
    if (adi) sweep_y_launch<F, 5, false, true>(L, m, s, out, dt);
    else sweep_y_launch<F, 4, false, false>(L, m, s, out, dt);
  }
  prof_end(L, K_SWEEP_Y);
}

template <typename F>
void launch_sweep_z(Launch &L, const Mesh &m, const F *vz, const TSetT<F> &in, const TSetT<F> &out, const double *dt) {
  prof_begin(L, K_SWEEP_Z);
  if (in.nq == 7) sweep_z_launch<F, 7>(L, m, vz, in, out, dt);
  else sweep_z_launch<F, 6>(L, m, vz, in, out, dt);
  prof_end(L, K_SWEEP_Z);
}

// Block of B <= 512 threads with M = ceil(nx / B) zones each.
template <typename F>
void launch_ring_x(Launch &L, const Mesh &m, const F *vx2, const TSetT<F> &T, const StateT<F> &s, const double *v0,
                   const int32_t *N, const double *xi, const double *dt) {
  int B = m.nx < 512 ? (m.nx + 63) / 64 * 64 : 512;
  int M = (m.nx + B - 1) / B;
  prof_begin(L, K_RING_X);
  if (M == 1) ring_launch<F, 1>(L, m, B, vx2, T, s, v0, N, xi, dt);
  else if (M == 2) ring_launch<F, 2>(L, m, B, vx2, T, s, v0, N, xi, dt);
  else if (M == 3) ring_launch<F, 3>(L, m, B, vx2, T, s, v0, N, xi, dt);
  else ring_launch<F, 4>(L, m, B, vx2, T, s, v0, N, xi, dt);
  prof_end(L, K_RING_X);
}

template <typename F>
void launch_vel(Launch &L, const Mesh &m, const StateT<F> &s, const TSetT<F> &T) {
  int nib, bs;
  row_blocks(m.nx, nib, bs);
  unsigned nb = (unsigned)nib * (unsigned)m.ny * (unsigned)m.nz;
  prof_begin(L, K_VEL);
  k_vel<F><<<nb, bs, 0, L.s>>>(m, s, T);
  prof_end(L, K_VEL);
}

#define FARGO_TRANSPORT_INST(F)                                                                                    \
  template void launch_sweep_y<F>(Launch &, const Mesh &, const StateT<F> &, const TSetT<F> &, const double *);   \
  template void launch_sweep_z<F>(Launch &, const Mesh &, const F *, const TSetT<F> &, const TSetT<F> &,         \
                                  const double *);                                                               \
  template void launch_ring_x<F>(Launch &, const Mesh &, const F *, const TSetT<F> &, const StateT<F> &,         \
                                 const double *, const int32_t *, const double *, const double *);               \
  template void launch_vel<F>(Launch &, const Mesh &, const StateT<F> &, const TSetT<F> &);
FARGO_TRANSPORT_INST(double)
FARGO_TRANSPORT_INST(float)
#undef FARGO_TRANSPORT_INST

} // namespace fargo
