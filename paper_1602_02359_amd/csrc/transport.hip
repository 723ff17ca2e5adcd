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
// PPA residual xi are formed in FP64 and rounded to F).  In FP32, v_x and the
// X momenta are deviations from a per-ring FP64 background (v_x - vb and
// rho R (v_x - vb)): the Y and Z sweeps add the background's increments
// between rings (column_sweep), the X transport, where it is constant, needs
// nothing, and 12d forms the deviation again.
#include <type_traits>

#include "fargo_internal.h"

namespace fargo {

namespace {

// Reciprocal and quotient for the ring kernel, which is bound by its vector
// instruction count: the hardware reciprocal estimate refined by
// Newton-Raphson steps r <- r + r (1 - d r), two in FP64 and one in FP32,
// which leaves r within about one unit in the last place of 1/d (the correctly
// rounded division costs about twice the instructions).  The rounding of such
// a quotient varies from zone to zone like that of a division.  d must be a
// normal number; a zero or denormal d, which the kernel only meets in
// discarded selects and halo lanes, gives an infinite or meaningless value and
// no trap.
__device__ inline double ring_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}
__device__ inline double ring_div(double n, double d) { return n * ring_rcp(d); }
__device__ inline float ring_rcp(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  return fmaf(r, fmaf(-d, r, 1.0f), r);
}
__device__ inline float ring_div(float n, float d) { return n * ring_rcp(d); }
// The quotient of a column sweep's van Leer slope: correctly rounded in FP64
// (the sweeps there are bound by memory), the refined reciprocal in FP32,
// where the Y sweep is bound by its vector instructions (as in the ring
// kernel and the Z part of k_zx)
__device__ inline double sweep_div(double n, double d) { return n / d; }
__device__ inline float sweep_div(float n, float d) { return ring_div(n, d); }

// van Leer slope per unit length from the one-sided differences and the
// centre distances below (hm) and above (hp): 2 dl dr/(dl + dr) with
// dl = dm/hm, dr = dp/hp, zero unless dl dr > 0.
// Contraction is off in the slopes: a sweep forms the first slope of a chunk
// of zones before its loop and the others inside it, and the same rounding
// in both places keeps the result independent of the chunk size.
template <typename F>
__device__ inline F vl_slope(F qm, F q0, F qp, F hm, F hp) {
#pragma clang fp contract(off)
  F dm = q0 - qm, dp = qp - q0;
  F pr = dm * dp;
  return pr > F(0) ? sweep_div(F(2) * pr, dm * hp + dp * hm) : F(0);
}

// The same slope for a quantity stored as a deviation from a background that
// changes from zone to zone: bm and bp are the background's increments across
// the lower and upper face, so the differences are those of the full values.
template <typename F>
__device__ inline F vl_slope_b(F qm, F q0, F qp, F hm, F hp, F bm, F bp) {
#pragma clang fp contract(off)
  F dm = (q0 - qm) + bm, dp = (qp - q0) + bp;
  F pr = dm * dp;
  return pr > F(0) ? sweep_div(F(2) * pr, dm * hp + dp * hm) : F(0);
}

// half-step interface value at a face, upwinded on w (Eq. 15)
template <typename F>
__device__ inline F vl_star(F w, F dt, F ql, F al, F Ll, F qr, F ar, F Lr) {
  return w >= F(0) ? ql + al * (Ll - w * dt) * F(0.5) : qr - ar * (Lr + w * dt) * F(0.5);
}

template <typename F, int NQ, bool CT>
struct Zone {
  F rho, q[NQ]; // density, Q/rho
  F w;          // velocity on the zone's lower face in the sweep direction
  F T[CT ? NQ : 1]; // conserved Q, when carried in the window (CT)
};

// Column sweep over zones [a0, a1) of one column.  `raw(a, RW&)` issues the
// loads of zone a, `derive(a, const RW&, Zone&)` forms its density, Q/rho and
// lower-face velocity, `Tof(a, const Zone&, q)` gives the conserved Q of zone
// a (carried in the window when CT, else formed again); `geo` gives L(a) (zone width), h(f)
// (centre distance at face f), S(f), Vi(a); `st(a, rho, T[])` stores the
// updated zone.  The loads of zone f + 1 + PD are issued while zone f is
// being computed (PD = 1 or 2 zones of loads in flight; with two, the two
// load buffers take turns, so that no copy waits for a load).
// With DEV, quantities 0 and 1 (the X momenta) are deviations from a
// background ell that is constant on a ring (the FP32-bulk state): `dl(f)`
// gives ell(f) - ell(f - 1) at face f.  Slopes take the full differences,
// the interface value is taken relative to the background of the face's
// lower zone, and the update of a zone adds the background carried in
// through its lower face, so that in exact arithmetic the result is the
// full update minus ell times the updated density.
template <typename F, int NQ, bool CT, bool DEV, class RW, int PD = 1, class RAW, class DER, class TOF, class GEO,
          class ST, class DLF>
__device__ inline void column_sweep(int a0, int a1, F dt, const RAW &raw, const DER &derive, const TOF &Tof,
                                    const GEO &geo, const ST &st, const DLF &dl) {
  static_assert(PD == 1 || PD == 2, "one or two zones of loads in flight");
  Zone<F, NQ, CT> zm, z0, zp;
  RW rn, rn2;
  raw(a0 - 2, rn);
  derive(a0 - 2, rn, zp); // used only for the first slope
  raw(a0 - 1, rn);
  derive(a0 - 1, rn, zm);
  raw(a0, rn);
  derive(a0, rn, z0);
  raw(a0 + 1, rn);
  if (PD == 2 && a0 + 2 <= a1 + 1) raw(a0 + 2, rn2);
  F sm[NQ + 1], s0[NQ + 1];
  F dlf = DEV ? dl(a0) : F(0); // background increment at face f
  {
    F hm = geo.h(a0 - 1), hp = geo.h(a0);
    sm[NQ] = vl_slope(zp.rho, zm.rho, z0.rho, hm, hp);
#pragma unroll
    for (int q = 0; q < NQ; q++)
      sm[q] = (DEV && q < 2) ? vl_slope_b(zp.q[q], zm.q[q], z0.q[q], hm, hp, dl(a0 - 1), dlf)
                             : vl_slope(zp.q[q], zm.q[q], z0.q[q], hm, hp);
  }
  F Fp = F(0), FQp[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) FQp[q] = F(0);
  F Lm = geo.L(a0 - 1);
  // face f: zone f + 1 from buffer cur, whose loads are then refilled with
  // those of zone f + 1 + PD
  auto face = [&](int f, RW &cur) {
    derive(f + 1, cur, zp);
    if (f + 1 + PD <= a1 + 1) raw(f + 1 + PD, cur);
    const F dlf1 = DEV ? dl(f + 1) : F(0);
    F hm = geo.h(f), hp = geo.h(f + 1);
    s0[NQ] = vl_slope(zm.rho, z0.rho, zp.rho, hm, hp);
#pragma unroll
    for (int q = 0; q < NQ; q++)
      s0[q] = (DEV && q < 2) ? vl_slope_b(zm.q[q], z0.q[q], zp.q[q], hm, hp, dlf, dlf1)
                             : vl_slope(zm.q[q], z0.q[q], zp.q[q], hm, hp);
    F L0 = geo.L(f);
    F w = z0.w;
    F Fr = w * vl_star(w, dt, zm.rho, sm[NQ], Lm, z0.rho, s0[NQ], L0) * geo.S(f) * dt;
    F FQ[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++)
      FQ[q] = vl_star(w, dt, zm.q[q], sm[q], Lm, (DEV && q < 2) ? z0.q[q] + dlf : z0.q[q], s0[q], L0) * Fr;
    if (f > a0) {
      F vi = geo.Vi(f - 1);
      F Tn[NQ];
#pragma unroll
      for (int q = 0; q < NQ; q++) Tn[q] = Tof(f - 1, zm, q) - vi * (FQ[q] - FQp[q]);
      st(f - 1, zm.rho - vi * (Fr - Fp), Tn);
    }
    Fp = Fr;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      // the flux through face f relative to the background of its upper zone
      FQp[q] = (DEV && q < 2) ? FQ[q] - dlf * Fr : FQ[q];
      sm[q] = s0[q];
    }
    sm[NQ] = s0[NQ];
    zm = z0;
    z0 = zp;
    Lm = L0;
    dlf = dlf1;
  };
  if constexpr (PD == 1) {
#pragma unroll 1
    for (int f = a0; f <= a1; f++) face(f, rn);
  } else {
#pragma unroll 1
    for (int f = a0; f <= a1; f += 2) {
      face(f, rn);
      if (f + 1 <= a1) face(f + 1, rn2);
    }
  }
}

// ------------------------------------------------------------------------
// Y sweep, forming the momenta from the post-source state (box 12a fused).
// Quantities: Pi-_x, Pi+_x, Pi-_y, Pi+_y [, Pi-_z, Pi+_z] [, e].
// ------------------------------------------------------------------------
template <typename F, int NQ, bool D3, bool ADI>
__device__ __forceinline__ void sweep_y_body(Mesh m, const F *__restrict__ rho, const F *__restrict__ vx,
                                                 const F *__restrict__ vy, const F *__restrict__ vz,
                                                 const F *__restrict__ e, TSetT<F> out,
                                                 const double *__restrict__ dtp, int nchunk, unsigned bid_, unsigned nbk_) {
  const int nrows = D3 ? m.nz + 4 : 1, kbase = D3 ? m.k0 - 2 : 0;
  unsigned Lb = xcd_remap(bid_, nbk_);
  int kr = (int)(Lb % (unsigned)nrows);
  unsigned rest = Lb / (unsigned)nrows;
  int ch = (int)(rest % (unsigned)nchunk), ib = (int)(rest / (unsigned)nchunk);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  const int k = kbase + kr;
  const int a0 = m.j0 + ch * m.chunk, a1 = min(a0 + m.chunk, m.jn);
  const F dt = (F)*dtp;
  const int ip = i + 1 == m.nx ? 0 : i + 1;
  constexpr bool DEV = sizeof(F) == 4;
  const unsigned pitch = m.pitch, plane = (unsigned)m.plane();
  struct Raw {
    F rho, vx0, vx1, vy0, vy1, vz0, vz1, e;
  };
  auto raw = [&](int a, Raw &z) {
    const unsigned c = m.o32(i, a, k);
    z.rho = rho[c];
    z.vx0 = vx[c];
    z.vx1 = vx[c - i + ip];
    z.vy0 = vy[c];
    z.vy1 = vy[c + pitch];
    if (D3) {
      z.vz0 = vz[c];
      z.vz1 = vz[c + plane];
    }
    if (ADI) z.e = e[c];
  };
  auto derive = [&](int a, const Raw &w, Zone<F, NQ, false> &z) {
    const F r = w.rho;
    z.rho = r;
    z.w = w.vy0;
    if constexpr (DEV) { // FP32: v_x is a deviation, and so are the X momenta
      z.q[0] = m.mxd(a, k, w.vx0);
      z.q[1] = m.mxd(a, k, w.vx1);
    } else {
      z.q[0] = m.mx(a, k, w.vx0);
      z.q[1] = m.mx(a, k, w.vx1);
    }
    z.q[2] = w.vy0;
    z.q[3] = w.vy1;
    if (D3) {
      z.q[4] = m.mz(a, w.vz0);
      z.q[5] = m.mz(a, w.vz1);
    }
    if (ADI) {
      z.q[NQ - 1] = w.e / r;
      z.T[0] = w.e; // the window carries no other conserved value (CT is false)
    }
  };
  // the momenta are rho m(v) exactly as formed; e as loaded, carried in the
  // window (read again three rows later, it would come from memory again)
  auto Tof = [&](int, const Zone<F, NQ, false> &z, int q) {
    if (ADI && q == NQ - 1) return z.T[0];
    return z.rho * z.q[q];
  };
  struct Geo {
    const Mesh &m;
    int k;
    __device__ F L(int a) const { return (F)m.g.Ly(a); }
    __device__ F h(int f) const { return (F)m.g.hy(f); }
    __device__ F S(int f) const { return (F)m.Sy(f, k); }
    __device__ F Vi(int a) const { return (F)m.Vinv(a, k); }
  } geo{m, k};
  auto st = [&](int a, F r, const F (&T)[NQ]) {
    unsigned c = m.o32(i, a, k);
    out.a[T_RHO][c] = r;
#pragma unroll
    for (int q = 0; q < NQ; q++) out.q[q][c] = T[q];
  };
  auto dl = [&](int f) { return (F)m.bg(BG_DLY, f, k); };
  // two zones of loads in flight (measured faster on 3D meshes and on the
  // fused batch of 2D disks; the Z sweep, whose window holds the conserved
  // values too, gains nothing from it)
  column_sweep<F, NQ, false, DEV, Raw, 2>(a0, a1, dt, raw, derive, Tof, geo, st, dl);
}
template <typename F, int NQ, bool D3, bool ADI>
__global__ __launch_bounds__(256) void k_sweep_y(Mesh m, const F *__restrict__ rho, const F *__restrict__ vx,
                                                 const F *__restrict__ vy, const F *__restrict__ vz,
                                                 const F *__restrict__ e, TSetT<F> out,
                                                 const double *__restrict__ dtp, int nchunk) {
  sweep_y_body<F, NQ, D3, ADI>(m, rho, vx, vy, vz, e, out, dtp, nchunk, blockIdx.x, gridDim.x);
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
  const int a0 = m.k0 + ch * m.chunk, a1 = min(a0 + m.chunk, m.kn);
  const F dt = (F)*dtp;
  struct Raw {
    F rho, w, T[NQ];
  };
  auto raw = [&](int a, Raw &z) {
    const unsigned c = m.o32(i, j, a);
    z.rho = in.a[T_RHO][c];
    z.w = vz[c];
#pragma unroll
    for (int q = 0; q < NQ; q++) z.T[q] = in.q[q][c];
  };
  auto derive = [&](int, const Raw &w, Zone<F, NQ, true> &z) {
    const F ri = F(1) / w.rho;
    z.rho = w.rho;
    z.w = w.w;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      z.T[q] = w.T[q];
      z.q[q] = w.T[q] * ri;
    }
  };
  auto Tof = [&](int, const Zone<F, NQ, true> &z, int q) { return z.T[q]; };
  struct Geo {
    const Mesh &m;
    int j;
    __device__ F L(int a) const { return (F)m.Lz(j, a); }
    __device__ F h(int f) const { return (F)m.hz(j, f); }
    __device__ F S(int f) const { return (F)m.Sz(j, f); }
    __device__ F Vi(int a) const { return (F)m.Vinv(j, a); }
  } geo{m, j};
  auto st = [&](int a, F r, const F (&T)[NQ]) {
    unsigned c = m.o32(i, j, a);
    out.a[T_RHO][c] = r;
#pragma unroll
    for (int q = 0; q < NQ; q++) out.q[q][c] = T[q];
  };
  auto dl = [&](int f) { return (F)m.bg(BG_DLZ, j, f); };
  column_sweep<F, NQ, true, sizeof(F) == 4, Raw>(a0, a1, dt, raw, derive, Tof, geo, st, dl);
}

// Monotonised central slope of the PPA edge values (Eq. 34): zero at an
// extremum, else the central difference limited by twice each one-sided one.
// min(2 a, 2 b, |d| / 2) is formed as 2 min(a, b, |d| / 4) (exact: scaling by
// powers of two) and takes the sign of d (d = 0 only at an extremum).
template <typename F>
__device__ inline F mc_slope(F qm, F q0, F qp) {
  const F d = qp - qm;
  if ((qp - q0) * (q0 - qm) <= F(0)) return F(0);
  const F mag = F(2) * fmin(fmin(fabs(q0 - qm), fabs(qp - q0)), F(0.25) * fabs(d));
  return copysign(mag, d);
}

// ------------------------------------------------------------------------
// X: every wave owns a segment of one ring.  Lane l holds the M consecutive
// zones z0 + M l .. z0 + M l + M - 1 of a window of 64 M zones that starts
// HL zones before the segment and ends HR zones after it; zone neighbours
// come from the lane's own registers or, across lanes, by DPP lane moves.  The
// halo is recomputed instead of exchanged, so no wave waits for another and
// nothing goes through LDS.  The dependency cone of an output zone (van Leer
// residual sweep, PPA residual, 12d along X) spans zones z-6 .. z+5.
// Outputs are written out of place (shifted by N on store), so that the
// segments of a ring can run in any order.
// ------------------------------------------------------------------------
// Two zones per lane in both precisions (in FP32 four zones per lane, with
// fewer halo lanes, measured no faster: the larger register window lowers the
// number of waves that hide the loads).
template <typename F>
struct RingShape {
  static constexpr int M = 2, HLL = 3, HRL = 3; // halo lanes on each side
};

// Neighbour lanes through DPP whole-wave shifts by one lane (wave_shr:1,
// wave_shl:1): a VALU move, with no trip through the LDS crossbar.  The lane
// at the end of the wave, which has no source lane, reads zero (bound_ctrl);
// it is a halo lane, whose outputs are never stored.  Taking no old value
// lets the move write its destination directly, without a copy first.
template <int CTRL>
__device__ inline int dpp_lane(int x) { return __builtin_amdgcn_mov_dpp(x, CTRL, 0xf, 0xf, true); }
template <int CTRL, typename F>
__device__ inline F dpp_move(F x) {
  if constexpr (sizeof(F) == 8) {
    const long long v = __double_as_longlong(x);
    const int lo = dpp_lane<CTRL>((int)v), hi = dpp_lane<CTRL>((int)(v >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  } else {
    return __int_as_float(dpp_lane<CTRL>(__float_as_int(x)));
  }
}
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;
template <typename F>
__device__ inline F from_prev_lane(F x) { return dpp_move<DPP_WAVE_SHR1>(x); }
template <typename F>
__device__ inline F from_next_lane(F x) { return dpp_move<DPP_WAVE_SHL1>(x); }

// a[] of the lane's M zones and its two neighbours on each side
template <typename F, int M>
struct Span {
  F a[M];
  F p2, p1, n1, n2;
  __device__ inline void edges() {
    p2 = from_prev_lane(a[M - 2]);
    p1 = from_prev_lane(a[M - 1]);
    n1 = from_next_lane(a[0]);
    n2 = from_next_lane(a[1]);
  }
  __device__ inline F operator()(int x) const { // x in [-2, M + 1], static after unrolling
    return x == -2 ? p2 : x == -1 ? p1 : x == M ? n1 : x == M + 1 ? n2 : a[x];
  }
};

template <typename F, int M>
__device__ inline void next_of(const F (&a)[M], F (&out)[M]) { // value of zone z + 1
  const F n1 = from_next_lane(a[0]);
#pragma unroll
  for (int m = 0; m < M; m++) out[m] = m + 1 < M ? a[m + 1] : n1;
}
template <typename F, int M>
__device__ inline void prev_of(const F (&a)[M], F (&out)[M]) { // value of zone z - 1
  const F p1 = from_prev_lane(a[M - 1]);
#pragma unroll
  for (int m = 0; m < M; m++) out[m] = m > 0 ? a[m - 1] : p1;
}

// PPA on one zone (Eqs. 34-36): limit the parabola through the edge values
// l, r (flat at an extremum, steepened away from an overshoot), then the
// interface value supplied by the zone, the mean of the parabola over the
// fraction |xi| next to its right edge (xi >= 0) or left edge (xi < 0).
// The fraction enters through the ring constants X: x = |xi|, x (1 - x) and
// the sign of xi, which are the same for every zone of the ring.
template <typename F>
struct PpaX {
  F x, x1x;
  bool right; // xi >= 0
};
// (At an extremum both edges are q0 and the mean is q0 exactly; that case is
// taken at the end, so the steepening selects do not test it.)
template <typename F>
__device__ inline F ppa_eval(F qm, F q0, F qp, F l, F r, const PpaX<F> &X) {
  const F sixth = F(1) / F(6);
  const F D = r - l, C = q0 - F(0.5) * (l + r);
  const F DC = D * C, DD6 = D * D * sixth;
  const bool flat = (qp - q0) * (q0 - qm) <= F(0);
  const bool stl = DC > DD6, str = !stl && -DD6 > DC;
  const F ln = stl ? F(3) * q0 - F(2) * r : l;
  const F rn = str ? F(3) * q0 - F(2) * l : r;
  const F ed = X.right ? rn : ln;
  const F v = ed + X.x * (q0 - ed) + X.x1x * (F(2) * q0 - rn - ln);
  return flat ? q0 : v;
}

// Interface values on the lane's zones; each zone's slope and each face's
// edge value is computed once and handed to the neighbouring zone (in a
// register, or by a DPP lane move).
//   vlx_faces: van Leer on a uniform zone width, slopes in units of the zone
//   (harmonic mean of the two one-sided differences, zero unless they have
//   the same sign), and the half-step value at each zone's lower face
//   upwinded on w, with cw = w dt / dX (Eq. 15).
//   The upwind factors depend on the face velocity only and are formed once
//   for all quantities: (1 - cw)/2 and (1 + cw)/2 (the halving is exact).
template <typename F, int M>
struct Upwind {
  bool pos[M]; // w >= 0
  F cl[M], cr[M];
  __device__ inline void set(const F (&w)[M], F cdt) {
#pragma unroll
    for (int q = 0; q < M; q++) {
      const F cw = w[q] * cdt;
      pos[q] = w[q] >= F(0);
      cl[q] = (F(1) - cw) * F(0.5);
      cr[q] = (F(1) + cw) * F(0.5);
    }
  }
};
template <typename F, int M>
__device__ inline void vlx_faces(const Span<F, M> &Q, const Upwind<F, M> &U, F (&out)[M]) {
  F a[M], ap[M];
#pragma unroll
  for (int q = 0; q < M; q++) {
    const F dm = Q(q) - Q(q - 1), dp = Q(q + 1) - Q(q), pr = dm * dp;
    a[q] = pr > F(0) ? ring_div(F(2) * pr, dm + dp) : F(0);
  }
  prev_of(a, ap);
#pragma unroll
  for (int q = 0; q < M; q++) out[q] = U.pos[q] ? Q(q - 1) + ap[q] * U.cl[q] : Q(q) - a[q] * U.cr[q];
}
//   ppa_values: monotonised central slopes, the edge value of each face
//   (Eq. 34) and the interface value supplied by each zone.
template <typename F, int M>
__device__ inline void ppa_values(const Span<F, M> &Q, const PpaX<F> &X, F (&out)[M]) {
  const F sixth = F(1) / F(6);
  F d[M], dp[M], l[M], r[M];
#pragma unroll
  for (int q = 0; q < M; q++) d[q] = mc_slope(Q(q - 1), Q(q), Q(q + 1));
  prev_of(d, dp);
#pragma unroll
  for (int q = 0; q < M; q++) l[q] = Q(q - 1) + F(0.5) * (Q(q) - Q(q - 1)) - (d[q] - dp[q]) * sixth;
  next_of(l, r);
#pragma unroll
  for (int q = 0; q < M; q++) out[q] = ppa_eval(Q(q - 1), Q(q), Q(q + 1), l[q], r[q], X);
}

// Element i of the row that starts at p, for 0 <= i < 2^31 / sizeof(T): a
// uniform (scalar) row pointer plus a 32-bit byte offset, the addressing mode
// of a global access with a scalar base, which saves the 64-bit address
// arithmetic of every access.
template <typename T>
__device__ inline T *at(T *p, unsigned i) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T *>(reinterpret_cast<B *>(p) + i * (unsigned)sizeof(T));
}

// The lane's place in a segment of a ring: its M zones start at window (=
// ring) coordinate zl, iz[] are their ring indices (wrapped into [0, n)), and
// contig tells whether they are consecutive in memory.  Only the lanes outside
// the halo store, and only zones before the end of the segment.
template <typename F>
struct RingLane {
  static constexpr int M = RingShape<F>::M, HLL = RingShape<F>::HLL, HRL = RingShape<F>::HRL;
  static constexpr int U = (WAVE - HLL - HRL) * M; // output zones per wave
  int n, lane, zl, aend, iz[M];
  bool contig;
  __device__ inline RingLane(int nx, int seg, int ln) : n(nx), lane(ln) {
    const int a0 = seg * U;      // first output zone of the segment
    zl = a0 - HLL * M + ln * M;  // first zone of the lane
    aend = min(a0 + U, n);
    contig = zl >= 0 && zl + M <= n;
#pragma unroll
    for (int q = 0; q < M; q++) {
      const int z = (zl + q) % n;
      iz[q] = z < 0 ? z + n : z;
    }
  }
  __device__ inline bool useful(int q) const { return lane >= HLL && lane < WAVE - HRL && zl + q < aend; }
  // the lane's zones of the row that starts at p, one load per zone and no
  // branch on contig (for loads inside a loop)
  __device__ inline void load_each(const F *p, F (&out)[M]) const {
#pragma unroll
    for (int q = 0; q < M; q++) out[q] = *at(p, (unsigned)iz[q]);
  }
  // the lane's zones of the row that starts at p (two-element vector loads
  // where they are consecutive)
  __device__ inline void load(const F *p, F (&out)[M]) const {
    static_assert(M % 2 == 0, "pairs of zones per lane");
    if (contig) {
      using V2 = typename std::conditional<sizeof(F) == 8, double2, float2>::type;
      const V2 *v = reinterpret_cast<const V2 *>(at(p, (unsigned)zl));
#pragma unroll
      for (int q = 0; q < M / 2; q++) {
        const V2 t = v[q];
        out[2 * q] = t.x;
        out[2 * q + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < M; q++) out[q] = *at(p, (unsigned)iz[q]);
    }
  }
};

// Constants of ring (j, k): time step, face area, inverse volume, the
// shift velocity v0, the integer shift (as a store offset in [0, n)) and the
// PPA residual xi (Eqs. 32, 33), dt/dX, the PPA flux factor xi dX S, and the
// factors of 12d along X (Tab. "momenta": v = Pi/R - R Omega; R = 1 and
// Omega = 0 on a Cartesian mesh).
template <typename F>
struct RingConst {
  F dt, S, vinv, vb, cdt, pfac, R, iR, Rw;
  PpaX<F> X;
  bool fg;
  int Nm;
};
// The split of Eq. 29 for one ring: D = v0 dt / dX in this operation order
// with contraction off, N the nearest integer (ties away from zero) and
// xi = D - N, exact; the same arithmetic as the stand-alone split and the
// oracle, so N is reproduced bit for bit.
__device__ inline void ring_split_at(double v0, double dt, double dX, int &N, double &xi) {
#pragma clang fp contract(off)
  const double D = (v0 * dt) / dX;
  const double rn = round(D);
  N = (int)rn;
  xi = D - rn;
}

template <typename F>
__device__ inline RingConst<F> ring_const(const Mesh &m, int j, int k, int r, double dtd,
                                          const double *__restrict__ v0) {
  RingConst<F> C;
  const int n = m.nx;
  const double dXd = m.DX(j, k), Sd = m.Sx(j, k);
  C.dt = (F)dtd;
  C.S = (F)Sd;
  C.vinv = (F)m.Vinv(j, k);
  C.fg = m.fargo != 0;
  const double v0d = C.fg ? v0[r] : 0.0;
  // an FP32 v_x is a deviation from the ring's background vb: the residual
  // velocity is v_x - (v0 - vb)
  if constexpr (sizeof(F) == 4) C.vb = (F)(v0d - m.bg(BG_V, j, k));
  else C.vb = (F)v0d;
  int N = 0;
  double xid = 0.0;
  if (C.fg) ring_split_at(v0d, dtd, dXd, N, xid);
  C.Nm = ((N % n) + n) % n; // shift on store: zone i goes to (i + Nm) mod n
  const F xi = (F)xid;
  C.X = PpaX<F>{fabs(xi), fabs(xi) * (F(1) - fabs(xi)), xi >= F(0)};
  C.cdt = (F)(dtd / dXd);
  C.pfac = (F)(xid * dXd * Sd);
  if (m.geo == FARGO_CARTESIAN) {
    C.R = C.iR = F(1);
    C.Rw = F(0);
  } else {
    C.R = (F)m.Rcyl(j, k);
    C.iR = (F)(1.0 / m.Rcyl(j, k));
    // FP32: the X momenta are deviations R (v_x - vb) from the ring's
    // background, and so is the v_x formed from them (no frame term)
    C.Rw = sizeof(F) == 4 ? F(0) : C.R * (F)m.omega;
  }
  return C;
}

// Load order of the quantities of a ring: Pi-_y, Pi+_y [, Pi-_z, Pi+_z] [, e],
// then Pi-_x and Pi+_x, which 12d needs last (T.q holds Pi-_x, Pi+_x first).
template <int NQ>
__device__ constexpr int ring_qorder(int t) { return t + 2 < NQ ? t + 2 : t + 2 - NQ; }

// X transport of one ring segment held in registers (Ra: density, w: v_x on
// the lower faces, Qall[t]: quantity ring_qorder(t)), and its stores:
// van Leer residual sweep with w - v0, PPA residual, 12d along X; every
// output is stored shifted by N zones, out of place (Pi+-_y and Pi+-_z into
// Tout, e and the density and v_x into the state).
template <typename F, int NQ>
__device__ inline void ring_update(const RingLane<F> &L, const RingConst<F> &C, unsigned base,
                                   const F (&Ra)[RingShape<F>::M], F (&w)[RingShape<F>::M],
                                   const F (&Qall)[NQ][RingShape<F>::M], const TSetT<F> &Tout, bool has_e,
                                   const StateT<F> &s) {
  constexpr int M = RingShape<F>::M;
  const int n = L.n;
  auto out_at = [&](int q) { // index in the ring of the lane's zone q after the shift
    const int o = L.iz[q] + C.Nm;
    return (unsigned)(o >= n ? o - n : o);
  };
  const F dt = C.dt, S = C.S, vinv = C.vinv;
  F ri0[M], Fl[M], ri1[M], El[M], rf[M];
  Span<F, M> R;
#pragma unroll
  for (int q = 0; q < M; q++) R.a[q] = Ra[q];
  // ---- density: van Leer residual sweep, then the PPA residual
  Upwind<F, M> Uw;
  {
#pragma unroll
    for (int q = 0; q < M; q++) {
      w[q] -= C.vb;
      ri0[q] = ring_rcp(R.a[q]);
    }
    R.edges();
    F st[M];
    Uw.set(w, C.cdt);
    vlx_faces(R, Uw, st);
#pragma unroll
    for (int q = 0; q < M; q++) Fl[q] = w[q] * st[q] * S * dt;
    F Fh[M];
    next_of(Fl, Fh);
    Span<F, M> R1;
#pragma unroll
    for (int q = 0; q < M; q++) {
      R1.a[q] = R.a[q] - vinv * (Fh[q] - Fl[q]);
      ri1[q] = ring_rcp(R1.a[q]);
      rf[q] = R1.a[q];
    }
    if (C.fg) {
      R1.edges();
      F val[M];
      ppa_values(R1, C.X, val);
#pragma unroll
      for (int q = 0; q < M; q++) val[q] = C.pfac * val[q];
      // El: PPA mass flux through the zone's lower face (supplied by the
      // upstream zone of that face)
      if (C.X.right) prev_of(val, El);
      else {
#pragma unroll
        for (int q = 0; q < M; q++) El[q] = val[q];
      }
      F Eh[M];
      next_of(El, Eh);
#pragma unroll
      for (int q = 0; q < M; q++) rf[q] = R1.a[q] - vinv * (Eh[q] - El[q]);
    }
  }
  // ---- the other quantities
  F pxm[M], pxp[M];
#pragma unroll
  for (int t = 0; t < NQ; t++) {
    const int qi = ring_qorder<NQ>(t);
    Span<F, M> Qs;
    F Qv[M];
#pragma unroll
    for (int q = 0; q < M; q++) Qv[q] = Qall[t][q];
#pragma unroll
    for (int q = 0; q < M; q++) Qs.a[q] = Qv[q] * ri0[q];
    Qs.edges();
    F G[M], Gh[M];
    vlx_faces(Qs, Uw, G);
#pragma unroll
    for (int q = 0; q < M; q++) G[q] = G[q] * Fl[q];
    next_of(G, Gh);
#pragma unroll
    for (int q = 0; q < M; q++) Qv[q] = Qv[q] - vinv * (Gh[q] - G[q]);
    if (C.fg) {
#pragma unroll
      for (int q = 0; q < M; q++) Qs.a[q] = Qv[q] * ri1[q];
      Qs.edges();
      F st[M], Hl[M], Hh[M];
      ppa_values(Qs, C.X, st);
      if (C.X.right) {
        prev_of(st, Hl);
#pragma unroll
        for (int q = 0; q < M; q++) Hl[q] *= El[q];
      } else {
#pragma unroll
        for (int q = 0; q < M; q++) Hl[q] = st[q] * El[q];
      }
      next_of(Hl, Hh);
#pragma unroll
      for (int q = 0; q < M; q++) Qv[q] = Qv[q] - vinv * (Hh[q] - Hl[q]);
    }
    if (qi == 0) {
#pragma unroll
      for (int q = 0; q < M; q++) pxm[q] = Qv[q];
    } else if (qi == 1) {
#pragma unroll
      for (int q = 0; q < M; q++) pxp[q] = Qv[q];
    } else {
      F *dst = ((has_e && qi == NQ - 1) ? s.e : Tout.q[qi]) + base;
#pragma unroll
      for (int q = 0; q < M; q++)
        if (L.useful(q)) *at(dst, out_at(q)) = Qv[q];
    }
  }
  // ---- box 12d along X (Eq. 18) on the shifted ring: face i + N takes zones i - 1, i
  F pp[M], rp[M];
  prev_of(pxp, pp);
  prev_of(rf, rp);
#pragma unroll
  for (int q = 0; q < M; q++) {
    if (!L.useful(q)) continue;
    const F mom = ring_div(pp[q] + pxm[q], rp[q] + rf[q]);
    const unsigned o = out_at(q);
    // FP64: the product with the ring's 1/R; FP32 divides, since there a
    // rounded 1/R would bias v_x the same way at every step
    if constexpr (sizeof(F) == 8) *at(s.vx + base, o) = mom * C.iR - C.Rw;
    else *at(s.vx + base, o) = mom / C.R - C.Rw;
    *at(s.rho + base, o) = rf[q];
  }
}

// X transport of every active ring (2D meshes, where there is no Z sweep).
template <typename F, int NQ>
__device__ __forceinline__ void ring_x_body(Mesh m, const F *__restrict__ vx2, TSetT<F> T, TSetT<F> Tout,
                                                StateT<F> s, const double *__restrict__ v0,
                                                const double *__restrict__ dtp, int nseg, unsigned bid_, unsigned nbk_) {
  constexpr int M = RingShape<F>::M;
  const unsigned blk = xcd_remap(bid_, nbk_);
  const int lane = threadIdx.x & (WAVE - 1);
  // wave-uniform (readfirstlane), so that the ring's constants come through
  // scalar loads
  const long gw = (long)blk * (blockDim.x / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  if (gw >= (long)m.nring * nseg) return;
  const int r = (int)(gw / nseg), seg = (int)(gw % nseg);
  const int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  const unsigned base = m.o32(0, j, k);
  const RingLane<F> L(m.nx, seg, lane);
  const RingConst<F> C = ring_const<F>(m, j, k, r, *dtp, v0);
  // every load of the window is issued before the first use
  F w[M], Ra[M], Qall[NQ][M];
  L.load(T.a[T_RHO] + base, Ra);
  L.load(vx2 + base, w);
#pragma unroll
  for (int t = 0; t < NQ; t++) L.load(T.q[ring_qorder<NQ>(t)] + base, Qall[t]);
  ring_update<F, NQ>(L, C, base, Ra, w, Qall, Tout, T.a[T_E] != nullptr, s);
}
template <typename F, int NQ>
__global__ __launch_bounds__(256, 3) void k_ring_x(Mesh m, const F *__restrict__ vx2, TSetT<F> T, TSetT<F> Tout,
                                                StateT<F> s, const double *__restrict__ v0,
                                                const double *__restrict__ dtp, int nseg) {
  ring_x_body<F, NQ>(m, vx2, T, Tout, s, v0, dtp, nseg, blockIdx.x, gridDim.x);
}

// Z sweep and X transport fused (3D meshes).  A wave owns one segment of the
// rings of row j and walks up a chunk of planes.  For each of its M zones a
// lane carries the Z column window of the sweep (three zones, the slopes and
// the flux through the lower face), as a column sweep does; once the fluxes
// through face k are known the Z update of plane k - 1 is complete, and it is
// handed, in registers, to the X transport of ring (j, k - 1).  The Z-swept
// quantities never go through memory.  The halo zones of the segment are
// swept along Z as well, so segments stay independent.  The conserved
// quantities handed on are formed again as rho (Q/rho).
// Used for the FP32-bulk state, where the window and the X transport fit in
// about 160 VGPRs (three waves per SIMD); in FP64 the kernel needs about 310
// (one wave per SIMD) and the separate Z sweep and ring kernel are faster.
// Its quotients, in the Z part as in the X part, are those of ring_div.
template <typename F, int NQ>
__global__ __launch_bounds__(256, 3) void k_zx(Mesh m, const F *__restrict__ vx2, const F *__restrict__ vz,
                                            TSetT<F> T, TSetT<F> Tout, StateT<F> s, const double *__restrict__ v0,
                                            const double *__restrict__ dtp, int nseg, int nkc) {
  constexpr int M = RingShape<F>::M;
  const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & (WAVE - 1);
  const long gw = (long)blk * (blockDim.x / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  if (gw >= (long)nseg * m.ny * nkc) return;
  const int seg = (int)(gw % nseg);
  const long rest = gw / nseg;
  const int j = m.j0 + (int)(rest % m.ny), kc = (int)(rest / m.ny);
  const int a0 = m.k0 + kc * m.chunk, a1 = min(a0 + m.chunk, m.kn);
  const RingLane<F> L(m.nx, seg, lane);
  const double dtd = *dtp;
  const F dt = (F)dtd;
  const bool has_e = T.a[T_E] != nullptr;
  // a zone of the window (M columns): density, Q/rho, v_z on the lower face,
  // v_x on the lower X face (for the X transport)
  struct Zw {
    F rho[M], q[NQ][M], w[M], vx[M];
  };
  struct Zr {
    F rho[M], T[NQ][M], w[M], vx[M];
  };
  auto raw = [&](int a, Zr &z) {
    const unsigned b = m.o32(0, j, a);
    L.load_each(T.a[T_RHO] + b, z.rho);
#pragma unroll
    for (int q = 0; q < NQ; q++) L.load_each(T.q[q] + b, z.T[q]);
    L.load_each(vz + b, z.w);
    L.load_each(vx2 + b, z.vx);
  };
  auto derive = [&](const Zr &r, Zw &z) {
#pragma unroll
    for (int c = 0; c < M; c++) {
      const F ri = ring_rcp(r.rho[c]);
      z.rho[c] = r.rho[c];
      z.w[c] = r.w[c];
      z.vx[c] = r.vx[c];
#pragma unroll
      for (int q = 0; q < NQ; q++) z.q[q][c] = r.T[q][c] * ri;
    }
  };
  auto Lz = [&](int a) { return (F)m.Lz(j, a); };
  // the van Leer slopes of vl_slope and vl_slope_b with the quotient of
  // ring_div
  auto vl_slope_q = [](F qm, F q0, F qp, F hm, F hp) {
#pragma clang fp contract(off)
    const F dm = q0 - qm, dp = qp - q0, pr = dm * dp;
    return pr > F(0) ? ring_div(F(2) * pr, dm * hp + dp * hm) : F(0);
  };
  auto vl_slope_qb = [](F qm, F q0, F qp, F hm, F hp, F bm, F bp) {
#pragma clang fp contract(off)
    const F dm = (q0 - qm) + bm, dp = (qp - q0) + bp, pr = dm * dp;
    return pr > F(0) ? ring_div(F(2) * pr, dm * hp + dp * hm) : F(0);
  };
  // FP32: the X momenta (quantities 0 and 1) are deviations from a background
  // constant on each ring, as in column_sweep; dl(f) is its increment across
  // Z face f
  constexpr bool DEV = sizeof(F) == 4;
  auto dl = [&](int f) { return DEV ? (F)m.bg(BG_DLZ, j, f) : F(0); };
  auto hz = [&](int f) { return (F)m.hz(j, f); };
  Zw zm, z0, zp;
  Zr rn;
  raw(a0 - 2, rn);
  derive(rn, zp); // used only for the first slope
  raw(a0 - 1, rn);
  derive(rn, zm);
  raw(a0, rn);
  derive(rn, z0);
  raw(a0 + 1, rn);
  F sm[NQ + 1][M], s0[NQ + 1][M];
  F dlf = dl(a0); // background increment at face f
  {
    const F hm = hz(a0 - 1), hp = hz(a0), dlm = dl(a0 - 1);
#pragma unroll
    for (int c = 0; c < M; c++) {
      sm[NQ][c] = vl_slope_q(zp.rho[c], zm.rho[c], z0.rho[c], hm, hp);
#pragma unroll
      for (int q = 0; q < NQ; q++)
        sm[q][c] = (DEV && q < 2) ? vl_slope_qb(zp.q[q][c], zm.q[q][c], z0.q[q][c], hm, hp, dlm, dlf)
                                  : vl_slope_q(zp.q[q][c], zm.q[q][c], z0.q[q][c], hm, hp);
    }
  }
  F Fp[M], FQp[NQ][M];
#pragma unroll
  for (int c = 0; c < M; c++) {
    Fp[c] = F(0);
#pragma unroll
    for (int q = 0; q < NQ; q++) FQp[q][c] = F(0);
  }
  F Lm = Lz(a0 - 1);
#pragma unroll 1
  for (int f = a0; f <= a1; f++) {
    derive(rn, zp); // zone f + 1
    if (f + 2 <= a1 + 1) raw(f + 2, rn);
    const F hm = hz(f), hp = hz(f + 1), L0 = Lz(f), Sf = (F)m.Sz(j, f), dlf1 = dl(f + 1);
    F Fr[M], FQ[NQ][M];
#pragma unroll
    for (int c = 0; c < M; c++) {
      s0[NQ][c] = vl_slope_q(zm.rho[c], z0.rho[c], zp.rho[c], hm, hp);
#pragma unroll
      for (int q = 0; q < NQ; q++)
        s0[q][c] = (DEV && q < 2) ? vl_slope_qb(zm.q[q][c], z0.q[q][c], zp.q[q][c], hm, hp, dlf, dlf1)
                                  : vl_slope_q(zm.q[q][c], z0.q[q][c], zp.q[q][c], hm, hp);
      const F w = z0.w[c];
      Fr[c] = w * vl_star(w, dt, zm.rho[c], sm[NQ][c], Lm, z0.rho[c], s0[NQ][c], L0) * Sf * dt;
#pragma unroll
      for (int q = 0; q < NQ; q++) {
        // relative to the background of the face's lower zone
        const F qr = (DEV && q < 2) ? z0.q[q][c] + dlf : z0.q[q][c];
        FQ[q][c] = vl_star(w, dt, zm.q[q][c], sm[q][c], Lm, qr, s0[q][c], L0) * Fr[c];
      }
    }
    if (f > a0) {
      // Z update of plane k = f - 1, then its ring
      const int k = f - 1;
      const F vi = (F)m.Vinv(j, k);
      F Ra[M], Qall[NQ][M], w[M];
#pragma unroll
      for (int c = 0; c < M; c++) {
        Ra[c] = zm.rho[c] - vi * (Fr[c] - Fp[c]);
        w[c] = zm.vx[c];
#pragma unroll
        for (int t = 0; t < NQ; t++) {
          const int q = ring_qorder<NQ>(t);
          Qall[t][c] = zm.rho[c] * zm.q[q][c] - vi * (FQ[q][c] - FQp[q][c]);
        }
      }
      const int r = (k - m.k0) * m.ny + (j - m.j0);
      const RingConst<F> C = ring_const<F>(m, j, k, r, dtd, v0);
      ring_update<F, NQ>(L, C, m.o32(0, j, k), Ra, w, Qall, Tout, has_e, s);
    }
#pragma unroll
    for (int c = 0; c < M; c++) {
      Fp[c] = Fr[c];
#pragma unroll
      for (int q = 0; q <= NQ; q++) sm[q][c] = s0[q][c];
#pragma unroll
      for (int q = 0; q < NQ; q++) // relative to the background of the face's upper zone
        FQp[q][c] = (DEV && q < 2) ? FQ[q][c] - dlf * Fr[c] : FQ[q][c];
    }
    zm = z0;
    z0 = zp;
    Lm = L0;
    dlf = dlf1;
  }
}

// ------------------------------------------------------------------------
// 12d along Y and Z on the owned faces (Eq. 18 with Tab. "momenta").
// ------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void vel_body(Mesh m, StateT<F> s, TSetT<F> T, unsigned bid_, unsigned nbk_) {
  unsigned Lb = xcd_remap(bid_, nbk_);
  int kk = (int)(Lb % (unsigned)m.nz);
  unsigned rest = Lb / (unsigned)m.nz;
  int jj = (int)(rest % (unsigned)m.ny), ib = (int)(rest / (unsigned)m.ny);
  int i = ib * (int)blockDim.x + (int)threadIdx.x;
  if (i >= m.nx) return;
  int j = m.j0 + jj, k = m.k0 + kk;
  unsigned c = m.o32(i, j, k);
  const bool dy = j >= m.ylo(), dz = m.d3 && k >= m.zlo();
  // all loads first: the stores below may alias them as far as the compiler
  // knows, and would otherwise hold the Z loads back behind the Y store
  F rc = s.rho[c], ry = F(0), py = F(0), my = F(0), rz = F(0), pz = F(0), mz = F(0);
  if (dy) {
    const unsigned cm = m.o32(i, m.jbelow(j), k);
    ry = s.rho[cm];
    py = T.a[T_PYP][cm];
    my = T.a[T_PYM][c];
  }
  if (dz) {
    const unsigned cm = m.o32(i, j, m.kbelow(k));
    rz = s.rho[cm];
    pz = T.a[T_PZP][cm];
    mz = T.a[T_PZM][c];
  }
  if (dy) s.vy[c] = (py + my) / (ry + rc);
  if (dz) {
    F v = (pz + mz) / (rz + rc);
    s.vz[c] = m.geo == FARGO_SPHERICAL ? v / (F)m.g.ymed(j) : v;
  }
}
template <typename F>
__global__ __launch_bounds__(256) void k_vel(Mesh m, StateT<F> s, TSetT<F> T) {
  vel_body<F>(m, s, T, blockIdx.x, gridDim.x);
}

// The zones of a direction split into the fewest chunks of at most m.chunk
// zones, of equal length (the last one shorter by less than the count), so
// that the threads of a sweep end together.  Returns the mesh with the chunk
// length the kernels use, and the number of chunks.
inline Mesh balanced(const Mesh &m, int n, int &nchunk) {
  nchunk = (n + m.chunk - 1) / m.chunk;
  Mesh mm = m;
  mm.chunk = (n + nchunk - 1) / nchunk;
  return mm;
}

template <typename F, int NQ, bool D3, bool ADI>
void sweep_y_launch(Launch &L, const Mesh &m0, const StateT<F> &s, const TSetT<F> &out, const double *dt) {
  int nib, bs, nchunk;
  const Mesh m = balanced(m0, m0.ny, nchunk);
  row_blocks(m.nx, nib, bs);
  int nrows = D3 ? m.nz + 4 : 1;
  unsigned nb = (unsigned)nib * (unsigned)nchunk * (unsigned)nrows;
  k_sweep_y<F, NQ, D3, ADI><<<nb, bs, 0, L.s>>>(m, s.rho, s.vx, s.vy, s.vz, s.e, out, dt, nchunk);
}

template <typename F, int NQ>
void sweep_z_launch(Launch &L, const Mesh &m0, const F *vz, const TSetT<F> &in, const TSetT<F> &out, const double *dt) {
  int nib, bs, nchunk;
  const Mesh m = balanced(m0, m0.nz, nchunk);
  row_blocks(m.nx, nib, bs);
  unsigned nb = (unsigned)nib * (unsigned)nchunk * (unsigned)m.ny;
  k_sweep_z<F, NQ><<<nb, bs, 0, L.s>>>(m, vz, in, out, dt, nchunk);
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

// Waves of 64 lanes, four per block; ceil(nx / U) waves per ring.
template <typename F>
void launch_ring_x(Launch &L, const Mesh &m, const F *vx2, const TSetT<F> &T, const TSetT<F> &Tout,
                   const StateT<F> &s, const double *v0, const double *dt) {
  constexpr int U = (WAVE - RingShape<F>::HLL - RingShape<F>::HRL) * RingShape<F>::M;
  const int nseg = (m.nx + U - 1) / U;
  const long waves = (long)m.nring * nseg;
  const unsigned nb = (unsigned)((waves + 3) / 4);
  prof_begin(L, K_RING_X);
  switch (T.nq) { // Pi-+_x, Pi-+_y [, Pi-+_z] [, e]
  case 4: k_ring_x<F, 4><<<nb, 256, 0, L.s>>>(m, vx2, T, Tout, s, v0, dt, nseg); break;
  case 5: k_ring_x<F, 5><<<nb, 256, 0, L.s>>>(m, vx2, T, Tout, s, v0, dt, nseg); break;
  case 6: k_ring_x<F, 6><<<nb, 256, 0, L.s>>>(m, vx2, T, Tout, s, v0, dt, nseg); break;
  default: k_ring_x<F, 7><<<nb, 256, 0, L.s>>>(m, vx2, T, Tout, s, v0, dt, nseg); break;
  }
  prof_end(L, K_RING_X);
}

// Fused Z sweep and X transport: one wave per (segment, row, chunk of planes).
template <typename F>
void launch_zx(Launch &L, const Mesh &m0, const F *vx2, const F *vz, const TSetT<F> &T, const TSetT<F> &Tout,
               const StateT<F> &s, const double *v0, const double *dt) {
  constexpr int U = RingLane<F>::U;
  int nkc;
  const Mesh m = balanced(m0, m0.nz, nkc);
  const int nseg = (m.nx + U - 1) / U;
  const long waves = (long)nseg * m.ny * nkc;
  const unsigned nb = (unsigned)((waves + 3) / 4);
  prof_begin(L, K_ZX);
  if (T.nq == 7) k_zx<F, 7><<<nb, 256, 0, L.s>>>(m, vx2, vz, T, Tout, s, v0, dt, nseg, nkc);
  else k_zx<F, 6><<<nb, 256, 0, L.s>>>(m, vx2, vz, T, Tout, s, v0, dt, nseg, nkc);
  prof_end(L, K_ZX);
}

// The same with two consecutive zones per thread (16-byte loads and stores
// in FP64); rows of an even number of zones.
template <typename F>
__device__ __forceinline__ void vel2_body(Mesh m, StateT<F> s, TSetT<F> T, unsigned bid_, unsigned nbk_) {
  using V2 = typename std::conditional<sizeof(F) == 8, double2, float2>::type;
  unsigned Lb = xcd_remap(bid_, nbk_);
  int kk = (int)(Lb % (unsigned)m.nz);
  unsigned rest = Lb / (unsigned)m.nz;
  int jj = (int)(rest % (unsigned)m.ny), ib = (int)(rest / (unsigned)m.ny);
  int i = 2 * (ib * (int)blockDim.x + (int)threadIdx.x);
  if (i >= m.nx) return;
  int j = m.j0 + jj, k = m.k0 + kk;
  unsigned c = m.o32(i, j, k);
  const bool dy = j >= m.ylo(), dz = m.d3 && k >= m.zlo();
  auto ld = [&](const F *p, unsigned o) { return *reinterpret_cast<const V2 *>(p + o); };
  const V2 zero{F(0), F(0)};
  V2 rc = ld(s.rho, c), ry = zero, py = zero, my = zero, rz = zero, pz = zero, mz = zero;
  if (dy) {
    const unsigned cm = m.o32(i, m.jbelow(j), k);
    ry = ld(s.rho, cm);
    py = ld(T.a[T_PYP], cm);
    my = ld(T.a[T_PYM], c);
  }
  if (dz) {
    const unsigned cm = m.o32(i, j, m.kbelow(k));
    rz = ld(s.rho, cm);
    pz = ld(T.a[T_PZP], cm);
    mz = ld(T.a[T_PZM], c);
  }
  if (dy) *reinterpret_cast<V2 *>(s.vy + c) = V2{(py.x + my.x) / (ry.x + rc.x), (py.y + my.y) / (ry.y + rc.y)};
  if (dz) {
    V2 v{(pz.x + mz.x) / (rz.x + rc.x), (pz.y + mz.y) / (rz.y + rc.y)};
    if (m.geo == FARGO_SPHERICAL) {
      const F r = (F)m.g.ymed(j);
      v.x = v.x / r;
      v.y = v.y / r;
    }
    *reinterpret_cast<V2 *>(s.vz + c) = v;
  }
}
template <typename F>
__global__ __launch_bounds__(256) void k_vel2(Mesh m, StateT<F> s, TSetT<F> T) {
  vel2_body<F>(m, s, T, blockIdx.x, gridDim.x);
}

// multi-mesh forms (ManyGrid): the sweep and 12d in blocks of one wave
template <typename F>
struct SweepYArgs {
  Mesh m; // with the balanced chunk length
  const F *rho, *vx, *vy, *vz, *e;
  TSetT<F> out;
  const double *dt;
  int nchunk;
  unsigned nb;
};
template <typename F, int NQ, bool D3, bool ADI>
__global__ __launch_bounds__(256) void k_sweep_y_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const SweepYArgs<F> a = many_args<SweepYArgs<F>>(args, t.x);
  sweep_y_body<F, NQ, D3, ADI>(a.m, a.rho, a.vx, a.vy, a.vz, a.e, a.out, a.dt, a.nchunk, t.y, a.nb);
}
template <typename F>
struct RingArgs {
  Mesh m;
  const F *vx2;
  TSetT<F> T, Tout;
  StateT<F> s;
  const double *v0, *dt;
  int nseg;
  unsigned nb;
};
template <typename F, int NQ>
__global__ __launch_bounds__(256, 3) void k_ring_x_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const RingArgs<F> a = many_args<RingArgs<F>>(args, t.x);
  ring_x_body<F, NQ>(a.m, a.vx2, a.T, a.Tout, a.s, a.v0, a.dt, a.nseg, t.y, a.nb);
}
template <typename F>
struct VelArgs {
  Mesh m;
  StateT<F> s;
  TSetT<F> T;
  unsigned nb;
};
template <typename F>
__global__ __launch_bounds__(256) void k_vel_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const VelArgs<F> a = many_args<VelArgs<F>>(args, t.x);
  if (a.m.nx % 2 == 0) vel2_body<F>(a.m, a.s, a.T, t.y, a.nb); // two zones per thread
  else vel_body<F>(a.m, a.s, a.T, t.y, a.nb);
}

template <typename F>
void launch_vel(Launch &L, const Mesh &m, const StateT<F> &s, const TSetT<F> &T) {
  int nib, bs;
  prof_begin(L, K_VEL);
  if (m.nx % 2 == 0) {
    row_blocks(m.nx / 2, nib, bs);
    unsigned nb = (unsigned)nib * (unsigned)m.ny * (unsigned)m.nz;
    k_vel2<F><<<nb, bs, 0, L.s>>>(m, s, T);
  } else {
    row_blocks(m.nx, nib, bs);
    unsigned nb = (unsigned)nib * (unsigned)m.ny * (unsigned)m.nz;
    k_vel<F><<<nb, bs, 0, L.s>>>(m, s, T);
  }
  prof_end(L, K_VEL);
}

// multi-mesh launches (ManyGrid) on 2D meshes: blocks of one wave for the
// column sweep and 12d, so that narrow meshes leave few threads idle
constexpr int MANY_BS = 64;

template <typename F>
size_t sweep_y_args_bytes() { return sizeof(SweepYArgs<F>); }

template <typename F>
unsigned sweep_y_args(const Mesh &m0, const StateT<F> &s, const TSetT<F> &out, const double *dt, void *dst) {
  int nchunk;
  const Mesh m = balanced(m0, m0.ny, nchunk);
  const unsigned nb = (unsigned)((m.nx + MANY_BS - 1) / MANY_BS) * (unsigned)nchunk;
  *(SweepYArgs<F> *)dst = SweepYArgs<F>{m, s.rho, s.vx, s.vy, s.vz, s.e, out, dt, nchunk, nb};
  return nb;
}

template <typename F>
void launch_sweep_y_many(Launch &L, const Mesh &m0, const ManyGrid &g) {
  prof_begin(L, K_SWEEP_Y);
  if (m0.eos == FARGO_ADIABATIC) k_sweep_y_many<F, 5, false, true><<<g.nblk, MANY_BS, 0, L.s>>>(g.args, g.tab);
  else k_sweep_y_many<F, 4, false, false><<<g.nblk, MANY_BS, 0, L.s>>>(g.args, g.tab);
  prof_end(L, K_SWEEP_Y);
}

template <typename F>
size_t ring_x_args_bytes() { return sizeof(RingArgs<F>); }

template <typename F>
unsigned ring_x_args(const Mesh &m, const F *vx2, const TSetT<F> &T, const TSetT<F> &Tout, const StateT<F> &s,
                     const double *v0, const double *dt, void *dst) {
  constexpr int U = (WAVE - RingShape<F>::HLL - RingShape<F>::HRL) * RingShape<F>::M;
  const int nseg = (m.nx + U - 1) / U;
  const unsigned nb = (unsigned)(((long)m.nring * nseg + 3) / 4);
  *(RingArgs<F> *)dst = RingArgs<F>{m, vx2, T, Tout, s, v0, dt, nseg, nb};
  return nb;
}

template <typename F>
void launch_ring_x_many(Launch &L, int nq, const ManyGrid &g) {
  prof_begin(L, K_RING_X);
  if (nq == 5) k_ring_x_many<F, 5><<<g.nblk, 256, 0, L.s>>>(g.args, g.tab);
  else k_ring_x_many<F, 4><<<g.nblk, 256, 0, L.s>>>(g.args, g.tab);
  prof_end(L, K_RING_X);
}

template <typename F>
size_t vel_args_bytes() { return sizeof(VelArgs<F>); }

// two zones per thread on rows of an even number of zones, else one
template <typename F>
unsigned vel_args(const Mesh &m, const StateT<F> &s, const TSetT<F> &T, void *dst) {
  const int w = m.nx % 2 == 0 ? m.nx / 2 : m.nx;
  const unsigned nb = (unsigned)((w + MANY_BS - 1) / MANY_BS) * (unsigned)m.ny * (unsigned)m.nz;
  *(VelArgs<F> *)dst = VelArgs<F>{m, s, T, nb};
  return nb;
}

template <typename F>
void launch_vel_many(Launch &L, const ManyGrid &g) {
  prof_begin(L, K_VEL);
  k_vel_many<F><<<g.nblk, MANY_BS, 0, L.s>>>(g.args, g.tab);
  prof_end(L, K_VEL);
}

#define FARGO_TRANSPORT_MANY(F)                                                                                     \
  template size_t sweep_y_args_bytes<F>();                                                                         \
  template unsigned sweep_y_args<F>(const Mesh &, const StateT<F> &, const TSetT<F> &, const double *, void *);    \
  template void launch_sweep_y_many<F>(Launch &, const Mesh &, const ManyGrid &);                                  \
  template size_t ring_x_args_bytes<F>();                                                                          \
  template unsigned ring_x_args<F>(const Mesh &, const F *, const TSetT<F> &, const TSetT<F> &, const StateT<F> &, \
                                   const double *, const double *, void *);                                        \
  template void launch_ring_x_many<F>(Launch &, int, const ManyGrid &);                                            \
  template size_t vel_args_bytes<F>();                                                                             \
  template unsigned vel_args<F>(const Mesh &, const StateT<F> &, const TSetT<F> &, void *);                        \
  template void launch_vel_many<F>(Launch &, const ManyGrid &);
FARGO_TRANSPORT_MANY(double)
FARGO_TRANSPORT_MANY(float)
#undef FARGO_TRANSPORT_MANY

#define FARGO_TRANSPORT_INST(F)                                                                                    \
  template void launch_sweep_y<F>(Launch &, const Mesh &, const StateT<F> &, const TSetT<F> &, const double *);   \
  template void launch_sweep_z<F>(Launch &, const Mesh &, const F *, const TSetT<F> &, const TSetT<F> &,         \
                                  const double *);                                                               \
  template void launch_ring_x<F>(Launch &, const Mesh &, const F *, const TSetT<F> &, const TSetT<F> &,         \
                                 const StateT<F> &, const double *, const double *);                             \
  template void launch_vel<F>(Launch &, const Mesh &, const StateT<F> &, const TSetT<F> &);
FARGO_TRANSPORT_INST(double)
FARGO_TRANSPORT_INST(float)
#undef FARGO_TRANSPORT_INST
template void launch_zx<float>(Launch &, const Mesh &, const float *, const float *, const TSetT<float> &,
                               const TSetT<float> &, const StateT<float> &, const double *, const double *);

} // namespace fargo
