// Box 3 (bulk azimuthal velocity per ring, Eq. 37), box 6 (time step,
// Eq. cfl2 items 1-3, Eq. 38) and the orbital-advection split of Eq. 29.
//
// One workgroup per active ring computes the ring's v0 and, for each of its
// zones, the cell time step and the shear rate; the ring minimum/maximum goes
// to a per-ring slot.  A single workgroup then reduces the slots (exact and
// order independent: min/max) and forms dt.  The split of every ring's
// displacement into (N, xi) is taken by the ring kernel of the X transport
// (and by k_split for the stand-alone entry point).  The time step and the
// split use floating-point contraction off and the operation order of the
// written definition, so that the integer shift N is reproducible bit for bit.
#include "fargo_internal.h"

namespace fargo {

namespace {

constexpr int MAXW = 16; // waves per block, at most

template <typename Op>
__device__ inline double block_reduce(double v, Op op, double id, double *lds) {
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  int nw = (blockDim.x + 63) >> 6;
  v = lane < nw ? lds[lane] : id;
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  return v; // valid in every lane
}

// A lane move of a double by DPP (two 32-bit moves); lanes with no source
// lane, and the rows the row mask leaves out, take id.
template <int CTRL, int RM = 0xf>
__device__ inline double dpp_or(double x, double id) {
  const long long xv = __double_as_longlong(x), iv = __double_as_longlong(id);
  const int lo = __builtin_amdgcn_update_dpp((int)iv, (int)xv, CTRL, RM, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(iv >> 32), (int)(xv >> 32), CTRL, RM, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// The maximum or minimum of a wave's 64 values, in lane 63, by VALU lane
// moves alone: shifts by 1, 2, 4 and 8 within each row of 16 lanes (lane 15
// of a row then holds the row's result), then the broadcasts of lane 15 into
// rows 1 and 3 and of lane 31 into rows 2 and 3.  Exact in any order, so it
// serves min and max only.
template <typename Op>
__device__ inline double wave_reduce_dpp(double v, Op op, double id) {
  constexpr int ROW_SHR = 0x110, ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
  v = op(v, dpp_or<ROW_SHR + 1>(v, id));
  v = op(v, dpp_or<ROW_SHR + 2>(v, id));
  v = op(v, dpp_or<ROW_SHR + 4>(v, id));
  v = op(v, dpp_or<ROW_SHR + 8>(v, id));
  v = op(v, dpp_or<ROW_BCAST15, 0xa>(v, id));
  v = op(v, dpp_or<ROW_BCAST31, 0xc>(v, id));
  return v;
}

// Two reductions of a block at once (min or max: exact in any order), with
// two barriers for both: each wave reduces by DPP lane moves, its lane 63
// puts the result in LDS, and every lane then reads the waves' results and
// reduces them itself; lds holds 2 * MAXW values.  With `flag`, the OR of
// every thread's *flag rides along (a wave ballot, then MAXW more values of
// lds) and is left in *flag of every thread.
template <typename OpA, typename OpB>
__device__ inline void block_reduce2(double &a, OpA opa, double ida, double &b, OpB opb, double idb, double *lds,
                                     int *flag = nullptr) {
  a = wave_reduce_dpp(a, opa, ida);
  b = wave_reduce_dpp(b, opb, idb);
  const bool fw = flag && __builtin_amdgcn_ballot_w64(*flag != 0) != 0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 63) {
    lds[wid] = a;
    lds[MAXW + wid] = b;
    if (flag) lds[2 * MAXW + wid] = fw ? 1.0 : 0.0;
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  a = ida;
  b = idb;
  int f = 0;
  for (int w = 0; w < nw; w++) {
    a = opa(a, lds[w]);
    b = opb(b, lds[MAXW + w]);
    if (flag) f |= lds[2 * MAXW + w] != 0.0;
  }
  if (flag) *flag = f;
}

struct Max { __device__ double operator()(double a, double b) const { return a > b ? a : b; } };
struct Min { __device__ double operator()(double a, double b) const { return a < b ? a : b; } };
struct Add { __device__ double operator()(double a, double b) const { return a + b; } };

__global__ void k_set_dt(DevWords w, double dt) { *w.dt = dt; }

// Bulk velocity of a ring (max/min exact; the mean in a fixed tree order).
template <int M>
__device__ inline double ring_bulk(const Mesh &m, const double (&v)[M], int tid, double *lds) {
  const int B = blockDim.x;
  if (m.v0_mean) {
    double s = 0.0;
#pragma unroll
    for (int mm = 0; mm < M; mm++)
      if (tid + B * mm < m.nx) s += v[mm];
    return block_reduce(s, Add(), 0.0, lds) / m.nx;
  }
  double vmax = -HUGE_VAL, vmin = HUGE_VAL;
#pragma unroll
  for (int mm = 0; mm < M; mm++)
    if (tid + B * mm < m.nx) {
      vmax = v[mm] > vmax ? v[mm] : vmax;
      vmin = v[mm] < vmin ? v[mm] : vmin;
    }
  block_reduce2(vmax, Max(), -HUGE_VAL, vmin, Min(), HUGE_VAL, lds);
  return 0.5 * (vmax + vmin);
}

// Constants of Eq. cfl2 for ring (j, k): lengths and their reciprocals.
struct CflRing {
  double Lx, iLx, iLy, iLz, iL2, k3, dXp;
};
__device__ inline CflRing cfl_ring(const Mesh &m, int j, int k, bool shear_on) {
#pragma clang fp contract(off)
  CflRing C;
  const double Lyy = m.g.Ly(j), Lzz = m.d3 ? m.Lz(j, k) : 0.0;
  C.Lx = m.DX(j, k);
  C.iLx = 1.0 / C.Lx;
  C.iLy = 1.0 / Lyy;
  C.iLz = m.d3 ? 1.0 / Lzz : 0.0;
  double Lmin = fmin(C.Lx, Lyy);
  if (m.d3) Lmin = fmin(Lmin, Lzz);
  C.iL2 = 1.0 / (Lmin * Lmin);
  C.k3 = 4.0 * m.cvnr * m.cvnr;
  C.dXp = shear_on ? m.DX(j + 1, k) : 1.0;
  return C;
}

// Eq. cfl2 for one zone through the inverse steps (rates u / Delta): the
// minimum step of a cell over directions is its maximum rate; returns the sum
// of the squared rates of items 1-3 (and 4 with viscosity), and flags a
// non-finite or non-positive state in `bad`.  q: sound speed (isothermal)
// or internal energy; vxc, vxp: full v_x on the zone's two X faces; vb: the
// ring's bulk velocity (0 without orbital advection).
__device__ inline double zone_rate2(const Mesh &m, const CflRing &C, double vb, double vxc, double vxp, double rho,
                                    double q, double vyc, double vyp, double vzc, double vzp, double nu, int &bad) {
#pragma clang fp contract(off)
  double cw2; // squared wave speed
  if (m.eos == FARGO_ISOTHERMAL) cw2 = q * q;
  else cw2 = m.gamma * ((m.gamma - 1.0) * q) / rho;
  bad |= !(rho > 0.0) || !isfinite(rho) || !isfinite(cw2) || !isfinite(vxc) || !isfinite(vyc);
  // item 1: sound waves (squared rate); item 2: fluid motion; item 3:
  // artificial viscosity on compressed directions
  const double r1s = cw2 * C.iL2;
  const double ux = fmax(fabs(vxc - vb), fabs(vxp - vb));
  const double uy = fmax(fabs(vyc), fabs(vyp));
  double r2 = fmax(ux * C.iLx, uy * C.iLy);
  const double dvx = vxp - vxc, dvy = vyp - vyc;
  double r3 = 0.0;
  if (dvx < 0.0) r3 = fmax(r3, C.k3 * fabs(dvx) * C.iLx);
  if (dvy < 0.0) r3 = fmax(r3, C.k3 * fabs(dvy) * C.iLy);
  if (m.d3) {
    bad |= !isfinite(vzc);
    const double uz = fmax(fabs(vzc), fabs(vzp));
    r2 = fmax(r2, uz * C.iLz);
    const double dvz = vzp - vzc;
    if (dvz < 0.0) r3 = fmax(r3, C.k3 * fabs(dvz) * C.iLz);
  }
  double rate2 = r1s + r2 * r2 + r3 * r3;
  if (m.visc) { // item 4: viscosity, 4 nu / Delta^2
    const double r4 = 4.0 * nu * C.iL2;
    rate2 += r4 * r4;
  }
  if (!(rate2 >= 0.0)) bad = 1;
  return rate2;
}

// Rings in XCD-contiguous logical order, by tiles of 16 planes with k fastest
// within a tile: the rings holding a ring's k + 1 and j + 1 neighbours (v_z
// and v_y on its upper faces) were read one and 16 rings earlier, still in L2
// except across a tile boundary.  M zones per thread.
// The state may be stored in FP32 (R = float); the time step is always formed
// in FP64 from the stored values.
template <int M, typename R, int NB>
__device__ __forceinline__ void cfl_ring_body(Mesh m, StateT<R> s, int with_cfl, double *__restrict__ v0,
                                                  double *__restrict__ ringrate, double *__restrict__ ringshear,
                                                  int *__restrict__ err, unsigned bid_, unsigned nbk_) {
#pragma clang fp contract(off)
  extern __shared__ double V[]; // the ring's v_x
  __shared__ double red[3 * MAXW];
  const unsigned L = xcd_remap(bid_, nbk_);
  constexpr int KT = 16;
  const unsigned tile = L / ((unsigned)m.ny * KT), q = L % ((unsigned)m.ny * KT);
  const int kb = (int)tile * KT, kt = min(KT, m.nz - kb);
  const int kk = kb + (int)(q % (unsigned)kt), jj = (int)(q / (unsigned)kt);
  const int j = m.j0 + jj, k = m.k0 + kk;
  const int r = kk * m.ny + jj; // ring index (k - k0) * ny + (j - j0)
  const int tid = threadIdx.x, B = blockDim.x, n = m.nx;
  const unsigned base = m.o32(0, j, k);
  const bool shear_on = with_cfl && m.fargo && m.shear_c0 > 0.0 && j + 1 < m.jn;
  const unsigned py = (unsigned)m.pitch, pz = (unsigned)m.plane();
  // Every load of the ring is issued before the first use (indices clamped
  // to the ring, so no load sits behind a branch), which keeps all of them
  // in flight together.
  const R *qf = m.eos == FARGO_ISOTHERMAL ? s.cs : s.e;
  R fx[M], fr[M] = {}, fq[M] = {}, fy0[M] = {}, fy1[M] = {}, fz0[M] = {}, fz1[M] = {}, fn[M] = {}, fs[M] = {};
#pragma unroll
  for (int mm = 0; mm < M; mm++) {
    const unsigned c = base + (unsigned)min(tid + B * mm, n - 1);
    fx[mm] = s.vx[c];
    if (with_cfl) {
      fr[mm] = s.rho[c];
      fq[mm] = qf[c];
      fy0[mm] = s.vy[c];
      fy1[mm] = s.vy[c + py];
      if (m.d3) {
        fz0[mm] = s.vz[c];
        fz1[mm] = s.vz[c + pz];
      }
      if (m.visc) fn[mm] = s.nu[c];
      if (shear_on) fs[mm] = s.vx[c + py];
    }
  }
  // an FP32 v_x is a deviation from the ring's FP64 background: the full
  // velocity is formed in FP64
  double vbg = 0.0, vbg_p = 0.0;
  if constexpr (sizeof(R) == 4) {
    vbg = m.bg(BG_V, j, k);
    if (shear_on) vbg_p = m.bg(BG_V, j + 1, k);
  }
  double vx[M];
#pragma unroll
  for (int mm = 0; mm < M; mm++) {
    int i = tid + B * mm;
    vx[mm] = i < n ? (double)fx[mm] + vbg : 0.0;
    if (i < n) V[i] = vx[mm];
  }
  // the barriers of the reduction also make V visible to the block
  const double vb_ring = ring_bulk<M>(m, vx, tid, red);
  if (tid == 0) v0[r] = vb_ring;
  if (!with_cfl) return;
  const double vb = m.fargo ? vb_ring : 0.0;
  // the smallest step is 1 / sqrt of the largest sum of squared rates (taken
  // in k_dt_final)
  const CflRing C = cfl_ring(m, j, k, shear_on);
  double rmax = 0.0, smax = 0.0;
  int bad = 0;
#pragma unroll
  for (int mm = 0; mm < M; mm++) {
    int i = tid + B * mm;
    if (i >= n) continue;
    const double vxc = vx[mm], vxp = V[i + 1 == n ? 0 : i + 1];
    const double rate2 = zone_rate2(m, C, vb, vxc, vxp, (double)fr[mm], (double)fq[mm], (double)fy0[mm],
                                    (double)fy1[mm], (double)fz0[mm], (double)fz1[mm], (double)fn[mm], bad);
    if (rate2 >= 0.0) rmax = rate2 > rmax ? rate2 : rmax;
    if (shear_on) {
      double sh = fabs(vxc / C.Lx - ((double)fs[mm] + vbg_p) / C.dXp);
      if (sh > smax) smax = sh;
    }
  }
  int anybad = bad;
  block_reduce2(rmax, Max(), 0.0, smax, Max(), 0.0, red, &anybad);
  if (tid == 0) {
    ringrate[r] = rmax; // the ring's largest squared rate
    ringshear[r] = smax;
    if (anybad) atomicOr(err, 1);
  }
}
template <int M, typename R, int NB>
__global__ __launch_bounds__(NB) void k_cfl_ring(Mesh m, StateT<R> s, int with_cfl, double *__restrict__ v0,
                                                  double *__restrict__ ringrate, double *__restrict__ ringshear,
                                                  int *__restrict__ err) {
  cfl_ring_body<M, R, NB>(m, s, with_cfl, v0, ringrate, ringshear, err, blockIdx.x, gridDim.x);
}

// Rings longer than one workgroup holds, in segments of CFL_SEG zones (256
// threads, four zones each).  First each segment's largest and smallest
// full v_x (or its sum, for the mean), then each segment combines its ring's
// entries into v0 (min/max exactly as in ring_bulk; the mean as the sum of the
// segment sums in segment order, over nx) and takes Eq. cfl2 on its zones,
// with the v_x of the zone after its last read from memory.
template <typename R>
__device__ inline double full_vx(const Mesh &m, const StateT<R> &s, unsigned c, double vbg) {
  return (double)s.vx[c] + vbg;
}

template <typename R>
__global__ __launch_bounds__(256) void k_bulk_seg(Mesh m, StateT<R> s) {
  constexpr int M = CFL_SEG / 256;
  __shared__ double red[2 * MAXW];
  const int r = (int)(blockIdx.x / (unsigned)m.cseg), g = (int)(blockIdx.x % (unsigned)m.cseg);
  const int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  const unsigned base = m.o32(0, j, k);
  const double vbg = sizeof(R) == 4 ? m.bg(BG_V, j, k) : 0.0;
  const int i0 = g * CFL_SEG, i1 = min(i0 + CFL_SEG, m.nx);
  double a = m.v0_mean ? 0.0 : -HUGE_VAL, b = HUGE_VAL;
#pragma unroll
  for (int mm = 0; mm < M; mm++) {
    const int i = i0 + (int)threadIdx.x + 256 * mm;
    if (i >= i1) continue;
    const double v = full_vx(m, s, base + (unsigned)i, vbg);
    if (m.v0_mean) a += v;
    else {
      a = v > a ? v : a;
      b = v < b ? v : b;
    }
  }
  if (m.v0_mean) {
    a = block_reduce(a, Add(), 0.0, red);
    b = 0.0;
  } else {
    block_reduce2(a, Max(), -HUGE_VAL, b, Min(), HUGE_VAL, red);
  }
  if (threadIdx.x == 0) {
    m.segmm[2 * (size_t)blockIdx.x] = a;
    m.segmm[2 * (size_t)blockIdx.x + 1] = b;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_cfl_seg(Mesh m, StateT<R> s, int with_cfl, double *__restrict__ v0,
                                                 double *__restrict__ ringrate, double *__restrict__ ringshear,
                                                 int *__restrict__ err) {
#pragma clang fp contract(off)
  constexpr int M = CFL_SEG / 256;
  __shared__ double red[3 * MAXW];
  __shared__ double V[CFL_SEG + 1]; // the segment's full v_x and the next zone's
  const int r = (int)(blockIdx.x / (unsigned)m.cseg), g = (int)(blockIdx.x % (unsigned)m.cseg);
  const int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  const int tid = threadIdx.x, n = m.nx;
  const unsigned base = m.o32(0, j, k);
  const bool shear_on = with_cfl && m.fargo && m.shear_c0 > 0.0 && j + 1 < m.jn;
  double vbg = 0.0, vbg_p = 0.0;
  if constexpr (sizeof(R) == 4) {
    vbg = m.bg(BG_V, j, k);
    if (shear_on) vbg_p = m.bg(BG_V, j + 1, k);
  }
  // the ring's bulk velocity from its segments' entries
  double a = m.v0_mean ? 0.0 : -HUGE_VAL, b = HUGE_VAL;
  const double *e = m.segmm + 2 * (size_t)r * m.cseg;
  if (m.v0_mean) {
    if (tid == 0)
      for (int q = 0; q < m.cseg; q++) a += e[2 * q];
    a = block_reduce(tid == 0 ? a : 0.0, Add(), 0.0, red);
  } else {
    for (int q = tid; q < m.cseg; q += 256) {
      a = e[2 * q] > a ? e[2 * q] : a;
      b = e[2 * q + 1] < b ? e[2 * q + 1] : b;
    }
    block_reduce2(a, Max(), -HUGE_VAL, b, Min(), HUGE_VAL, red);
  }
  const double vb_ring = m.v0_mean ? a / n : 0.5 * (a + b);
  if (g == 0 && tid == 0) v0[r] = vb_ring;
  if (!with_cfl) return;
  const int i0 = g * CFL_SEG, i1 = min(i0 + CFL_SEG, n);
  for (int i = i0 + tid; i <= i1; i += 256) V[i - i0] = full_vx(m, s, base + (unsigned)(i == n ? 0 : i), vbg);
  __syncthreads();
  const double vb = m.fargo ? vb_ring : 0.0;
  const CflRing C = cfl_ring(m, j, k, shear_on);
  const unsigned py = (unsigned)m.pitch, pz = (unsigned)m.plane();
  const R *qf = m.eos == FARGO_ISOTHERMAL ? s.cs : s.e;
  double rmax = 0.0, smax = 0.0;
  int bad = 0;
#pragma unroll
  for (int mm = 0; mm < M; mm++) {
    const int i = i0 + tid + 256 * mm;
    if (i >= i1) continue;
    const unsigned c = base + (unsigned)i;
    const double vxc = V[i - i0], vxp = V[i - i0 + 1];
    const double rate2 = zone_rate2(m, C, vb, vxc, vxp, (double)s.rho[c], (double)qf[c], (double)s.vy[c],
                                    (double)s.vy[c + py], m.d3 ? (double)s.vz[c] : 0.0,
                                    m.d3 ? (double)s.vz[c + pz] : 0.0, m.visc ? (double)s.nu[c] : 0.0, bad);
    if (rate2 >= 0.0) rmax = rate2 > rmax ? rate2 : rmax;
    if (shear_on) {
      const double sh = fabs(vxc / C.Lx - ((double)s.vx[c + py] + vbg_p) / C.dXp);
      if (sh > smax) smax = sh;
    }
  }
  int anybad = bad;
  block_reduce2(rmax, Max(), 0.0, smax, Max(), 0.0, red, &anybad);
  if (tid == 0) {
    ringrate[blockIdx.x] = rmax;
    ringshear[blockIdx.x] = smax;
    if (anybad) atomicOr(err, 1);
  }
}

// One workgroup: dt from the ring slots (or the imposed value), then the split
// of every ring.  A non-positive or non-finite dt is flagged and replaced by 0,
// which leaves the state unchanged.
__device__ __forceinline__ void dt_final_body(const Mesh &m, const DevWords &w, const double *__restrict__ ringrate,
                                              const double *__restrict__ ringshear) {
#pragma clang fp contract(off)
  __shared__ double red[2 * MAXW];
  constexpr int U = 8; // loads in flight per thread
  double rmax = 0.0, smax = 0.0;
  const int nslot = m.nring * m.cseg;
  for (int r0 = threadIdx.x; r0 < nslot; r0 += U * blockDim.x) {
    double a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int r = r0 + u * (int)blockDim.x;
      a[u] = r < nslot ? ringrate[r] : 0.0;
      b[u] = r < nslot ? ringshear[r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      rmax = a[u] > rmax ? a[u] : rmax;
      smax = b[u] > smax ? b[u] : smax;
    }
  }
  block_reduce2(rmax, Max(), 0.0, smax, Max(), 0.0, red);
  if (threadIdx.x == 0) {
    double dt = m.courant * (1.0 / sqrt(rmax));
    if (m.fargo && m.shear_c0 > 0.0 && smax > 0.0) dt = fmin(dt, m.shear_c0 / smax);
    if (!(dt > 0.0) || !isfinite(dt)) {
      atomicOr(w.err, 2);
      dt = 0.0;
    }
    *w.dt = dt;
  }
}
__global__ __launch_bounds__(1024) void k_dt_final(Mesh m, DevWords w, const double *__restrict__ ringrate,
                                                   const double *__restrict__ ringshear) {
  dt_final_body(m, w, ringrate, ringshear);
}

// multi-mesh forms (ManyGrid)
template <typename R>
struct CflArgs {
  Mesh m;
  StateT<R> s;
  double *v0, *ringrate, *ringshear;
  int *err;
  unsigned nb;
};
template <int M, typename R>
__global__ __launch_bounds__(256) void k_cfl_ring_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const CflArgs<R> a = many_args<CflArgs<R>>(args, t.x);
  cfl_ring_body<M, R, 256>(a.m, a.s, 1, a.v0, a.ringrate, a.ringshear, a.err, t.y, a.nb);
}
struct DtArgs {
  Mesh m;
  DevWords w;
  const double *ringrate, *ringshear;
};
__global__ __launch_bounds__(1024) void k_dt_final_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const DtArgs a = many_args<DtArgs>(args, t.x);
  dt_final_body(a.m, a.w, a.ringrate, a.ringshear);
}

// The split of Eq. 29, one thread per ring, with dt given by value or, if
// dtp is not null, read from the device.
__global__ __launch_bounds__(256) void k_split(Mesh m, const double *__restrict__ v0, const double *__restrict__ dtp,
                                               double dtv, int32_t *__restrict__ N, double *__restrict__ xi) {
#pragma clang fp contract(off)
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m.nring) return;
  const double dt = dtp ? *dtp : dtv;
  int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  double D = (v0[r] * dt) / m.DX(j, k);
  double rn = round(D);
  N[r] = (int32_t)rn;
  xi[r] = D - rn;
}

// NB threads per ring: 256 up to 2048 zones, 512 up to 4096
template <int M, typename R, int NB = 256>
void cfl_launch(Launch &L, const Mesh &m, const StateT<R> &s, int with_cfl, double *v0, double *rmin, double *rsh,
                int *err) {
  k_cfl_ring<M, R, NB><<<m.nring, NB, (size_t)m.nx * sizeof(double), L.s>>>(m, s, with_cfl, v0, rmin, rsh, err);
}

} // namespace

void launch_set_dt(Launch &L, const DevWords &w, double dt) {
  prof_begin(L, K_SET_DT);
  k_set_dt<<<1, 1, 0, L.s>>>(w, dt);
  prof_end(L, K_SET_DT);
}

template <typename R>
void launch_cfl(Launch &L, const Mesh &m, const StateT<R> &s, int with_cfl, double *v0, double *ringrate,
                double *ringshear, int *err) {
  prof_begin(L, K_CFL);
  if (m.cseg > 1) { // rings in segments
    const unsigned nb = (unsigned)m.nring * (unsigned)m.cseg;
    k_bulk_seg<R><<<nb, 256, 0, L.s>>>(m, s);
    k_cfl_seg<R><<<nb, 256, 0, L.s>>>(m, s, with_cfl, v0, ringrate, ringshear, err);
    prof_end(L, K_CFL);
    return;
  }
  if (m.nx > 1792 && m.nx <= 2048) { // 512 threads of 4 zones
    cfl_launch<4, R, 512>(L, m, s, with_cfl, v0, ringrate, ringshear, err);
    prof_end(L, K_CFL);
    return;
  }
  if (m.nx > 2048) { // nx <= 4096: 512 threads, 5 to 8 zones each
    switch ((m.nx + 511) / 512) {
    case 5: cfl_launch<5, R, 512>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
    case 6: cfl_launch<6, R, 512>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
    case 7: cfl_launch<7, R, 512>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
    default: cfl_launch<8, R, 512>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
    }
    prof_end(L, K_CFL);
    return;
  }
  switch ((m.nx + 255) / 256) { // zones per thread
  case 1: cfl_launch<1, R>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
  case 2: cfl_launch<2, R>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
  case 3: cfl_launch<3, R>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
  case 4: cfl_launch<4, R>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
  case 5: cfl_launch<5, R>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
  case 6: cfl_launch<6, R>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
  case 7: cfl_launch<7, R>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
  default: cfl_launch<8, R>(L, m, s, with_cfl, v0, ringrate, ringshear, err); break;
  }
  prof_end(L, K_CFL);
}

template void launch_cfl<double>(Launch &, const Mesh &, const StateT<double> &, int, double *, double *, double *,
                                 int *);
template void launch_cfl<float>(Launch &, const Mesh &, const StateT<float> &, int, double *, double *, double *,
                                int *);

void launch_dt_final(Launch &L, const Mesh &m, const DevWords &w, const double *ringrate, const double *ringshear,
                     int use_given) {
  if (use_given) return;
  prof_begin(L, K_DT_FINAL);
  k_dt_final<<<1, 1024, 0, L.s>>>(m, w, ringrate, ringshear);
  prof_end(L, K_DT_FINAL);
}

void launch_split(Launch &L, const Mesh &m, const double *v0, double dt, int32_t *N, double *xi) {
  prof_begin(L, K_SPLIT);
  k_split<<<(m.nring + 255) / 256, 256, 0, L.s>>>(m, v0, nullptr, dt, N, xi);
  prof_end(L, K_SPLIT);
}

template <typename R>
size_t cfl_args_bytes() { return sizeof(CflArgs<R>); }

template <typename R>
unsigned cfl_args(const Mesh &m, const StateT<R> &s, double *v0, double *ringrate, double *ringshear, int *err,
                  void *dst) {
  *(CflArgs<R> *)dst = CflArgs<R>{m, s, v0, ringrate, ringshear, err, (unsigned)m.nring};
  return (unsigned)m.nring;
}

// rings of at most 1792 zones: 256 threads of M = ceil(nxmax / 256) zones for
// every mesh of the launch (a shorter ring leaves some of them idle)
template <typename R>
void launch_cfl_many(Launch &L, const ManyGrid &g, int nxmax) {
  prof_begin(L, K_CFL);
  const size_t sh = (size_t)nxmax * sizeof(double);
  switch ((nxmax + 255) / 256) {
  case 1: k_cfl_ring_many<1, R><<<g.nblk, 256, sh, L.s>>>(g.args, g.tab); break;
  case 2: k_cfl_ring_many<2, R><<<g.nblk, 256, sh, L.s>>>(g.args, g.tab); break;
  case 3: k_cfl_ring_many<3, R><<<g.nblk, 256, sh, L.s>>>(g.args, g.tab); break;
  case 4: k_cfl_ring_many<4, R><<<g.nblk, 256, sh, L.s>>>(g.args, g.tab); break;
  case 5: k_cfl_ring_many<5, R><<<g.nblk, 256, sh, L.s>>>(g.args, g.tab); break;
  case 6: k_cfl_ring_many<6, R><<<g.nblk, 256, sh, L.s>>>(g.args, g.tab); break;
  default: k_cfl_ring_many<7, R><<<g.nblk, 256, sh, L.s>>>(g.args, g.tab); break;
  }
  prof_end(L, K_CFL);
}

size_t dt_final_args_bytes() { return sizeof(DtArgs); }

unsigned dt_final_args(const Mesh &m, const DevWords &w, const double *ringrate, const double *ringshear, void *dst) {
  *(DtArgs *)dst = DtArgs{m, w, ringrate, ringshear};
  return 1;
}

void launch_dt_final_many(Launch &L, const ManyGrid &g) {
  prof_begin(L, K_DT_FINAL);
  k_dt_final_many<<<g.nblk, 1024, 0, L.s>>>(g.args, g.tab);
  prof_end(L, K_DT_FINAL);
}

template unsigned cfl_args<double>(const Mesh &, const StateT<double> &, double *, double *, double *, int *, void *);
template unsigned cfl_args<float>(const Mesh &, const StateT<float> &, double *, double *, double *, int *, void *);
template size_t cfl_args_bytes<double>();
template size_t cfl_args_bytes<float>();
template void launch_cfl_many<double>(Launch &, const ManyGrid &, int);
template void launch_cfl_many<float>(Launch &, const ManyGrid &, int);

} // namespace fargo
