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

// Two reductions of a block at once (two barriers for both); lds holds
// 2 * MAXW values.
template <typename OpA, typename OpB>
__device__ inline void block_reduce2(double &a, OpA opa, double ida, double &b, OpB opb, double idb, double *lds) {
  for (int o = 32; o > 0; o >>= 1) {
    a = opa(a, __shfl_xor(a, o, 64));
    b = opb(b, __shfl_xor(b, o, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    lds[wid] = a;
    lds[MAXW + wid] = b;
  }
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  a = lane < nw ? lds[lane] : ida;
  b = lane < nw ? lds[MAXW + lane] : idb;
  for (int o = 32; o > 0; o >>= 1) {
    a = opa(a, __shfl_xor(a, o, 64));
    b = opb(b, __shfl_xor(b, o, 64));
  }
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

// Rings in XCD-contiguous logical order, by tiles of 16 planes with k fastest
// within a tile: the rings holding a ring's k + 1 and j + 1 neighbours (v_z
// and v_y on its upper faces) were read one and 16 rings earlier, still in L2
// except across a tile boundary.  M zones per thread.
// The state may be stored in FP32 (R = float); the time step is always formed
// in FP64 from the stored values.
template <int M, typename R, int NB>
__global__ __launch_bounds__(NB) void k_cfl_ring(Mesh m, StateT<R> s, int with_cfl, double *__restrict__ v0,
                                                  double *__restrict__ ringrate, double *__restrict__ ringshear,
                                                  int *__restrict__ err) {
#pragma clang fp contract(off)
  extern __shared__ double V[]; // the ring's v_x
  __shared__ double red[2 * MAXW];
  const unsigned L = xcd_remap(blockIdx.x, gridDim.x);
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
  // Eq. cfl2 through the inverse steps (rates u / Delta): the minimum step of
  // a cell over directions is its maximum rate, and the smallest step is
  // 1 / sqrt of the largest sum of squared rates (taken in k_dt_final)
  const double Lx = m.DX(j, k), Lyy = m.g.Ly(j);
  const double Lzz = m.d3 ? m.Lz(j, k) : 0.0;
  const double iLx = 1.0 / Lx, iLy = 1.0 / Lyy, iLz = m.d3 ? 1.0 / Lzz : 0.0;
  double Lmin = fmin(Lx, Lyy);
  if (m.d3) Lmin = fmin(Lmin, Lzz);
  const double iL2 = 1.0 / (Lmin * Lmin);
  const double k3 = 4.0 * m.cvnr * m.cvnr;
  const double dXp = shear_on ? m.DX(j + 1, k) : 1.0;
  double rmax = 0.0, smax = 0.0;
  int bad = 0;
#pragma unroll
  for (int mm = 0; mm < M; mm++) {
    int i = tid + B * mm;
    if (i >= n) continue;
    double vxc = vx[mm], vxp = V[i + 1 == n ? 0 : i + 1];
    double rho = (double)fr[mm];
    double cw2; // squared wave speed
    if (m.eos == FARGO_ISOTHERMAL) cw2 = (double)fq[mm] * (double)fq[mm];
    else cw2 = m.gamma * ((m.gamma - 1.0) * (double)fq[mm]) / rho;
    double vyc = (double)fy0[mm], vyp = (double)fy1[mm];
    bad |= !(rho > 0.0) || !isfinite(rho) || !isfinite(cw2) || !isfinite(vxc) || !isfinite(vyc);
    // item 1: sound waves (squared rate); item 2: fluid motion; item 3:
    // artificial viscosity on compressed directions
    double r1s = cw2 * iL2;
    double ux = fmax(fabs(vxc - vb), fabs(vxp - vb));
    double uy = fmax(fabs(vyc), fabs(vyp));
    double r2 = fmax(ux * iLx, uy * iLy);
    double dvx = vxp - vxc, dvy = vyp - vyc;
    double r3 = 0.0;
    if (dvx < 0.0) r3 = fmax(r3, k3 * fabs(dvx) * iLx);
    if (dvy < 0.0) r3 = fmax(r3, k3 * fabs(dvy) * iLy);
    if (m.d3) {
      double vzc = (double)fz0[mm], vzp = (double)fz1[mm];
      bad |= !isfinite(vzc);
      double uz = fmax(fabs(vzc), fabs(vzp));
      r2 = fmax(r2, uz * iLz);
      double dvz = vzp - vzc;
      if (dvz < 0.0) r3 = fmax(r3, k3 * fabs(dvz) * iLz);
    }
    double rate2 = r1s + r2 * r2 + r3 * r3;
    if (m.visc) {
      // item 4: viscosity, 4 nu / Delta^2
      double r4 = 4.0 * (double)fn[mm] * iL2;
      rate2 += r4 * r4;
    }
    if (!(rate2 >= 0.0)) bad = 1;
    else rmax = rate2 > rmax ? rate2 : rmax;
    if (shear_on) {
      double sh = fabs(vxc / Lx - ((double)fs[mm] + vbg_p) / dXp);
      if (sh > smax) smax = sh;
    }
  }
  block_reduce2(rmax, Max(), 0.0, smax, Max(), 0.0, red);
  int anybad = __syncthreads_or(bad);
  if (tid == 0) {
    ringrate[r] = rmax; // the ring's largest squared rate
    ringshear[r] = smax;
    if (anybad) atomicOr(err, 1);
  }
}

// One workgroup: dt from the ring slots (or the imposed value), then the split
// of every ring.  A non-positive or non-finite dt is flagged and replaced by 0,
// which leaves the state unchanged.
__global__ __launch_bounds__(1024) void k_dt_final(Mesh m, DevWords w, const double *__restrict__ ringrate,
                                                   const double *__restrict__ ringshear) {
#pragma clang fp contract(off)
  __shared__ double red[2 * MAXW];
  constexpr int U = 8; // loads in flight per thread
  double rmax = 0.0, smax = 0.0;
  for (int r0 = threadIdx.x; r0 < m.nring; r0 += U * blockDim.x) {
    double a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int r = r0 + u * (int)blockDim.x;
      a[u] = r < m.nring ? ringrate[r] : 0.0;
      b[u] = r < m.nring ? ringshear[r] : 0.0;
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

} // namespace fargo
