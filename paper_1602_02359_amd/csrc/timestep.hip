// Box 3 (bulk azimuthal velocity per ring, Eq. 37), box 6 (time step,
// Eq. cfl2 items 1-3, Eq. 38) and the orbital-advection split of Eq. 29.
//
// The time step and the split (D, N, xi) are computed with floating-point
// contraction off and in the same operation order as the written definition,
// so that the integer shift N is reproducible bit for bit; the global minimum
// is exact and order independent (atomic min on the bit pattern of positive
// doubles, which orders like the values).
#include "fargo_internal.h"

namespace fargo {

namespace {

constexpr unsigned long long INF_BITS = 0x7FF0000000000000ull;

__global__ void k_reset(DevWords w) {
  *w.min_cell = INF_BITS;
  *w.max_shear = 0ull;
}

__global__ void k_set_dt(DevWords w, double dt) { *w.dt = dt; }

// `id` is the identity of `op` (pads the lanes past the number of waves).
template <typename T, typename Op>
__device__ inline T block_reduce(T v, Op op, T id, T *lds) {
  // 64-lane wave reduction then across the (at most 16) waves of the block
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  int nw = (blockDim.x + 63) >> 6;
  if (wid == 0) {
    v = lane < nw ? lds[lane] : id;
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  }
  return v; // valid in thread 0
}

struct Max { __device__ double operator()(double a, double b) const { return a > b ? a : b; } };
struct Min { __device__ double operator()(double a, double b) const { return a < b ? a : b; } };
struct Add { __device__ double operator()(double a, double b) const { return a + b; } };

// One workgroup per active ring: max, min (exact) or the mean of v_x.
__global__ __launch_bounds__(256) void k_ring_v0(Mesh m, const double *__restrict__ vx, double *__restrict__ v0) {
  __shared__ double lds[16];
  int r = blockIdx.x;
  int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  const double *row = vx + m.idx(0, j, k);
  double vmax = row[0], vmin = row[0], sum = 0.0;
  for (int i = threadIdx.x; i < m.nx; i += blockDim.x) {
    double v = row[i];
    vmax = v > vmax ? v : vmax;
    vmin = v < vmin ? v : vmin;
    sum += v;
  }
  if (m.v0_mean) {
    sum = block_reduce(sum, Add(), 0.0, lds);
    if (threadIdx.x == 0) v0[r] = sum / m.nx;
    return;
  }
  vmax = block_reduce(vmax, Max(), -HUGE_VAL, lds);
  __syncthreads();
  vmin = block_reduce(vmin, Min(), HUGE_VAL, lds);
  if (threadIdx.x == 0) v0[r] = 0.5 * (vmax + vmin);
}

// Per active zone: cell time step (Eq. cfl2, items 1-3), shear rate (Eq. 38)
// and validity; block min/max, then one atomic per block.
__global__ __launch_bounds__(256) void k_cfl(Mesh m, StateP s, const double *__restrict__ v0, DevWords w) {
#pragma clang fp contract(off)
  __shared__ double lds[16];
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)m.nx * m.ny * m.nz;
  double cell = __longlong_as_double((long long)INF_BITS);
  double shear = 0.0;
  int bad = 0;
  if (t < total) {
    int i = (int)(t % m.nx);
    long rr = t / m.nx;
    int j = m.j0 + (int)(rr % m.ny), k = m.k0 + (int)(rr / m.ny);
    int ip = i + 1 == m.nx ? 0 : i + 1;
    size_t c = m.idx(i, j, k);
    double vb = m.fargo ? v0[rr] : 0.0;
    double Lx = m.DX(j, k), Lyy = m.g.Ly[j];
    double rho = s.rho[c];
    double cw;
    if (m.eos == FARGO_ISOTHERMAL) cw = s.cs[c];
    else {
      double P = (m.gamma - 1.0) * s.e[c];
      cw = sqrt(m.gamma * P / rho);
    }
    double vxc = s.vx[c], vxp = s.vx[m.idx(ip, j, k)];
    double vyc = s.vy[c], vyp = s.vy[m.idx(i, j + 1, k)];
    bad = !(rho > 0.0) || !isfinite(rho) || !isfinite(cw) || !isfinite(vxc) || !isfinite(vyc);
    double dt1 = fmin(Lx / cw, Lyy / cw);
    double ux = fmax(fabs(vxc - vb), fabs(vxp - vb));
    double uy = fmax(fabs(vyc), fabs(vyp));
    double dt2 = fmin(Lx / ux, Lyy / uy);
    double dvx = vxp - vxc, dvy = vyp - vyc;
    double dt3 = __longlong_as_double((long long)INF_BITS);
    if (dvx < 0.0) dt3 = fmin(dt3, Lx / (4.0 * m.cvnr * m.cvnr * fabs(dvx)));
    if (dvy < 0.0) dt3 = fmin(dt3, Lyy / (4.0 * m.cvnr * m.cvnr * fabs(dvy)));
    if (m.d3) {
      double Lzz = m.Lz(j, k);
      double vzc = s.vz[c], vzp = s.vz[m.idx(i, j, k + 1)];
      bad |= !isfinite(vzc);
      dt1 = fmin(dt1, Lzz / cw);
      double uz = fmax(fabs(vzc), fabs(vzp));
      dt2 = fmin(dt2, Lzz / uz);
      double dvz = vzp - vzc;
      if (dvz < 0.0) dt3 = fmin(dt3, Lzz / (4.0 * m.cvnr * m.cvnr * fabs(dvz)));
    }
    cell = 1.0 / sqrt(1.0 / (dt1 * dt1) + 1.0 / (dt2 * dt2) + 1.0 / (dt3 * dt3));
    if (!(cell >= 0.0)) { bad = 1; cell = __longlong_as_double((long long)INF_BITS); }
    if (m.fargo && m.shear_c0 > 0.0 && j + 1 < m.jn) {
      double sh = fabs(vxc / Lx - s.vx[m.idx(i, j + 1, k)] / m.DX(j + 1, k));
      shear = sh == sh ? sh : 0.0;
    }
  }
  cell = block_reduce(cell, Min(), (double)HUGE_VAL, lds);
  __syncthreads();
  shear = block_reduce(shear, Max(), 0.0, lds);
  int anybad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    atomicMin(w.min_cell, dbits(cell));
    if (shear > 0.0) atomicMax(w.max_shear, dbits(shear));
    if (anybad) atomicOr(w.err, 1);
  }
}

__global__ void k_dt_final(Mesh m, DevWords w, int use_given) {
#pragma clang fp contract(off)
  double mincell = __longlong_as_double((long long)*w.min_cell);
  double maxshear = __longlong_as_double((long long)*w.max_shear);
  double dt = m.courant * mincell;
  if (m.fargo && m.shear_c0 > 0.0 && maxshear > 0.0) dt = fmin(dt, m.shear_c0 / maxshear);
  if (use_given) return;
  if (!(dt > 0.0) || !isfinite(dt)) {
    atomicOr(w.err, 2);
    dt = 0.0; // a zero step leaves the state unchanged
  }
  *w.dt = dt;
}

// Eq. 29: D = (v0 dt)/dX, N = nearest integer (ties away from zero), xi = D - N.
__global__ __launch_bounds__(256) void k_split(Mesh m, const double *__restrict__ v0, const double *__restrict__ dtp,
                                               double dt_val, int32_t *__restrict__ N, double *__restrict__ xi) {
#pragma clang fp contract(off)
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m.nring) return;
  int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  double dt = dtp ? *dtp : dt_val;
  double D = (v0[r] * dt) / m.DX(j, k);
  double n = round(D);
  N[r] = (int32_t)n;
  xi[r] = D - n;
}

} // namespace

void launch_reset(Launch &L, const DevWords &w) {
  prof_begin(L, K_RESET);
  k_reset<<<1, 1, 0, L.s>>>(w);
  prof_end(L, K_RESET);
}

void launch_set_dt(Launch &L, const DevWords &w, double dt) {
  prof_begin(L, K_SET_DT);
  k_set_dt<<<1, 1, 0, L.s>>>(w, dt);
  prof_end(L, K_SET_DT);
}

void launch_ring_v0(Launch &L, const Mesh &m, const double *vx, double *v0) {
  prof_begin(L, K_RING_V0);
  k_ring_v0<<<m.nring, 256, 0, L.s>>>(m, vx, v0);
  prof_end(L, K_RING_V0);
}

void launch_cfl(Launch &L, const Mesh &m, const StateP &s, const double *v0, const DevWords &w) {
  long total = (long)m.nx * m.ny * m.nz;
  prof_begin(L, K_CFL);
  k_cfl<<<(unsigned)((total + 255) / 256), 256, 0, L.s>>>(m, s, v0, w);
  prof_end(L, K_CFL);
}

void launch_dt_final(Launch &L, const Mesh &m, const DevWords &w, int use_given) {
  prof_begin(L, K_DT_FINAL);
  k_dt_final<<<1, 1, 0, L.s>>>(m, w, use_given);
  prof_end(L, K_DT_FINAL);
}

void launch_split(Launch &L, const Mesh &m, const double *v0, const double *dt, double dt_val, int32_t *N,
                  double *xi) {
  prof_begin(L, K_SPLIT);
  k_split<<<(m.nring + 255) / 256, 256, 0, L.s>>>(m, v0, dt, dt_val, N, xi);
  prof_end(L, K_SPLIT);
}

} // namespace fargo
