// Stand-alone circular shift of rings (Eq. 32) and conserved sums (mass,
// momenta of Tab. "momenta" with the zone momentum of Eq. 19, internal
// energy) with double-double accumulation in a fixed order.  Both take the
// field type F (double, or float for the FP32-bulk state); the sums are always
// formed in FP64 from the stored values.
#include <mutex>
#include <type_traits>

#include "fargo_internal.h"

namespace fargo {

namespace {

// Eq. 32 in place: one workgroup per active ring, the ring staged in LDS.
template <typename F>
__global__ __launch_bounds__(256) void k_shift(Mesh m, F *__restrict__ f, const int32_t *__restrict__ N) {
  extern __shared__ __align__(16) unsigned char ring_raw[];
  F *ring = reinterpret_cast<F *>(ring_raw);
  int r = blockIdx.x;
  int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  F *row = f + m.idx(0, j, k);
  int n = m.nx;
  for (int i = threadIdx.x; i < n; i += blockDim.x) ring[i] = row[i];
  __syncthreads();
  int s = N[r] % n;
  if (s < 0) s += n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int src = i - s;
    if (src < 0) src += n;
    row[i] = ring[src];
  }
}

// Rings longer than the LDS holds: Eq. 32 out of place into a scratch field
// (one row of blocks per ring), then the active rings copied back.
template <typename F>
__global__ __launch_bounds__(256) void k_shift_out(Mesh m, const F *__restrict__ f, F *__restrict__ t,
                                                   const int32_t *__restrict__ N, int nib) {
  const int r = blockIdx.x / nib, ib = blockIdx.x % nib;
  const int i = ib * 256 + (int)threadIdx.x;
  if (i >= m.nx) return;
  const int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny, n = m.nx;
  int s = N[r] % n;
  if (s < 0) s += n;
  int src = i - s;
  if (src < 0) src += n;
  const size_t row = m.idx(0, j, k);
  t[row + i] = f[row + src];
}
template <typename F>
__global__ __launch_bounds__(256) void k_shift_back(Mesh m, F *__restrict__ f, const F *__restrict__ t, int nib) {
  const int r = blockIdx.x / nib, ib = blockIdx.x % nib;
  const int i = ib * 256 + (int)threadIdx.x;
  if (i >= m.nx) return;
  const size_t o = m.idx(i, m.j0 + r % m.ny, m.k0 + r / m.ny);
  f[o] = t[o];
}

// double-double accumulation (error-free two-sum), contraction off
struct DD {
  double hi, lo;
};
__device__ inline DD dd_add(DD a, double b) {
#pragma clang fp contract(off)
  double s = a.hi + b;
  double bp = s - a.hi;
  double err = (a.hi - (s - bp)) + (b - bp);
  return DD{s, a.lo + err};
}
__device__ inline DD dd_add(DD a, DD b) {
#pragma clang fp contract(off)
  DD s = dd_add(a, b.hi);
  s.lo += b.lo;
  double hi = s.hi + s.lo;
  double lo = s.lo - (hi - s.hi);
  return DD{hi, lo};
}
__device__ inline DD shfl_dd(DD v, int o) { return DD{__shfl_xor(v.hi, o, 64), __shfl_xor(v.lo, o, 64)}; }

__device__ inline DD block_sum(DD v, DD *lds) {
  for (int o = 32; o > 0; o >>= 1) v = dd_add(v, shfl_dd(v, o));
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  DD out{0.0, 0.0};
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) out = dd_add(out, lds[w]);
  __syncthreads();
  return out;
}

// One workgroup per active ring: partial[r*10 + 2q + {0,1}] = (hi, lo) of sum q.
template <typename F>
__global__ __launch_bounds__(256) void k_sums(Mesh m, StateT<F> s, double *__restrict__ partial) {
#pragma clang fp contract(off)
  __shared__ DD lds[4];
  int r = blockIdx.x;
  int j = m.j0 + r % m.ny, k = m.k0 + r / m.ny;
  int jp = m.jabove(j), kp = m.d3 ? m.kabove(k) : k;
  double V = m.Vol(j, k);
  double vbg = 0.0; // an FP32 v_x is a deviation from the ring's FP64 background
  if constexpr (sizeof(F) == 4) vbg = m.bg(BG_V, j, k);
  DD acc[5];
  for (int q = 0; q < 5; q++) acc[q] = DD{0.0, 0.0};
  for (int i = threadIdx.x; i < m.nx; i += blockDim.x) {
    int ip = i + 1 == m.nx ? 0 : i + 1;
    size_t c = m.idx(i, j, k);
    double rho = (double)s.rho[c];
    double t0 = rho * V;
    double t1 = rho * 0.5 * (m.mx(j, k, (double)s.vx[c] + vbg) + m.mx(j, k, (double)s.vx[m.idx(ip, j, k)] + vbg)) * V;
    double t2 = rho * 0.5 * ((double)s.vy[c] + (double)s.vy[m.idx(i, jp, k)]) * V;
    double t3 = m.d3 ? rho * 0.5 * (m.mz(j, (double)s.vz[c]) + m.mz(j, (double)s.vz[m.idx(i, j, kp)])) * V : 0.0;
    double t4 = s.e ? (double)s.e[c] * V : 0.0;
    acc[0] = dd_add(acc[0], t0);
    acc[1] = dd_add(acc[1], t1);
    acc[2] = dd_add(acc[2], t2);
    acc[3] = dd_add(acc[3], t3);
    acc[4] = dd_add(acc[4], t4);
  }
  for (int q = 0; q < 5; q++) {
    DD v = block_sum(acc[q], lds);
    if (threadIdx.x == 0) {
      partial[(size_t)r * 10 + 2 * q] = v.hi;
      partial[(size_t)r * 10 + 2 * q + 1] = v.lo;
    }
  }
}

__global__ __launch_bounds__(256) void k_sums_final(int nring, const double *__restrict__ partial,
                                                    double *__restrict__ out) {
  __shared__ DD lds[4];
  for (int q = 0; q < 5; q++) {
    DD acc{0.0, 0.0};
    for (int r = threadIdx.x; r < nring; r += blockDim.x)
      acc = dd_add(acc, DD{partial[(size_t)r * 10 + 2 * q], partial[(size_t)r * 10 + 2 * q + 1]});
    DD v = block_sum(acc, lds);
    if (threadIdx.x == 0) out[q] = v.hi + v.lo;
  }
}

// Streaming copy for the bandwidth probe: each thread moves U 16-byte
// vectors per round, every load of a round issued before its stores, rounds
// strided over the whole grid.
template <int U>
__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x * U;
  for (size_t b = (size_t)blockIdx.x * blockDim.x * U + threadIdx.x; b < n; b += stride) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const size_t i = b + (size_t)u * blockDim.x;
      if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const size_t i = b + (size_t)u * blockDim.x;
      if (i < n) dst[i] = v[u];
    }
  }
}

// Bandwidth probe of a column sweep's access pattern: NI FP64 fields read,
// the first nout written (out[q] = in[q] + in[NI - 1]), either one element
// per thread (flat) or one (x, y) column per thread walking its nz planes
// (march), the loads of plane k + 1 issued before the stores of plane k.
template <int NI>
__global__ __launch_bounds__(256) void k_streams_flat(StreamPtrs p, int nout, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double v[NI];
#pragma unroll
  for (int q = 0; q < NI; q++) v[q] = p.in[q][i];
#pragma unroll
  for (int q = 0; q < NI; q++)
    if (q < nout) p.out[q][i] = v[q] + v[NI - 1];
}
template <int NI>
__global__ __launch_bounds__(256) void k_streams_march(StreamPtrs p, int nout, size_t ncol, int nz) {
  const size_t col = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= ncol) return;
  double v[NI], w[NI] = {};
  size_t c = col;
#pragma unroll
  for (int q = 0; q < NI; q++) v[q] = p.in[q][c];
#pragma unroll 1
  for (int k = 0; k < nz; k++) {
    const size_t cn = c + ncol;
    if (k + 1 < nz) {
#pragma unroll
      for (int q = 0; q < NI; q++) w[q] = p.in[q][cn];
    }
#pragma unroll
    for (int q = 0; q < NI; q++)
      if (q < nout) p.out[q][c] = v[q] + v[NI - 1];
#pragma unroll
    for (int q = 0; q < NI; q++) v[q] = w[q];
    c = cn;
  }
}

} // namespace

void launch_streams(hipStream_t s, const StreamPtrs &p, int nin, int nout, size_t ncol, int nz, int march) {
  const size_t n = march ? ncol : ncol * (size_t)nz;
  const unsigned nb = (unsigned)((n + 255) / 256);
  auto go = [&](auto ni) {
    constexpr int NI = decltype(ni)::value;
    if (march) k_streams_march<NI><<<nb, 256, 0, s>>>(p, nout, ncol, nz);
    else k_streams_flat<NI><<<nb, 256, 0, s>>>(p, nout, n);
  };
  switch (nin) {
  case 1: go(std::integral_constant<int, 1>{}); break;
  case 2: go(std::integral_constant<int, 2>{}); break;
  case 3: go(std::integral_constant<int, 3>{}); break;
  case 4: go(std::integral_constant<int, 4>{}); break;
  case 5: go(std::integral_constant<int, 5>{}); break;
  case 6: go(std::integral_constant<int, 6>{}); break;
  case 7: go(std::integral_constant<int, 7>{}); break;
  case 8: go(std::integral_constant<int, 8>{}); break;
  default: go(std::integral_constant<int, STREAMS_MAX>{}); break;
  }
}

void launch_stream_copy(hipStream_t s, const void *src, void *dst, size_t bytes, int blocks) {
  const size_t n = bytes / 16;
  if (blocks > 0) k_stream_copy<4><<<(unsigned)blocks, 256, 0, s>>>((const uint4 *)src, (uint4 *)dst, n);
  else k_stream_copy<1><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const uint4 *)src, (uint4 *)dst, n);
}

template <typename F>
void launch_shift(Launch &L, const Mesh &m, F *field, const int32_t *N, F *scratch) {
  prof_begin(L, K_SHIFT);
  if ((size_t)m.nx * sizeof(F) <= 65536) {
    k_shift<F><<<m.nring, 256, (size_t)m.nx * sizeof(F), L.s>>>(m, field, N);
  } else {
    const int nib = (m.nx + 255) / 256;
    const unsigned nb = (unsigned)m.nring * (unsigned)nib;
    k_shift_out<F><<<nb, 256, 0, L.s>>>(m, field, scratch, N, nib);
    k_shift_back<F><<<nb, 256, 0, L.s>>>(m, field, scratch, nib);
  }
  prof_end(L, K_SHIFT);
}

template <typename F>
void launch_sums(Launch &L, const Mesh &m, const StateT<F> &s, double *partial, double *out) {
  prof_begin(L, K_SUMS);
  k_sums<F><<<m.nring, 256, 0, L.s>>>(m, s, partial);
  prof_end(L, K_SUMS);
  prof_begin(L, K_SUMS_FINAL);
  k_sums_final<<<1, 256, 0, L.s>>>(m.nring, partial, out);
  prof_end(L, K_SUMS_FINAL);
}

// Scratch of fargo_conserved_sums_noalloc: the per-ring double-double
// partials (10 doubles a ring) of at most SUMS_STATIC_RINGS rings, then the
// five results.  One copy per device, held until the process ends.  Host code
// must not pass `scratch` itself to a kernel (in host code the name stands for
// a host-side shadow, not the device copy): it uses the device address that
// hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) double scratch[(size_t)SUMS_STATIC_RINGS * 10 + 8];

namespace {
std::mutex scratch_mu;
double *scratch_dev[SCRATCH_MAX_DEVICES] = {};
} // namespace

int static_scratch_setup(int dev) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return FARGO_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_dev[dev]) return FARGO_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != dev) return FARGO_EHIP;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FARGO_EHIP;
  scratch_dev[dev] = (double *)p;
  return FARGO_OK;
}

double *static_scratch(int dev) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  return scratch_dev[dev];
}

template void launch_shift<double>(Launch &, const Mesh &, double *, const int32_t *, double *);
template void launch_shift<float>(Launch &, const Mesh &, float *, const int32_t *, float *);
template void launch_sums<double>(Launch &, const Mesh &, const StateT<double> &, double *, double *);
template void launch_sums<float>(Launch &, const Mesh &, const StateT<float> &, double *, double *);

} // namespace fargo
