// Learned flux correction (not in the paper).  A three-layer 3 x 3
// convolutional net on the coarse 2D (phi, r) state predicts corrections to
// the mass fluxes through each zone's lower X and lower Y face; they enter as
// a conservative flux-divergence update of the density, so the mass change
// telescopes to zero over the mesh (the conservation argument of Sect. 3.4
// applied to the added fluxes).  The net is trained on device: forward pass,
// loss, backward pass and Adam (Kingma & Ba 2015).
//
// The convolutions are implicit GEMMs on the bfloat16 matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation), one 16-row tile per wave:
//   forward     out[p][co] = sum_k A[p][k] W[co][k],  k = tap Cin + ci,
//               A[p][k] = act[p shifted by tap][ci]               (M = pixels)
//   input grad  the adjoint convolution, a forward one with the weights
//               transposed and their taps flipped                  (M = pixels)
//   weight grad dW[co][k] = sum_p g[p][co] A[p][k]                 (M = Cout,
//               reduced over pixel chunks, partial sums per chunk)
// Operand layouts of the 16x16x16 MFMA: lane l holds row (or column) l % 16
// and the four k values 4 (l / 16) .. 4 (l / 16) + 3; the result tile gives
// lane l column l % 16 and rows 4 (l / 16) .. 4 (l / 16) + 3.
//
// Activations are channels-last bfloat16, [pixel][channel] with pixel =
// j nx + i over the active zones (j = 0 the innermost ring), zero beyond the
// radial rows and periodic in i; weights [co][tap][ci], tap = 3 ty + tx.
#include "fargo_internal.h"

namespace fargo {

namespace {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int LB = 256; // threads per block of the elementwise kernels

// FP32 -> bfloat16, round to nearest even (finite values)
__device__ inline unsigned short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// four consecutive bfloat16 (8-byte aligned) as an MFMA operand
__device__ inline bf4 ld4(const unsigned short *p) {
  const uint2 v = *reinterpret_cast<const uint2 *>(p);
  bf4 r;
  r[0] = (short)(v.x & 0xFFFFu);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xFFFFu);
  r[3] = (short)(v.y >> 16);
  return r;
}
__device__ inline bf4 zero4() {
  bf4 r;
  r[0] = r[1] = r[2] = r[3] = 0;
  return r;
}

// ---------------------------------------------------------------------------
// features (FP64 arithmetic, rounded to FP32 then to bfloat16)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LB) void k_features(Mesh m, const double *__restrict__ rho,
                                                 const double *__restrict__ vx, const double *__restrict__ vy,
                                                 LfcScales sc, unsigned short *__restrict__ f) {
#pragma clang fp contract(off)
  const int npix = m.nx * m.ny;
  const int p = blockIdx.x * LB + threadIdx.x;
  if (p >= npix) return;
  const int j = p / m.nx, i = p - j * m.nx;
  const unsigned c = m.o32(i, j + m.j0, 0);
  const double f0 = rho[c] / sc.rho_s - 1.0;
  const double f1 = vy[c] / sc.u_s;
  const double f2 = vx[c] / sc.u_s;
  const double f3 = (m.g.ymed(j + m.j0) - sc.r_mid) / sc.r_span;
  uint2 v;
  v.x = (unsigned)to_bf16((float)f0) | ((unsigned)to_bf16((float)f1) << 16);
  v.y = (unsigned)to_bf16((float)f2) | ((unsigned)to_bf16((float)f3) << 16);
  *reinterpret_cast<uint2 *>(f + (size_t)p * 4) = v;
}

// ---------------------------------------------------------------------------
// 3 x 3 convolution through LDS.  A block takes 64 pixels of one row (a wave
// per 16 of them) and stages the three input rows they read, 66 columns wide
// (periodic in i, zero rows outside the mesh), so that each input value is
// read from memory once per block rather than once per tap; the MFMA A
// operands then come from LDS.  Wb is [16 NT][KP] bfloat16, KP = 9 CIN
// rounded up to 16.  Modes: CV_HID, out = bf16(relu(conv + b)); CV_OUT,
// out = conv + b (FP32); CV_ADJ, the adjoint convolution (weights transposed
// and their taps flipped), out = bf16([h > 0] conv).
// ---------------------------------------------------------------------------
enum { CV_HID = 0, CV_OUT = 1, CV_ADJ = 2 };

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(int nx, int ny, const unsigned short *__restrict__ act,
                                              const unsigned short *__restrict__ Wb,
                                              const float *__restrict__ bias, const unsigned short *__restrict__ h,
                                              unsigned short *__restrict__ hout, float *__restrict__ fout) {
  constexpr int K = 9 * CIN, KP = (K + 15) / 16 * 16, NT = (COUT + 15) / 16;
  constexpr int CP = CIN + 4, TW = 66, CH = CIN / 4; // padded pixel stride; staged columns
  __shared__ __align__(16) unsigned short T[3][TW][CP];
  const int tid = threadIdx.x, lane = tid & 63, m = lane & 15, kq = lane >> 4, wv = tid >> 6;
  const int pb = blockIdx.x * 64; // first pixel of the block: a row segment, since nx % 64 == 0
  const int y = pb / nx, x0 = pb - y * nx;
  for (int e = tid; e < 3 * TW * CH; e += 256) {
    const int c4 = e % CH, col = (e / CH) % TW, ry = e / (CH * TW);
    const int yy = y + ry - 1;
    int xx = x0 + col - 1;
    xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
    uint2 v = make_uint2(0u, 0u);
    if (yy >= 0 && yy < ny) v = *reinterpret_cast<const uint2 *>(act + ((size_t)yy * nx + xx) * CIN + 4 * c4);
    *reinterpret_cast<uint2 *>(&T[ry][col][4 * c4]) = v;
  }
  __syncthreads();
  const int xl = wv * 16 + m; // the lane's A row, as a staged column offset
  f4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int s = 0; s < KP / 16; s++) {
    const int k0 = 16 * s + 4 * kq;
    bf4 a = zero4();
    if (k0 < K) {
      const int tap = k0 / CIN, ci = k0 - tap * CIN;
      a = ld4(&T[tap / 3][xl + tap % 3][ci]);
    }
#pragma unroll
    for (int t = 0; t < NT; t++) {
      const bf4 b = ld4(Wb + (size_t)(16 * t + m) * KP + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; t++) {
    const int co = 16 * t + m;
    if (co >= COUT) continue;
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const size_t idx = (size_t)(pb + wv * 16 + 4 * kq + v) * COUT + co;
      if (MODE == CV_HID) {
        const float val = acc[t][v] + bias[co];
        hout[idx] = to_bf16(val > 0.f ? val : 0.f);
      } else if (MODE == CV_OUT) {
        fout[idx] = acc[t][v] + bias[co];
      } else {
        hout[idx] = to_bf16(from_bf16(h[idx]) > 0.f ? acc[t][v] : 0.f);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// density change from the net output, loss partial sums and dL/d(divergence)
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double *lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) s += lds[q];
  return s; // in thread 0
}

__global__ __launch_bounds__(LB) void k_drho(Mesh m, const float *__restrict__ o, double sF,
                                             const double *__restrict__ target, double sigma,
                                             double *__restrict__ drho, double *__restrict__ gD,
                                             double *__restrict__ lpart) {
#pragma clang fp contract(off)
  __shared__ double red[LB / 64];
  const int nx = m.nx, ny = m.ny, npix = nx * ny;
  const int p = blockIdx.x * LB + threadIdx.x;
  double e2 = 0.0;
  if (p < npix) {
    const int j = p / nx, i = p - j * nx;
    const int pr = j * nx + (i + 1 == nx ? 0 : i + 1), pu = p + nx;
    const double fx0 = sF * (double)o[2 * p], fx1 = sF * (double)o[2 * pr];
    const double fy0 = j == 0 ? 0.0 : sF * (double)o[2 * p + 1];
    const double fy1 = j + 1 == ny ? 0.0 : sF * (double)o[2 * pu + 1];
    const double div = (fx1 - fx0) + (fy1 - fy0);
    const double iv = m.g.invVj(j + m.j0);
    const double d = (-iv) * div;
    drho[p] = d;
    if (target) {
      const double t = target[p];
      const double e = (d - t) / sigma;
      e2 = e * e;
      const double g = 2.0 * (d - t) / ((double)npix * sigma * sigma);
      gD[p] = (-iv) * g;
    }
  }
  if (!target) return;
  const double s = block_sum(e2, red);
  if (threadIdx.x == 0) lpart[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_loss_final(const double *__restrict__ lpart, int n, int npix,
                                                    double *__restrict__ loss) {
  __shared__ double red[4];
  double s = 0.0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) s += lpart[q];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *loss = s / (double)npix;
}

// dL/d(net output) through the adjoint of the divergence; 4 channels (the
// last two zero) so that the input-gradient GEMM takes them in groups of 4
__global__ __launch_bounds__(LB) void k_flux_grad(int nx, int ny, const double *__restrict__ gD, double sF,
                                                  unsigned short *__restrict__ g3) {
#pragma clang fp contract(off)
  const int p = blockIdx.x * LB + threadIdx.x;
  if (p >= nx * ny) return;
  const int j = p / nx, i = p - j * nx;
  const double gx = gD[j * nx + (i == 0 ? nx - 1 : i - 1)] - gD[p];
  const double gy = j == 0 ? 0.0 : gD[p - nx] - gD[p];
  uint2 v;
  v.x = (unsigned)to_bf16((float)(sF * gx)) | ((unsigned)to_bf16((float)(sF * gy)) << 16);
  v.y = 0u;
  *reinterpret_cast<uint2 *>(g3 + (size_t)p * 4) = v;
}

// ---------------------------------------------------------------------------
// weight gradient through LDS: dW[co][tap CIN + ci] = sum_p g[p][co]
// act[p shifted by tap][ci] over a chunk of PC pixels (whole 64-pixel row
// segments).  Per segment the block stages the three activation rows (as
// the convolution does) and the layer gradient transposed to [co][pixel];
// each wave then owns a share of the (co tile, k tile) pairs and accumulates
// them over the chunk.  One partial sum per chunk, for the reduction below;
// the bias gradient (the sum of g) alongside.
// ---------------------------------------------------------------------------
constexpr int PC = LFC_CHUNK;

template <int CIN, int COUT, int GC>
__global__ __launch_bounds__(256) void k_conv_w(int nx, int ny, const unsigned short *__restrict__ g,
                                                const unsigned short *__restrict__ act, float *__restrict__ part,
                                                float *__restrict__ dbpart) {
  constexpr int K = 9 * CIN, KP = (K + 15) / 16 * 16, NTW = KP / 16, MT = (COUT + 15) / 16;
  constexpr int NTILE = MT * NTW, TPW = (NTILE + 3) / 4; // tiles, and tiles per wave
  constexpr int CP = CIN + 4, TW = 66, CH = CIN / 4, GP = 64 + 4;
  constexpr int DBC = 32, DBS = 256 / DBC; // bias sums: channel tid % DBC, pixel subset tid / DBC
  __shared__ __align__(16) unsigned short T[3][TW][CP];
  __shared__ __align__(16) unsigned short Gt[MT * 16][GP];
  __shared__ float dbr[DBS][DBC];
  const int tid = threadIdx.x, lane = tid & 63, m = lane & 15, kq = lane >> 4, wv = tid >> 6;
  const int chunk = blockIdx.x;
  f4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; t++) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  // the wave's tiles: the weight column of the lane in each
  int tmt[TPW], tty[TPW], ttx[TPW], tci[TPW];
  bool tok[TPW];
#pragma unroll
  for (int t = 0; t < TPW; t++) {
    const int tile = t * 4 + wv, mt = tile / NTW, nt = tile - mt * NTW, kk = 16 * nt + m;
    tok[t] = tile < NTILE && kk < K;
    tmt[t] = tile < NTILE ? mt : 0;
    const int tap = tok[t] ? kk / CIN : 0;
    tci[t] = tok[t] ? kk - tap * CIN : 0;
    tty[t] = tap / 3;
    ttx[t] = tap % 3;
  }
  float db = 0.f;
  for (int seg = 0; seg < PC / 64; seg++) {
    const int pb = chunk * PC + seg * 64;
    const int y = pb / nx, x0 = pb - y * nx;
    __syncthreads(); // the previous segment's reads are done
    for (int e = tid; e < 3 * TW * CH; e += 256) {
      const int c4 = e % CH, col = (e / CH) % TW, ry = e / (CH * TW);
      const int yy = y + ry - 1;
      int xx = x0 + col - 1;
      xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
      uint2 v = make_uint2(0u, 0u);
      if (yy >= 0 && yy < ny) v = *reinterpret_cast<const uint2 *>(act + ((size_t)yy * nx + xx) * CIN + 4 * c4);
      *reinterpret_cast<uint2 *>(&T[ry][col][4 * c4]) = v;
    }
    for (int e = tid; e < MT * 16 * 64; e += 256) {
      const int px = e & 63, co = e >> 6;
      Gt[co][px] = co < COUT ? g[(size_t)(pb + px) * GC + co] : (unsigned short)0;
    }
    __syncthreads();
    {
      const int co = tid % DBC, sub = tid / DBC;
      if (co < COUT)
        for (int px = sub; px < 64; px += DBS) db += from_bf16(Gt[co][px]);
    }
#pragma unroll
    for (int t = 0; t < TPW; t++) {
      if (!tok[t] && (t * 4 + wv) >= NTILE) continue;
#pragma unroll
      for (int ks = 0; ks < 4; ks++) {
        const int p4 = 16 * ks + 4 * kq; // the lane's four pixels of the segment
        const bf4 a = ld4(&Gt[16 * tmt[t] + m][p4]);
        bf4 b = zero4();
        if (tok[t]) {
#pragma unroll
          for (int v = 0; v < 4; v++) b[v] = (short)T[tty[t]][p4 + v + ttx[t]][tci[t]];
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  // result: lane holds column kk = 16 nt + m and rows co = 16 mt + 4 kq + v
#pragma unroll
  for (int t = 0; t < TPW; t++) {
    if (!tok[t]) continue;
    const int tile = t * 4 + wv, nt = tile - tmt[t] * NTW, kk = 16 * nt + m;
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int co = 16 * tmt[t] + 4 * kq + v;
      if (co < COUT) part[((size_t)chunk * COUT + co) * K + kk] = acc[t][v];
    }
  }
  dbr[tid / DBC][tid % DBC] = db;
  __syncthreads();
  if (tid < COUT) {
    float d = 0.f;
    for (int q = 0; q < DBS; q++) d += dbr[q][tid];
    dbpart[(size_t)chunk * COUT + tid] = d;
  }
}

// grad[W] = sum over chunks of the partials, grad[b] likewise.  A block takes
// RE consecutive entries; its RG thread groups sum interleaved subsets of the
// chunks, and the group sums are added in a fixed order (deterministic).
constexpr int RE = 64, RG = 16;
__global__ __launch_bounds__(RE * RG) void k_reduce_w(int nchunk, int cout, int K, const float *__restrict__ part,
                                                      const float *__restrict__ dbpart, float *__restrict__ gW,
                                                      float *__restrict__ gb) {
  __shared__ float red[RG][RE];
  const int el = threadIdx.x % RE, g = threadIdx.x / RE;
  const int e = blockIdx.x * RE + el;
  const int nw = cout * K;
  float s = 0.f;
  if (e < nw) {
#pragma unroll 8
    for (int c = g; c < nchunk; c += RG) s += part[(size_t)c * nw + e];
  } else if (e < nw + cout) {
    for (int c = g; c < nchunk; c += RG) s += dbpart[(size_t)c * cout + (e - nw)];
  }
  red[g][el] = s;
  __syncthreads();
  if (g == 0 && e < nw + cout) {
    float t = 0.f;
    for (int q = 0; q < RG; q++) t += red[q][el];
    if (e < nw) gW[e] = t;
    else gb[e - nw] = t;
  }
}

// ---------------------------------------------------------------------------
// Adam on the FP32 master parameters, and the bfloat16 copies of the weights
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LB) void k_adam(int n, float *__restrict__ w, float *__restrict__ mo,
                                             float *__restrict__ ve, const float *__restrict__ g, float lr,
                                             float b1, float b2, float c1, float c2, float eps) {
  const int e = blockIdx.x * LB + threadIdx.x;
  if (e >= n) return;
  const float ge = g[e];
  const float mn = b1 * mo[e] + (1.f - b1) * ge;
  const float vn = b2 * ve[e] + (1.f - b2) * ge * ge;
  mo[e] = mn;
  ve[e] = vn;
  w[e] = w[e] - lr * (mn / c1) / (sqrtf(vn / c2) + eps);
}

// Wb_l [16 NT][KP] for the forward GEMMs; Wt2 [32][288] and Wt3 [32][48]
// (tap-major over the 4-padded output channels) for the input gradients
__global__ __launch_bounds__(LB) void k_pack(const float *__restrict__ w, LfcWeights b) {
  const int e = blockIdx.x * LB + threadIdx.x;
  const float *W1 = w + LFC_OFF_W1, *W2 = w + LFC_OFF_W2, *W3 = w + LFC_OFF_W3;
  // forward copies
  if (e < 32 * 48) {
    const int co = e / 48, k = e - co * 48;
    b.wb1[e] = k < 36 ? to_bf16(W1[co * 36 + k]) : (unsigned short)0;
  }
  if (e < 32 * 288) {
    b.wb2[e] = to_bf16(W2[e]);
    const int ci = e / 288, k = e - ci * 288, tap = k / 32, co = k - tap * 32;
    b.wt2[e] = to_bf16(W2[co * 288 + (8 - tap) * 32 + ci]); // taps flipped: the adjoint as a convolution
  }
  if (e < 16 * 288) {
    const int co = e / 288, k = e - co * 288;
    b.wb3[e] = co < 2 ? to_bf16(W3[co * 288 + k]) : (unsigned short)0;
  }
  if (e < 32 * 48) {
    const int ci = e / 48, k = e - ci * 48, tap = k / 4, co = k - tap * 4;
    b.wt3[e] = (k < 36 && co < 2) ? to_bf16(W3[co * 288 + (8 - tap) * 32 + ci]) : (unsigned short)0;
  }
}

// ---------------------------------------------------------------------------
// guard and conservative update; restriction
// ---------------------------------------------------------------------------
__global__ void k_flag_clear(int *flag) { *flag = 0; }

__global__ __launch_bounds__(LB) void k_guard(Mesh m, const double *__restrict__ rho,
                                              const double *__restrict__ d, double guard, int *flag) {
#pragma clang fp contract(off)
  const int p = blockIdx.x * LB + threadIdx.x;
  if (p >= m.nx * m.ny) return;
  const int j = p / m.nx, i = p - j * m.nx;
  const double r = rho[m.o32(i, j + m.j0, 0)], dd = d[p];
  if (!(r + dd > 0.0) || !(fabs(dd) <= guard * r)) atomicOr(flag, 1);
}

__global__ __launch_bounds__(LB) void k_commit(Mesh m, double *__restrict__ rho, const double *__restrict__ d,
                                               const int *__restrict__ flag) {
  const int p = blockIdx.x * LB + threadIdx.x;
  if (p >= m.nx * m.ny || *flag) return;
  const int j = p / m.nx, i = p - j * m.nx;
  const unsigned c = m.o32(i, j + m.j0, 0);
  rho[c] = rho[c] + d[p];
}

__global__ __launch_bounds__(LB) void k_restrict(Mesh mf, Mesh mc, int R, const double *__restrict__ rf,
                                                 const double *__restrict__ vxf, const double *__restrict__ vyf,
                                                 double *__restrict__ rc, double *__restrict__ vxc,
                                                 double *__restrict__ vyc) {
#pragma clang fp contract(off)
  const int p = blockIdx.x * LB + threadIdx.x;
  if (p >= mc.nx * mc.ny) return;
  const int J = p / mc.nx, I = p - J * mc.nx;
  double mass = 0.0, wsum = 0.0, vx = 0.0, drs = 0.0, vy = 0.0;
  for (int b = 0; b < R; b++) {
    const int jf = R * J + b + mf.j0;
    const double ya = mf.g.ymin(jf), yb = mf.g.ymin(jf + 1);
    const double w = 0.5 * (yb * yb - ya * ya), dr = yb - ya;
    double s = 0.0;
    for (int a = 0; a < R; a++) s += rf[mf.o32(R * I + a, jf, 0)] * w;
    mass += s;
    wsum += w;
    vx += vxf[mf.o32(R * I, jf, 0)] * dr;
    drs += dr;
  }
  for (int a = 0; a < R; a++) vy += vyf[mf.o32(R * I + a, R * J + mf.j0, 0)];
  const unsigned c = mc.o32(I, J + mc.j0, 0);
  rc[c] = mass / (wsum * R);
  vxc[c] = vx / drs;
  vyc[c] = vy / R;
}

// training target: the density change that takes the plain coarse step to
// the restricted fine solution, over the active zones
__global__ __launch_bounds__(LB) void k_target(Mesh m, const double *__restrict__ ref,
                                               const double *__restrict__ plain, double *__restrict__ t) {
  const int p = blockIdx.x * LB + threadIdx.x;
  if (p >= m.nx * m.ny) return;
  const int j = p / m.nx, i = p - j * m.nx;
  const unsigned c = m.o32(i, j + m.j0, 0);
  t[p] = ref[c] - plain[c];
}

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

} // namespace

void lfc_forward(Launch &L, const Mesh &m, const double *rho, const double *vx, const double *vy,
                 const LfcScales &sc, const LfcBufs &B) {
  const int npix = m.nx * m.ny;
  prof_begin(L, K_LFC_FEATURES);
  k_features<<<nblk(npix, LB), LB, 0, L.s>>>(m, rho, vx, vy, sc, B.f);
  prof_end(L, K_LFC_FEATURES);
  const unsigned nb = (unsigned)(npix / 64);
  prof_begin(L, K_LFC_CONV_FWD);
  k_conv<4, 32, CV_HID><<<nb, 256, 0, L.s>>>(m.nx, m.ny, B.f, B.wt.wb1, B.w + LFC_OFF_B1, nullptr, B.h1, nullptr);
  prof_end(L, K_LFC_CONV_FWD);
  prof_begin(L, K_LFC_CONV_FWD);
  k_conv<32, 32, CV_HID><<<nb, 256, 0, L.s>>>(m.nx, m.ny, B.h1, B.wt.wb2, B.w + LFC_OFF_B2, nullptr, B.h2, nullptr);
  prof_end(L, K_LFC_CONV_FWD);
  prof_begin(L, K_LFC_CONV_FWD);
  k_conv<32, 2, CV_OUT><<<nb, 256, 0, L.s>>>(m.nx, m.ny, B.h2, B.wt.wb3, B.w + LFC_OFF_B3, nullptr, nullptr, B.o);
  prof_end(L, K_LFC_CONV_FWD);
}

void lfc_drho(Launch &L, const Mesh &m, const LfcBufs &B, double sF, const double *target, double sigma) {
  const int npix = m.nx * m.ny;
  const unsigned nb = nblk(npix, LB);
  prof_begin(L, K_LFC_DRHO);
  k_drho<<<nb, LB, 0, L.s>>>(m, B.o, sF, target, sigma, B.drho, B.gD, B.lpart);
  prof_end(L, K_LFC_DRHO);
  if (target) {
    prof_begin(L, K_LFC_DRHO);
    k_loss_final<<<1, 256, 0, L.s>>>(B.lpart, (int)nb, npix, B.loss);
    prof_end(L, K_LFC_DRHO);
  }
}

void lfc_backward(Launch &L, const Mesh &m, const LfcBufs &B, double sF) {
  const int nx = m.nx, ny = m.ny, npix = nx * ny, nchunk = npix / PC;
  const unsigned nb = (unsigned)(npix / 64);
  prof_begin(L, K_LFC_DRHO);
  k_flux_grad<<<nblk(npix, LB), LB, 0, L.s>>>(nx, ny, B.gD, sF, B.g3);
  prof_end(L, K_LFC_DRHO);
  // layer 3: weights from g3 and h2, then the gradient into h2
  prof_begin(L, K_LFC_BWD_W);
  k_conv_w<32, 2, 4><<<nchunk, 256, 0, L.s>>>(nx, ny, B.g3, B.h2, B.part, B.dbpart);
  prof_end(L, K_LFC_BWD_W);
  prof_begin(L, K_LFC_REDUCE);
  k_reduce_w<<<nblk(2 * 288 + 2, RE), RE * RG, 0, L.s>>>(nchunk, 2, 288, B.part, B.dbpart, B.grad + LFC_OFF_W3,
                                                     B.grad + LFC_OFF_B3);
  prof_end(L, K_LFC_REDUCE);
  prof_begin(L, K_LFC_BWD_DATA);
  k_conv<4, 32, CV_ADJ><<<nb, 256, 0, L.s>>>(nx, ny, B.g3, B.wt.wt3, nullptr, B.h2, B.g2, nullptr);
  prof_end(L, K_LFC_BWD_DATA);
  // layer 2
  prof_begin(L, K_LFC_BWD_W);
  k_conv_w<32, 32, 32><<<nchunk, 256, 0, L.s>>>(nx, ny, B.g2, B.h1, B.part, B.dbpart);
  prof_end(L, K_LFC_BWD_W);
  prof_begin(L, K_LFC_REDUCE);
  k_reduce_w<<<nblk(32 * 288 + 32, RE), RE * RG, 0, L.s>>>(nchunk, 32, 288, B.part, B.dbpart, B.grad + LFC_OFF_W2,
                                                       B.grad + LFC_OFF_B2);
  prof_end(L, K_LFC_REDUCE);
  prof_begin(L, K_LFC_BWD_DATA);
  k_conv<32, 32, CV_ADJ><<<nb, 256, 0, L.s>>>(nx, ny, B.g2, B.wt.wt2, nullptr, B.h1, B.g1, nullptr);
  prof_end(L, K_LFC_BWD_DATA);
  // layer 1 (no gradient into the features)
  prof_begin(L, K_LFC_BWD_W);
  k_conv_w<4, 32, 32><<<nchunk, 256, 0, L.s>>>(nx, ny, B.g1, B.f, B.part, B.dbpart);
  prof_end(L, K_LFC_BWD_W);
  prof_begin(L, K_LFC_REDUCE);
  k_reduce_w<<<nblk(32 * 36 + 32, RE), RE * RG, 0, L.s>>>(nchunk, 32, 36, B.part, B.dbpart, B.grad + LFC_OFF_W1,
                                                      B.grad + LFC_OFF_B1);
  prof_end(L, K_LFC_REDUCE);
}

void lfc_adam(Launch &L, const LfcBufs &B, float lr, float c1, float c2) {
  prof_begin(L, K_LFC_ADAM);
  k_adam<<<nblk(LFC_NPARAM, LB), LB, 0, L.s>>>(LFC_NPARAM, B.w, B.mo, B.ve, B.grad, lr, 0.9f, 0.999f, c1, c2,
                                               1e-8f);
  prof_end(L, K_LFC_ADAM);
}

void lfc_pack(Launch &L, const LfcBufs &B) {
  prof_begin(L, K_LFC_ADAM);
  k_pack<<<nblk(32 * 288, LB), LB, 0, L.s>>>(B.w, B.wt);
  prof_end(L, K_LFC_ADAM);
}

void lfc_apply(Launch &L, const Mesh &m, const LfcBufs &B, double *rho, double guard, int *flag) {
  const int npix = m.nx * m.ny;
  prof_begin(L, K_LFC_APPLY);
  k_flag_clear<<<1, 1, 0, L.s>>>(flag);
  prof_end(L, K_LFC_APPLY);
  prof_begin(L, K_LFC_APPLY);
  k_guard<<<nblk(npix, LB), LB, 0, L.s>>>(m, rho, B.drho, guard, flag);
  prof_end(L, K_LFC_APPLY);
  prof_begin(L, K_LFC_APPLY);
  k_commit<<<nblk(npix, LB), LB, 0, L.s>>>(m, rho, B.drho, flag);
  prof_end(L, K_LFC_APPLY);
}

void lfc_target(Launch &L, const Mesh &m, const double *ref, const double *plain, double *t) {
  k_target<<<nblk((long)m.nx * m.ny, LB), LB, 0, L.s>>>(m, ref, plain, t);
}

void lfc_restrict(Launch &L, const Mesh &mf, const double *rf, const double *vxf, const double *vyf, const Mesh &mc,
                  double *rc, double *vxc, double *vyc) {
  k_restrict<<<nblk((long)mc.nx * mc.ny, LB), LB, 0, L.s>>>(mf, mc, mf.nx / mc.nx, rf, vxf, vyf, rc, vxc, vyc);
}

} // namespace fargo
