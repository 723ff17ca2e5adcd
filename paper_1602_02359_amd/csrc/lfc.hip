// Learned flux correction (not in the paper).  A three-layer 3 x 3
// convolutional net on the coarse 2D (phi, r) state predicts corrections to
// the mass fluxes through each zone's lower X and lower Y face; they enter as
// a conservative flux-divergence update of the density, so the mass change
// telescopes to zero over the mesh (the conservation argument of Sect. 3.4
// applied to the added fluxes).  The net is trained on device: forward pass,
// loss, backward pass and Adam (Kingma & Ba 2015), over a batch of samples
// of one mesh per step.
//
// The convolutions are implicit GEMMs on the bfloat16 matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation):
//   forward     out[p][co] = sum_k W[co][k] A[k][p],  k = tap Cin + ci,
//               A[k][p] = act[p shifted by tap][ci]       (M = Cout, N = pixels)
//   input grad  the adjoint convolution, a forward one with the weights
//               transposed and their taps flipped          (M = Cin, N = pixels)
//   weight grad dW[co][k] = sum_p g[p][co] A[k][p]         (M = Cout, N = k,
//               K = pixels; partial sums per block, reduced in a fixed order)
// Operand layout of the 16 x 16 x 32 MFMA: lane l supplies row (A) or
// column (B) l % 16 with eight k values, lane group l / 16 taking k = 8
// (l / 16) .. 8 (l / 16) + 7 (any assignment of k to the lane groups works,
// as long as A and B agree on it); the result gives lane l column l % 16 and
// rows 4 (l / 16) .. 4 (l / 16) + 3.
//
// Activations are channels-last bfloat16, [sample][pixel][channel] with
// pixel = j nx + i over the active zones (j = 0 the innermost ring), zero
// beyond the radial rows of each sample and periodic in i; weights
// [co][tap][ci], tap = 3 ty + tx.
#include "fargo_internal.h"

namespace fargo {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int LB = 256; // threads per block of the elementwise kernels

// FP32 -> bfloat16, round to nearest even (finite values)
__device__ inline unsigned short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ inline float lo_bf16(unsigned v) { return __uint_as_float(v << 16); }
__device__ inline float hi_bf16(unsigned v) { return __uint_as_float(v & 0xFFFF0000u); }
__device__ inline unsigned pack2(float a, float b) { return (unsigned)to_bf16(a) | ((unsigned)to_bf16(b) << 16); }

__device__ inline f4 mfma(uint4 a, uint4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// features (FP64 arithmetic, rounded to FP32 then to bfloat16), all samples
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LB) void k_features(Mesh m, LfcFeed in, int nsamp, LfcScales sc,
                                                 unsigned short *__restrict__ f) {
#pragma clang fp contract(off)
  const int npix = m.nx * m.ny;
  const long P = (long)blockIdx.x * LB + threadIdx.x;
  if (P >= (long)npix * nsamp) return;
  const int s = (int)(P / npix), p = (int)(P - (long)s * npix);
  const int j = p / m.nx, i = p - j * m.nx;
  const unsigned c = m.o32(i, j + m.j0, 0);
  const double f0 = in.rho[s][c] / sc.rho_s - 1.0;
  const double f1 = in.vy[s][c] / sc.u_s;
  const double f2 = in.vx[s][c] / sc.u_s;
  const double f3 = (m.g.ymed(j + m.j0) - sc.r_mid) / sc.r_span;
  uint2 v;
  v.x = (unsigned)to_bf16((float)f0) | ((unsigned)to_bf16((float)f1) << 16);
  v.y = (unsigned)to_bf16((float)f2) | ((unsigned)to_bf16((float)f3) << 16);
  *reinterpret_cast<uint2 *>(f + (size_t)P * 4) = v;
}

// ---------------------------------------------------------------------------
// 3 x 3 convolution.  A block of four waves takes 64 pixels of CV_RY rows of
// one sample and stages the rows they read, plus one above and below and one
// column on either side (periodic in i, zero rows outside the sample), in
// LDS once; wave w then computes columns 16 w .. 16 w + 15 of every row.
// The weights are the MFMA A operand and stay in registers for the whole
// block (packed per lane by k_pack); the activations are the B operand, one
// 16-byte LDS read per lane per k step.  Modes: CV_HID, out = bf16(relu(conv
// + b)); CV_OUT, out = conv + b (FP32, two channels); CV_ADJ, the adjoint
// convolution, out = bf16([h > 0] conv).
// ---------------------------------------------------------------------------
enum { CV_HID = 0, CV_OUT = 1, CV_ADJ = 2 };
constexpr int CV_RY = 8;

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(int nx, int ny, int ntile, const unsigned short *__restrict__ act,
                                              const uint4 *__restrict__ Wp, const float *__restrict__ bias,
                                              const unsigned short *__restrict__ h, unsigned short *__restrict__ hout,
                                              float *__restrict__ fout) {
  constexpr int MT = (COUT + 15) / 16, KS = (9 * CIN + 31) / 32;
  constexpr int CP = CIN == 32 ? 40 : 4; // staged pixel stride (elements): 16-byte aligned, banks spread
  constexpr int TW = 66, NR = CV_RY + 2;
  constexpr int CH = CIN == 32 ? 4 : 1;   // staged chunks per pixel (16 or 8 bytes)
  constexpr int NE = NR * TW * CH, NL = (NE + 255) / 256;
  __shared__ __align__(16) unsigned short T[NR][TW][CP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, ln = lane & 15, q = lane >> 4;
  const int strips = nx / 64, rt = (ny + CV_RY - 1) / CV_RY;
  uint4 w[MT][KS];
#pragma unroll
  for (int mt = 0; mt < MT; mt++)
#pragma unroll
    for (int ks = 0; ks < KS; ks++) w[mt][ks] = Wp[(mt * KS + ks) * 64 + lane];
  // A block takes tiles blockIdx.x, + gridDim.x, ...: the next tile's rows
  // are loaded into registers while the current one is computed from LDS.
  uint4 pre[NL];
  auto fetch = [&](int tile) {
    const int strip = tile % strips, rtile = (tile / strips) % rt, s = tile / (strips * rt);
    const int x0 = strip * 64, y0 = rtile * CV_RY;
    const size_t sb = (size_t)s * nx * ny;
#pragma unroll
    for (int l = 0; l < NL; l++) {
      const int e = tid + 256 * l;
      const int c8 = e % CH, col = (e / CH) % TW, r = (e / CH) / TW;
      const int yy = y0 + r - 1;
      int xx = x0 + col - 1;
      xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
      pre[l] = make_uint4(0u, 0u, 0u, 0u);
      if (e < NE && yy >= 0 && yy < ny) {
        const unsigned short *src = act + (sb + (size_t)yy * nx + xx) * CIN + 8 * c8;
        if (CIN == 32) pre[l] = *reinterpret_cast<const uint4 *>(src);
        else {
          const uint2 t = *reinterpret_cast<const uint2 *>(src);
          pre[l] = make_uint4(t.x, t.y, 0u, 0u);
        }
      }
    }
  };
  auto put = [&]() {
#pragma unroll
    for (int l = 0; l < NL; l++) {
      const int e = tid + 256 * l;
      if (e >= NE) continue;
      const int c8 = e % CH, col = (e / CH) % TW, r = (e / CH) / TW;
      if (CIN == 32) *reinterpret_cast<uint4 *>(&T[r][col][8 * c8]) = pre[l];
      else *reinterpret_cast<uint2 *>(&T[r][col][0]) = make_uint2(pre[l].x, pre[l].y);
    }
  };
  int tile = blockIdx.x;
  if (tile < ntile) fetch(tile);
  for (; tile < ntile; tile += gridDim.x) {
  __syncthreads(); // the previous tile's reads of T are done
  put();
  __syncthreads();
  const int strip = tile % strips, rtile = (tile / strips) % rt, s = tile / (strips * rt);
  const int x0 = strip * 64, y0 = rtile * CV_RY;
  const size_t sb = (size_t)s * nx * ny; // first pixel of the sample
  const int xl = wv * 16 + ln; // the lane's pixel (B column) within the 64
  const int nrow = min(CV_RY, ny - y0);
  // CV_ADJ: the ReLU mask of the tile's outputs is loaded before its
  // products, and before the next tile's rows (the loads are waited for in
  // issue order), so that the epilogue does not wait for memory; rows past
  // the sample load its last row (no branch around the loads)
  uint2 hm[MODE == CV_ADJ ? CV_RY : 1][MT];
  if constexpr (MODE == CV_ADJ) {
#pragma unroll
    for (int rr = 0; rr < CV_RY; rr++) {
      const size_t p = sb + (size_t)(y0 + min(rr, nrow - 1)) * nx + x0 + xl;
#pragma unroll
      for (int mt = 0; mt < MT; mt++) hm[rr][mt] = *reinterpret_cast<const uint2 *>(h + p * COUT + 16 * mt + 4 * q);
    }
  }
  if (tile + (int)gridDim.x < ntile) fetch(tile + gridDim.x);
#pragma unroll
  for (int r = 0; r < CV_RY; r += 2) {
    if (r >= nrow) break;
    f4 acc[2][MT];
#pragma unroll
    for (int rr = 0; rr < 2; rr++)
#pragma unroll
      for (int mt = 0; mt < MT; mt++) acc[rr][mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
#pragma unroll
      for (int rr = 0; rr < 2; rr++) {
        uint4 b;
        if (CIN == 32) { // k step = tap, lane group = 8 channels
          b = *reinterpret_cast<const uint4 *>(&T[r + rr + ks / 3][xl + ks % 3][8 * q]);
        } else { // k step = 8 taps of 4 channels, lane group = 2 taps
          const int ta = 8 * ks + 2 * q, tb = ta + 1;
          uint2 lo = make_uint2(0u, 0u), hi = make_uint2(0u, 0u);
          if (ta < 9) lo = *reinterpret_cast<const uint2 *>(&T[r + rr + ta / 3][xl + ta % 3][0]);
          if (tb < 9) hi = *reinterpret_cast<const uint2 *>(&T[r + rr + tb / 3][xl + tb % 3][0]);
          b = make_uint4(lo.x, lo.y, hi.x, hi.y);
        }
#pragma unroll
        for (int mt = 0; mt < MT; mt++) acc[rr][mt] = mfma(w[mt][ks], b, acc[rr][mt]);
      }
    }
#pragma unroll
    for (int rr = 0; rr < 2; rr++) {
      if (r + rr >= nrow) break;
      const size_t p = sb + (size_t)(y0 + r + rr) * nx + x0 + xl;
#pragma unroll
      for (int mt = 0; mt < MT; mt++) {
        const int co = 16 * mt + 4 * q;
        const f4 a = acc[rr][mt];
        if (MODE == CV_HID) {
          const float v0 = fmaxf(a[0] + bias[co], 0.f), v1 = fmaxf(a[1] + bias[co + 1], 0.f);
          const float v2 = fmaxf(a[2] + bias[co + 2], 0.f), v3 = fmaxf(a[3] + bias[co + 3], 0.f);
          *reinterpret_cast<uint2 *>(hout + p * COUT + co) = make_uint2(pack2(v0, v1), pack2(v2, v3));
        } else if (MODE == CV_OUT) {
          if (q == 0) *reinterpret_cast<float2 *>(fout + p * 2) = make_float2(a[0] + bias[0], a[1] + bias[1]);
        } else {
          const uint2 hv = hm[MODE == CV_ADJ ? r + rr : 0][mt];
          const float v0 = lo_bf16(hv.x) > 0.f ? a[0] : 0.f, v1 = hi_bf16(hv.x) > 0.f ? a[1] : 0.f;
          const float v2 = lo_bf16(hv.y) > 0.f ? a[2] : 0.f, v3 = hi_bf16(hv.y) > 0.f ? a[3] : 0.f;
          *reinterpret_cast<uint2 *>(hout + p * COUT + co) = make_uint2(pack2(v0, v1), pack2(v2, v3));
        }
      }
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

__global__ __launch_bounds__(LB) void k_drho(Mesh m, int nsamp, const float *__restrict__ o, double sF,
                                             LfcTargets tg, int with_target, double sigma,
                                             double *__restrict__ drho, double *__restrict__ gD,
                                             double *__restrict__ lpart) {
#pragma clang fp contract(off)
  __shared__ double red[LB / 64];
  const int nx = m.nx, ny = m.ny, npix = nx * ny;
  const long ntot = (long)npix * nsamp;
  const long P = (long)blockIdx.x * LB + threadIdx.x;
  double e2 = 0.0;
  if (P < ntot) {
    const int s = (int)(P / npix), p = (int)(P - (long)s * npix);
    const int j = p / nx, i = p - j * nx;
    const long b = (long)s * npix;
    const long pr = b + j * nx + (i + 1 == nx ? 0 : i + 1), pu = P + nx;
    const double fx0 = sF * (double)o[2 * P], fx1 = sF * (double)o[2 * pr];
    const double fy0 = j == 0 ? 0.0 : sF * (double)o[2 * P + 1];
    const double fy1 = j + 1 == ny ? 0.0 : sF * (double)o[2 * pu + 1];
    const double div = (fx1 - fx0) + (fy1 - fy0);
    const double iv = m.g.invVj(j + m.j0);
    const double d = (-iv) * div;
    drho[P] = d;
    if (with_target) {
      const double t = tg.t[s][p];
      const double e = (d - t) / sigma;
      e2 = e * e;
      const double g = 2.0 * (d - t) / ((double)ntot * sigma * sigma);
      gD[P] = (-iv) * g;
    }
  }
  if (!with_target) return;
  const double s = block_sum(e2, red);
  if (threadIdx.x == 0) lpart[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_loss_final(const double *__restrict__ lpart, int n, long ntot,
                                                    double *__restrict__ loss) {
  __shared__ double red[4];
  double s = 0.0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) s += lpart[q];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *loss = s / (double)ntot;
}

// dL/d(net output) through the adjoint of the divergence; 4 channels (the
// last two zero) so that the input-gradient GEMM takes them in groups of 4
__global__ __launch_bounds__(LB) void k_flux_grad(int nx, int ny, int nsamp, const double *__restrict__ gD, double sF,
                                                  unsigned short *__restrict__ g3) {
#pragma clang fp contract(off)
  const int npix = nx * ny;
  const long P = (long)blockIdx.x * LB + threadIdx.x;
  if (P >= (long)npix * nsamp) return;
  const int s = (int)(P / npix), p = (int)(P - (long)s * npix);
  const int j = p / nx, i = p - j * nx;
  const long b = (long)s * npix;
  const double gx = gD[b + j * nx + (i == 0 ? nx - 1 : i - 1)] - gD[P];
  const double gy = j == 0 ? 0.0 : gD[P - nx] - gD[P];
  uint2 v;
  v.x = (unsigned)to_bf16((float)(sF * gx)) | ((unsigned)to_bf16((float)(sF * gy)) << 16);
  v.y = 0u;
  *reinterpret_cast<uint2 *>(g3 + (size_t)P * 4) = v;
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][tap CIN + ci] = sum_p g[p][co] act[p shifted by
// tap][ci] over the pixels of a block: a 64-pixel column strip of one sample
// over a run of rows, taken CW_RG rows at a time.  K of the MFMA runs over
// pixels, so both operands are staged in LDS transposed, [channel][pixel]:
// the layer gradient of the group's rows and the activation rows from one
// above to one below them.  A staging thread loads four consecutive pixels'
// 16-byte channel chunks and writes each channel's four values as one 8-byte
// store (byte permutes in registers).  The next group's global loads are
// issued into registers before the current group is computed.  A lane's
// eight pixels are consecutive; the three taps along i read one 24-byte
// window and shift it by -2, 0 or +2 bytes.  Six waves: for 32 input
// channels wave w takes the row offset ty = w / 2 and 16 channels, all three
// tx; for 4 it takes one 16-wide column tile of the 36 (tap, ci) pairs and
// one 16-wide tile of output channels.  One partial sum per block, for the
// reduction below, and the bias gradient (the sum of g) alongside.
// ---------------------------------------------------------------------------
constexpr int CW_THREADS = 384, CW_RG = 4;
constexpr int CW_AW = 80; // staged activation columns: pixel x0 - 1 + c - 7 at column c (7..72)
constexpr int CW_GW = 72; // staged layer-gradient columns: pixel x0 + c (0..63)

// the B operand of tap column tx (0..2) from the window around LDS column c
// (16-byte aligned): columns c - 1 + tx .. c + 6 + tx
__device__ inline uint4 tap_run(const unsigned short *ap, int tx) {
  const unsigned dm = *reinterpret_cast<const unsigned *>(ap - 2);
  const uint4 d = *reinterpret_cast<const uint4 *>(ap);
  const unsigned dp = *reinterpret_cast<const unsigned *>(ap + 8);
  if (tx == 1) return d;
  const bool lo = tx == 0;
  return make_uint4(__builtin_amdgcn_alignbyte(lo ? d.x : d.y, lo ? dm : d.x, 2),
                    __builtin_amdgcn_alignbyte(lo ? d.y : d.z, lo ? d.x : d.y, 2),
                    __builtin_amdgcn_alignbyte(lo ? d.z : d.w, lo ? d.y : d.z, 2),
                    __builtin_amdgcn_alignbyte(lo ? d.w : dp, lo ? d.z : d.w, 2));
}

__device__ inline unsigned dword(const uint4 &v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

// channel k of four pixels' chunks as four consecutive bfloat16
__device__ inline uint2 chan4(const uint4 &p0, const uint4 &p1, const uint4 &p2, const uint4 &p3, int k) {
  const unsigned sel = (k & 1) ? 0x07060302u : 0x05040100u;
  return make_uint2(__builtin_amdgcn_perm(dword(p1, k >> 1), dword(p0, k >> 1), sel),
                    __builtin_amdgcn_perm(dword(p3, k >> 1), dword(p2, k >> 1), sel));
}

template <int CIN, int COUT, int GC>
__global__ __launch_bounds__(CW_THREADS) void k_conv_w(int nx, int ny, int rpc, int nrc,
                                                       const unsigned short *__restrict__ g,
                                                       const unsigned short *__restrict__ act,
                                                       float *__restrict__ part, float *__restrict__ dbpart) {
  constexpr int MT = (COUT + 15) / 16, K = 9 * CIN;
  constexpr int NA = CIN == 32 ? 3 : 1;  // accumulator tiles per M tile
  constexpr int AR = CW_RG + 2;          // staged activation rows
  constexpr int ACH = CIN == 32 ? 4 : 1; // channel chunks of 8 (or 4) per pixel
  constexpr int GCH = GC == 32 ? 4 : 1;
  constexpr int NAT = AR * 16 * ACH;     // activation tasks (4 pixels x one chunk) of a group
  constexpr int NHT = AR * 2 * ACH;      // halo tasks (one pixel x one chunk)
  constexpr int NGT = CW_RG * 16 * GCH;  // layer-gradient tasks
  constexpr int NAL = (NAT + CW_THREADS - 1) / CW_THREADS;
  static_assert(NHT <= CW_THREADS && NGT <= CW_THREADS, "one halo and one gradient task per thread");
  constexpr int A_BYTES = AR * CIN * CW_AW * 2, G_BYTES = CW_RG * 16 * MT * CW_GW * 2;
  constexpr int DB_BYTES = CW_THREADS * 8 * 4;
  constexpr int LDS_BYTES = A_BYTES + G_BYTES > DB_BYTES ? A_BYTES + G_BYTES : DB_BYTES;
  __shared__ __align__(16) unsigned char lds[LDS_BYTES];
  auto At = reinterpret_cast<unsigned short(*)[CIN][CW_AW]>(lds);
  auto Gt = reinterpret_cast<unsigned short(*)[16 * MT][CW_GW]>(lds + A_BYTES);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, ln = lane & 15, q = lane >> 4;
  const int strips = nx / 64;
  const int strip = blockIdx.x % strips, rc = (blockIdx.x / strips) % nrc, s = blockIdx.x / (strips * nrc);
  const int x0 = strip * 64, ya = rc * rpc, yb = min(ny, ya + rpc);
  const size_t sb = (size_t)s * nx * ny;
  // rows of the output-channel tile beyond COUT stay zero
  if (COUT < 16 * MT)
    for (int e = tid; e < CW_RG * (16 * MT - COUT) * CW_GW; e += CW_THREADS) {
      const int b = e / ((16 * MT - COUT) * CW_GW), r = e % ((16 * MT - COUT) * CW_GW);
      Gt[b][COUT + r / CW_GW][r % CW_GW] = 0;
    }
  auto ld = [&](const unsigned short *src, int wide) -> uint4 {
    if (wide) return *reinterpret_cast<const uint4 *>(src);
    const uint2 t = *reinterpret_cast<const uint2 *>(src);
    return make_uint4(t.x, t.y, 0u, 0u);
  };
  // a group's global loads, into registers: activation rows y - 1 .. y + CW_RG
  // (zero outside the sample) and layer-gradient rows y .. y + CW_RG - 1 (zero
  // from yb on)
  uint4 ra[NAL][4], rh, rg[4];
  auto load = [&](int y) {
#pragma unroll
    for (int i = 0; i < NAL; i++) {
      const int t = tid + CW_THREADS * i;
      const int r = t / (16 * ACH), w = t % (16 * ACH), m = w / ACH, c8 = w % ACH;
      const int yy = y + r - 1;
      const bool ok = t < NAT && yy >= 0 && yy < ny;
      const unsigned short *src = act + (sb + (size_t)(ok ? yy : 0) * nx + x0 + 4 * m) * CIN + 8 * c8;
#pragma unroll
      for (int u = 0; u < 4; u++) ra[i][u] = ok ? ld(src + u * CIN, CIN == 32) : make_uint4(0u, 0u, 0u, 0u);
    }
    {
      const int r = tid / (2 * ACH), w = tid % (2 * ACH), side = w / ACH, c8 = w % ACH;
      const int yy = y + r - 1;
      int xx = side ? x0 + 64 : x0 - 1;
      xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
      const bool ok = tid < NHT && yy >= 0 && yy < ny;
      rh = ok ? ld(act + (sb + (size_t)yy * nx + xx) * CIN + 8 * c8, CIN == 32) : make_uint4(0u, 0u, 0u, 0u);
    }
    {
      const int r = tid / (16 * GCH), w = tid % (16 * GCH), m = w / GCH, c8 = w % GCH;
      const bool ok = tid < NGT && y + r < yb;
      const unsigned short *src = g + (sb + (size_t)(ok ? y + r : 0) * nx + x0 + 4 * m) * GC + 8 * c8;
#pragma unroll
      for (int u = 0; u < 4; u++) rg[u] = ok ? ld(src + u * GC, GC == 32) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  // the registers into LDS, transposed; the bias sums of the thread's
  // layer-gradient channels (fixed per thread)
  float db[8];
#pragma unroll
  for (int i = 0; i < 8; i++) db[i] = 0.f;
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < NAL; i++) {
      const int t = tid + CW_THREADS * i;
      if (t < NAT) {
        const int r = t / (16 * ACH), w = t % (16 * ACH), m = w / ACH, c0 = 8 * (w % ACH);
#pragma unroll
        for (int k = 0; k < (CIN == 32 ? 8 : 4); k++)
          *reinterpret_cast<uint2 *>(&At[r][c0 + k][8 + 4 * m]) = chan4(ra[i][0], ra[i][1], ra[i][2], ra[i][3], k);
      }
    }
    if (tid < NHT) {
      const int r = tid / (2 * ACH), w = tid % (2 * ACH), side = w / ACH, c0 = 8 * (w % ACH);
#pragma unroll
      for (int k = 0; k < (CIN == 32 ? 8 : 4); k++) {
        const unsigned u = dword(rh, k >> 1);
        At[r][c0 + k][side ? 72 : 7] = (unsigned short)(k & 1 ? u >> 16 : u & 0xFFFFu);
      }
    }
    if (tid < NGT) {
      const int r = tid / (16 * GCH), w = tid % (16 * GCH), m = w / GCH, c0 = 8 * (w % GCH);
#pragma unroll
      for (int k = 0; k < (GC == 32 ? 8 : COUT); k++) {
        const uint2 v = chan4(rg[0], rg[1], rg[2], rg[3], k);
        *reinterpret_cast<uint2 *>(&Gt[r][c0 + k][4 * m]) = v;
        db[k] += (lo_bf16(v.x) + hi_bf16(v.x)) + (lo_bf16(v.y) + hi_bf16(v.y));
      }
    }
  };
  f4 acc[NA][MT];
#pragma unroll
  for (int a = 0; a < NA; a++)
#pragma unroll
    for (int mt = 0; mt < MT; mt++) acc[a][mt] = f4{0.f, 0.f, 0.f, 0.f};
  // the wave's operands: for CIN = 32, row offset ty and channel ci; for 4,
  // the (tap, ci) pair of its column tile and its output-channel tile
  int ty, ci, tx = 0, mt1 = 0;
  bool kok = true;
  if (CIN == 32) {
    ty = wv >> 1;
    ci = 16 * (wv & 1) + ln;
  } else {
    const int kk = 16 * (wv % 3) + ln, tap = kk >> 2;
    kok = kk < K;
    ty = kok ? tap / 3 : 0;
    tx = kok ? tap % 3 : 0;
    ci = kk & 3;
    mt1 = wv / 3;
  }
  load(ya);
  for (int y = ya; y < yb; y += CW_RG) {
    store();
    __syncthreads();
    if (y + CW_RG < yb) load(y + CW_RG);
    const int nr = min(CW_RG, yb - y);
    for (int rr = 0; rr < nr; rr++) {
#pragma unroll
      for (int ks = 0; ks < 2; ks++) {
        const int c0 = 32 * ks + 8 * q;
        const unsigned short *ap = &At[rr + ty][ci][8 + c0];
        if (CIN == 32) {
          const uint4 b0 = tap_run(ap, 0), b1 = tap_run(ap, 1), b2 = tap_run(ap, 2);
#pragma unroll
          for (int mt = 0; mt < MT; mt++) {
            const uint4 a = *reinterpret_cast<const uint4 *>(&Gt[rr][16 * mt + ln][c0]);
            acc[0][mt] = mfma(a, b0, acc[0][mt]);
            acc[1][mt] = mfma(a, b1, acc[1][mt]);
            acc[2][mt] = mfma(a, b2, acc[2][mt]);
          }
        } else {
          uint4 b = tap_run(ap, tx);
          if (!kok) b = make_uint4(0u, 0u, 0u, 0u);
          const uint4 a = *reinterpret_cast<const uint4 *>(&Gt[rr][16 * mt1 + ln][c0]);
          acc[0][0] = mfma(a, b, acc[0][0]);
        }
      }
    }
    __syncthreads();
  }
  // results: lane holds column ln of its tiles and rows 4 q .. 4 q + 3 (one
  // row of LFC_NPARAM partials per block, in the parameter vector's order)
  float *pw = part + (size_t)blockIdx.x * LFC_NPARAM;
  if (CIN == 32) {
#pragma unroll
    for (int a = 0; a < NA; a++)
#pragma unroll
      for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int co = 16 * mt + 4 * q + v;
          if (co < COUT) pw[co * K + (3 * ty + a) * 32 + ci] = acc[a][mt][v];
        }
  } else if (kok) {
    const int kk = 16 * (wv % 3) + ln;
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int co = 16 * mt1 + 4 * q + v;
      if (co < COUT) pw[co * K + kk] = acc[0][0][v];
    }
  }
  // bias gradient: the threads' channel sums, added in thread order (the LDS
  // of the staging is free after the last barrier of the loop)
  float(*dbr)[8] = reinterpret_cast<float(*)[8]>(lds);
#pragma unroll
  for (int k = 0; k < 8; k++) dbr[tid][k] = db[k];
  __syncthreads();
  if (tid < COUT) {
    const int c8 = GC == 32 ? tid >> 3 : 0, k = GC == 32 ? tid & 7 : tid;
    float t = 0.f;
    for (int u = c8; u < NGT; u += GCH) t += dbr[u][k];
    dbpart[(size_t)blockIdx.x * LFC_NPARAM + tid] = t;
  }
}

// The gradient of every parameter: the sum over blocks of the weight-gradient
// kernels' partials (one row of LFC_NPARAM per block, all three layers in one
// launch).  A block takes RE consecutive parameters; its RG thread groups sum
// interleaved subsets of the rows, and the group sums are added in a fixed
// order (deterministic).
constexpr int RE = 64, RG = 16;
__global__ __launch_bounds__(RE * RG) void k_reduce_w(int nchunk, const float *__restrict__ part,
                                                      float *__restrict__ grad) {
  __shared__ float red[RG][RE];
  const int el = threadIdx.x % RE, g = threadIdx.x / RE;
  const int e = blockIdx.x * RE + el;
  float s = 0.f;
  if (e < LFC_NPARAM) {
#pragma unroll 8
    for (int c = g; c < nchunk; c += RG) s += part[(size_t)c * LFC_NPARAM + e];
  }
  red[g][el] = s;
  __syncthreads();
  if (g == 0 && e < LFC_NPARAM) {
    float t = 0.f;
    for (int q = 0; q < RG; q++) t += red[q][el];
    grad[e] = t;
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

// bfloat16 weight matrices of the five convolutions, packed as MFMA A
// operands: entry ((mt KS + ks) 64 + lane) 8 + e holds row 16 mt + lane % 16,
// k = 32 ks + 8 (lane / 16) + e (zero beyond K).  Rows and k of each matrix:
//   L1  [co][tap 4 + ci]        L2, L3  [co][tap 32 + ci]
//   A3  [ci][tap' 4 + cg]       A2      [ci][tap' 32 + cg]
// with the adjoint's taps flipped, tap' = 8 - tap, and cg = 2, 3 zero in A3.
__device__ inline float lfc_wm(const float *w, int which, int row, int k) {
  const float *W1 = w + LFC_OFF_W1, *W2 = w + LFC_OFF_W2, *W3 = w + LFC_OFF_W3;
  switch (which) {
  case 0: return k < 36 ? W1[row * 36 + k] : 0.f;
  case 1: return W2[row * 288 + k];
  case 2: return row < 2 ? W3[row * 288 + k] : 0.f;
  case 3: {
    if (k >= 36) return 0.f;
    const int tap = k >> 2, cg = k & 3;
    return cg < 2 ? W3[cg * 288 + (8 - tap) * 32 + row] : 0.f;
  }
  default: {
    const int tap = k >> 5, cg = k & 31;
    return W2[cg * 288 + (8 - tap) * 32 + row];
  }
  }
}

__global__ __launch_bounds__(LB) void k_pack(const float *__restrict__ w, LfcWeights b) {
  const int e = blockIdx.x * LB + threadIdx.x;
  const int mts[5] = {2, 2, 1, 2, 2}, kss[5] = {2, 9, 9, 2, 9}, ks36[5] = {36, 288, 288, 36, 288};
  unsigned short *dst[5] = {b.wp1, b.wp2, b.wp3, b.wpa3, b.wpa2};
#pragma unroll
  for (int c = 0; c < 5; c++) {
    const int n = mts[c] * kss[c] * 512;
    if (e >= n) continue;
    const int el = e & 7, lane = (e >> 3) & 63, blk = e >> 9, ks = blk % kss[c], mt = blk / kss[c];
    const int row = 16 * mt + (lane & 15), k = 32 * ks + 8 * (lane >> 4) + el;
    dst[c][e] = k < ks36[c] ? to_bf16(lfc_wm(w, c, row, k)) : (unsigned short)0;
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

// tiles (64 pixels of CV_RY rows of one sample) of a convolution, and its
// grid: the tiles, or as many workgroups as the compute units hold at once
// (per unit: two of the 32-to-32-channel forms, three of the 32-to-2, five
// of the 4-channel forward and four of the 4-channel adjoint, by their
// registers) looping over them
inline int conv_tiles(const Mesh &m, int nsamp) { return nsamp * (m.nx / 64) * ((m.ny + CV_RY - 1) / CV_RY); }
inline unsigned conv_grid(int ntile, int per_cu) {
  return (unsigned)(ntile < per_cu * 256 ? ntile : per_cu * 256);
}

} // namespace

// Blocks of the weight-gradient kernels: nsamp x (nx / 64) strips, each split
// into row chunks of rpc rows, so that there are at most 512 blocks (two per
// compute unit, all resident at once) where the strips allow.
int lfc_wblocks(int nx, int ny, int nsamp, int *rpc, int *nrc) {
  const int strips = nsamp * (nx / 64);
  int want = 512 / strips;
  want = want < 1 ? 1 : (want > ny ? ny : want);
  const int r = (ny + want - 1) / want;
  if (rpc) *rpc = r;
  if (nrc) *nrc = (ny + r - 1) / r;
  return strips * ((ny + r - 1) / r);
}

void lfc_forward(Launch &L, const Mesh &m, const LfcFeed &in, int nsamp, const LfcScales &sc, const LfcBufs &B) {
  const long ntot = (long)m.nx * m.ny * nsamp;
  prof_begin(L, K_LFC_FEATURES);
  k_features<<<nblk(ntot, LB), LB, 0, L.s>>>(m, in, nsamp, sc, B.f);
  prof_end(L, K_LFC_FEATURES);
  const int nt = conv_tiles(m, nsamp);
  const unsigned nb = conv_grid(nt, 2), nb3 = conv_grid(nt, 3), nb5 = conv_grid(nt, 5);
  const uint4 *wp1 = (const uint4 *)B.wt.wp1, *wp2 = (const uint4 *)B.wt.wp2, *wp3 = (const uint4 *)B.wt.wp3;
  prof_begin(L, K_LFC_FWD1);
  k_conv<4, 32, CV_HID><<<nb5, 256, 0, L.s>>>(m.nx, m.ny, nt, B.f, wp1, B.w + LFC_OFF_B1, nullptr, B.h1, nullptr);
  prof_end(L, K_LFC_FWD1);
  prof_begin(L, K_LFC_FWD2);
  k_conv<32, 32, CV_HID><<<nb, 256, 0, L.s>>>(m.nx, m.ny, nt, B.h1, wp2, B.w + LFC_OFF_B2, nullptr, B.h2, nullptr);
  prof_end(L, K_LFC_FWD2);
  prof_begin(L, K_LFC_FWD3);
  k_conv<32, 2, CV_OUT><<<nb3, 256, 0, L.s>>>(m.nx, m.ny, nt, B.h2, wp3, B.w + LFC_OFF_B3, nullptr, nullptr, B.o);
  prof_end(L, K_LFC_FWD3);
}

void lfc_drho(Launch &L, const Mesh &m, int nsamp, const LfcBufs &B, double sF, const LfcTargets *tg,
              double sigma) {
  const long ntot = (long)m.nx * m.ny * nsamp;
  const unsigned nb = nblk(ntot, LB);
  LfcTargets none{};
  prof_begin(L, K_LFC_DRHO);
  k_drho<<<nb, LB, 0, L.s>>>(m, nsamp, B.o, sF, tg ? *tg : none, tg ? 1 : 0, sigma, B.drho, B.gD, B.lpart);
  prof_end(L, K_LFC_DRHO);
  if (tg) {
    prof_begin(L, K_LFC_DRHO);
    k_loss_final<<<1, 256, 0, L.s>>>(B.lpart, (int)nb, ntot, B.loss);
    prof_end(L, K_LFC_DRHO);
  }
}

void lfc_backward(Launch &L, const Mesh &m, int nsamp, const LfcBufs &B, double sF) {
  const int nx = m.nx, ny = m.ny;
  const long ntot = (long)nx * ny * nsamp;
  const int nt = conv_tiles(m, nsamp);
  const unsigned nb = conv_grid(nt, 2), nb4 = conv_grid(nt, 4);
  int rpc = 1, nrc = 1;
  const int nw = lfc_wblocks(nx, ny, nsamp, &rpc, &nrc);
  prof_begin(L, K_LFC_DRHO);
  k_flux_grad<<<nblk(ntot, LB), LB, 0, L.s>>>(nx, ny, nsamp, B.gD, sF, B.g3);
  prof_end(L, K_LFC_DRHO);
  // layer 3: weights from g3 and h2, then the gradient into h2
  prof_begin(L, K_LFC_W3);
  k_conv_w<32, 2, 4><<<nw, CW_THREADS, 0, L.s>>>(nx, ny, rpc, nrc, B.g3, B.h2, B.part + LFC_OFF_W3,
                                                 B.part + LFC_OFF_B3);
  prof_end(L, K_LFC_W3);
  prof_begin(L, K_LFC_ADJ3);
  k_conv<4, 32, CV_ADJ><<<nb4, 256, 0, L.s>>>(nx, ny, nt, B.g3, (const uint4 *)B.wt.wpa3, nullptr, B.h2, B.g2, nullptr);
  prof_end(L, K_LFC_ADJ3);
  // layer 2
  prof_begin(L, K_LFC_W2);
  k_conv_w<32, 32, 32><<<nw, CW_THREADS, 0, L.s>>>(nx, ny, rpc, nrc, B.g2, B.h1, B.part + LFC_OFF_W2,
                                                   B.part + LFC_OFF_B2);
  prof_end(L, K_LFC_W2);
  prof_begin(L, K_LFC_ADJ2);
  k_conv<32, 32, CV_ADJ><<<nb, 256, 0, L.s>>>(nx, ny, nt, B.g2, (const uint4 *)B.wt.wpa2, nullptr, B.h1, B.g1, nullptr);
  prof_end(L, K_LFC_ADJ2);
  // layer 1 (no gradient into the features)
  prof_begin(L, K_LFC_W1);
  k_conv_w<4, 32, 32><<<nw, CW_THREADS, 0, L.s>>>(nx, ny, rpc, nrc, B.g1, B.f, B.part + LFC_OFF_W1,
                                                  B.part + LFC_OFF_B1);
  prof_end(L, K_LFC_W1);
  // every parameter's gradient in one reduction
  prof_begin(L, K_LFC_REDUCE);
  k_reduce_w<<<nblk(LFC_NPARAM, RE), RE * RG, 0, L.s>>>(nw, B.part, B.grad);
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
  k_pack<<<nblk(2 * 9 * 512, LB), LB, 0, L.s>>>(B.w, B.wt);
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
