// Box 7: source step (Sect. 3.3), boxes 7a, 7b and 7c fused in one pass.
//   7a  pressure and potential gradients on the owned faces, centrifugal
//       terms as squares of four-point arithmetic averages (Eq. 12 and its
//       generalisation); Jacobi: every face reads only v^n.  The pressure
//       term uses the arithmetic mean of the two face densities (Eq. 20),
//       which makes it momentum conserving (Eqs. 21-25).
//   7b  von Neumann-Richtmyer artificial viscosity per direction,
//       q = C^2 rho dv^2 where dv < 0, its gradient in the same conservative
//       form, and the heating -q dv / L.
//   7c  compressional heating of a gamma-law gas, time-centred:
//       e <- e (1 - a)/(1 + a), a = dt (gamma - 1) div(v) / 2.
// A zone owns its lower X, Y and Z faces (the lower Y/Z boundary face only in
// a periodic direction); faces that are not owned keep v^n.  Results go to
// separate arrays (v'', e''), so the pass reads the state while it writes.
//
// Layout of the work: a workgroup takes a tile of TX x TY zones of one (X, Y)
// plane and marches through the Z planes.  For each plane the tile and a halo
// of two zones in X and Y are staged in LDS; the v' of every X and Y face of
// the tile (and of the halo faces its stencil needs) is computed once and
// kept in LDS (with the reciprocal of its density sum where room is left),
// then each zone forms q on its neighbours and its v'' and e''.  Along Z each
// thread keeps a sliding window of its own column in registers (planes
// k-1 .. k+2), which also
// supplies the tile's interior values to LDS, so each interior value is read
// from memory once.  Geometric lengths enter through reciprocal tables.
//
// The field type F is double, or float for the FP32-bulk state; arithmetic is
// carried out in F, geometric factors are rounded to F where they are used.
// An FP32 v_x is a deviation from its ring's FP64 background vb: the X-face
// update acts on it unchanged, and each centrifugal term splits into the
// square of the background (vb + R Omega), formed in FP64 together with the
// potential gradient it nearly cancels and rounded once, and the FP32 terms
// of the deviation.
#include <type_traits>

#include "fargo_internal.h"

namespace fargo {

namespace {

constexpr int TX = 64, SX = TX + 4; // tile width, with two halo zones on each side
// Tile height (one wave per tile row).  The Y halo of a tile is read once per
// tile, so taller tiles read less of it.  The FP64 3D march takes 16 rows
// (1024 threads, at most 128 registers a thread), or 12 where the spherical or
// adiabatic terms need more registers; FP32 marches and 2D meshes take 8
// (two workgroups per compute unit; the FP32 march measured slower with
// taller tiles).
template <typename F, bool D3, int GEO, bool ADI>
constexpr int tile_rows() {
  if (!D3 || sizeof(F) == 4) return 8;
  return ADI || GEO == FARGO_SPHERICAL ? 12 : 16;
}
template <typename F, bool D3, int GEO, bool ADI>
constexpr int src_threads() { return 64 * tile_rows<F, D3, GEO, ADI>(); }
// minimum waves per SIMD: one workgroup of the FP64 march per compute unit,
// at least four waves of the others
template <typename F, bool D3, int GEO, bool ADI>
constexpr int src_waves() {
  return sizeof(F) == 8 && D3 ? src_threads<F, D3, GEO, ADI>() / 256 : 4;
}

template <typename F>
__device__ inline F qvisc(F c2, F rho, F dv) { return dv < F(0) ? c2 * rho * dv * dv : F(0); }

template <typename F, int TY, int NB, bool SPH, bool KI>
struct Lds {
  // staging of a plane (NB planes in flight; density NB + 1 when NB > 1)
  static constexpr int SY = TY + 4, NR = NB > 1 ? NB + 1 : 1;
  F R[NR][SY][SX];      // density
  F P[NB][SY][SX];      // pressure
  double Ph[NB][SY][SX]; // potential (FP64 in every mode)
  F VX[NB][SY][SX];     // v_x on the lower X face of each zone slot
  F VY[NB][SY][TX];     // v_y on the lower Y face of each zone slot
  F VT[SPH ? NB : 1][SPH ? SY : 1][SPH ? TX : 1]; // spherical: v_theta on the zone's two Z faces, summed
  // v' of the faces of a plane (NB planes in flight)
  F AX[NB][TY][SX];     // v'_x of X faces of the tile rows
  F AY[NB][SY][TX];     // v'_y of Y faces
  F IX[KI ? NB : 1][KI ? TY : 1][KI ? SX : 1]; // KI: 1 / ((rho_i + rho_{i-1}) dX) on the X faces
  F IY[KI ? NB : 1][KI ? SY : 1][KI ? TX : 1]; // KI: 1 / ((rho_j + rho_{j-1}) h_y) on the Y faces
  double DX[NB][TY];    // 1 / dX of the tile rows, for the halo X faces
};
// (a 2D mesh has a single plane: one buffer of each, so that several
// workgroups share a compute unit)
constexpr size_t LDS_CU = 160 * 1024;
// the reciprocals of the faces' density sums are kept in LDS where they fit
// beside the rest, else formed again by the zones that use them
template <typename F, int TY, int NB, bool SPH>
constexpr bool keep_inv() { return sizeof(Lds<F, TY, NB, SPH, true>) <= LDS_CU; }

// An explicit register move.  The march keeps a window of plane records in
// registers and rotates it once per plane; moving the newest record out of its
// registers before the next plane's loads are issued lets those loads write
// the same registers, instead of temporaries whose copy into the window would
// wait for the loads to arrive.
template <typename T>
__device__ inline T vmove(T x) {
  T y;
  if constexpr (sizeof(T) == 8) asm("v_mov_b64 %0, %1" : "=v"(y) : "v"(x));
  else asm("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
  return y;
}

// A value the compiler is to keep in vector registers (every lane of a wave
// holding the same value), which leaves the scalar registers to the values
// that change along the march.
template <typename T>
__device__ inline T vreg(T x) {
  asm("" : "+v"(x));
  return x;
}

// one zone's values in one plane
template <typename F>
struct Zv {
  F rho, q; // q: sound speed (isothermal) or internal energy (adiabatic)
  double pot;
  F vz, vx, vxp; // vxp: v_x on the next X face
};

// A plane goes through three phases: staging into LDS (S), v' of its faces
// (F), and the zones (Z).  The march is software-pipelined over planes: one
// barrier interval runs Z(k), F(k+1) and S(k+2) on separate buffers, so each
// plane costs one barrier and the three phases overlap.
// The geometry and the equation of state are template parameters: fewer
// run-time conditions leave more scalar registers for the march.
template <typename F, bool D3, int GEO, bool ADI>
__device__ __forceinline__ void source_body(Mesh m, StateT<F> s, const double *__restrict__ dtp,
                                                  F *__restrict__ vx2, F *__restrict__ vy2, F *__restrict__ vz2,
                                                  F *__restrict__ e2, int nbx, int nby, unsigned bid_, unsigned nbk_) {
  constexpr int TY = tile_rows<F, D3, GEO, ADI>(), NB = D3 ? 2 : 1;
  constexpr bool KI = keep_inv<F, TY, NB, GEO == FARGO_SPHERICAL>();
  __shared__ Lds<F, TY, NB, GEO == FARGO_SPHERICAL, KI> L;
  static_assert(sizeof(L) <= LDS_CU, "source step tile exceeds the LDS of a compute unit");
  // the row is the wave index: uniform, so that geometric factors of the
  // row come through scalar loads, which do not stall behind the prefetches
  const int tid = threadIdx.x, r = __builtin_amdgcn_readfirstlane(tid >> 6), c = tid & 63;
  // Tiles in groups of G tile rows, Y fastest within a group.  The 16-row
  // FP64 march takes groups of 4: the 32 workgroups an XCD runs at once then
  // cover a patch 8 tiles wide and 4 tall, so that the X halo zones a tile
  // reads (each a 128-byte line of its neighbour's row) are mostly a running
  // neighbour's own, still in L2 (2.60 to 2.36 ms on the 2048 x 768 x 96 disk).
  // The FP32 march (two workgroups per compute unit) takes groups of 4 as well:
  // 29 % fewer bytes fetched, about as fast.  The 12-row spherical march and
  // 2D meshes keep Y fastest over the whole mesh (G = nby), which measured
  // faster for the former.
  const int G = TY == 16 || (D3 && sizeof(F) == 4) ? 4 : nby;
  const unsigned Lb = xcd_remap(bid_, nbk_), gsz = (unsigned)(G * nbx);
  const unsigned grp = Lb / gsz, idx = Lb % gsz, gy = (unsigned)min(G, nby - (int)grp * G);
  const int ty = (int)(grp * (unsigned)G + idx % gy), tx = (int)(idx / gy);
  const int i0 = tx * TX, jt0 = m.j0 + ty * TY;
  const int w = min(TX, m.nx - i0), h = min(TY, m.jn - jt0);
  const bool act = r < h && c < w;
  const int i = i0 + c, j = jt0 + r;
  constexpr bool adi = ADI;
  constexpr bool sph = GEO == FARGO_SPHERICAL, cyl = GEO == FARGO_CYLINDRICAL;
  const F dt = vreg((F)*dtp), c2 = vreg((F)(m.cvnr * m.cvnr)), om = vreg((F)m.omega), gm1 = vreg((F)(m.gamma - 1.0));
  const unsigned plane = (unsigned)m.plane();
  // geometric factors of the thread's row (the products with the plane
  // factors are those of Mesh::Sx, Sy, Sz and Vinv); rows past the tile
  // read the last active row
  const int jg = min(j, m.jn - 1);
  const double g_sxj = vreg(m.g.sxj(jg)), g_syj = vreg(m.g.syj(jg)), g_syj1 = vreg(m.g.syj(jg + 1)),
               g_szj = vreg(m.g.szj(jg)), g_invVj = vreg(m.g.invVj(jg)), g_invLy = vreg(m.g.inv_Ly(jg)),
               g_iymed = vreg(m.g.inv_ymed(jg)), g_ymed = vreg(m.g.ymed(jg));

  // storage column of X slot sl (i0 - 2 + sl, periodic) and row of Y slot t
  auto xcol = [&](int sl) {
    int x = i0 - 2 + sl;
    if (m.nx >= 2) return x < 0 ? x + m.nx : (x >= m.nx ? x - m.nx : x);
    return 0;
  };
  auto yrow = [&](int t) {
    int y = jt0 - 2 + t;
    if (m.yper()) y = y < m.j0 ? y + m.ny : (y >= m.jn ? y - m.ny : y);
    return y;
  };
  auto yowned = [&](int f) { return f >= m.ylo() && f < m.jn; };
  auto zowned = [&](int f) { return f >= m.zlo() && f < m.kn; };
  // Loads keep raw field values and derived ones are formed where they are
  // used, so that a prefetched load is not waited for when it is issued.
  auto pres = [&](F rho, F q) { return adi ? gm1 * q : q * q * rho; };
  auto loadz = [&](int k, Zv<F> &z) {
    const unsigned o = m.o32(i, j, k);
    const int ip = i + 1 == m.nx ? 0 : i + 1;
    z.rho = s.rho[o];
    z.q = adi ? s.e[o] : s.cs[o];
    z.pot = s.pot[o];
    z.vz = D3 ? s.vz[o] : F(0);
    z.vx = s.vx[o];
    z.vxp = sph ? s.vx[o - (unsigned)i + (unsigned)ip] : F(0);
  };
  // v'_z on face p between planes below(p) (zb) and p (z0); v^n if not owned.
  // iz receives 1 / ((rho + rho_below) h_z) for the viscous term.
  auto vz1 = [&](int p, const Zv<F> &zb, const Zv<F> &z0, F &iz) {
    iz = F(0);
    if (!zowned(p)) return z0.vz;
    const double ihzd = sph ? m.g.inv_dzmed(p) * g_iymed : m.g.inv_dzmed(p);
    iz = (F)ihzd / (z0.rho + zb.rho);
    F gradP = F(2) * (pres(z0.rho, z0.q) - pres(zb.rho, zb.q)) * iz;
    F gradPhi = (F)((z0.pot - zb.pot) * ihzd);
    F src = F(0);
    if constexpr (sizeof(F) == 4) {
      if (sph) {
        // an FP32 v_x is a deviation d from the ring's background: with W the
        // mean background of the two rings, vt^2 = W^2 + (2 W + d) d, and the
        // W^2 part, which the potential and pressure gradients nearly cancel,
        // is formed with the potential gradient in FP64 and rounded once
        const F W = (F)(0.5 * (m.bg(BG_VT, jg, p) + m.bg(BG_VT, jg, m.kbelow(p))));
        const F d = F(0.25) * ((z0.vx + z0.vxp) + (zb.vx + zb.vxp));
        const F base = (F)(m.bg(BG_CZ, jg, p) - (z0.pot - zb.pot) * ihzd);
        src = (F(2) * W + d) * d * (F)m.g.cotz(p) * (F)g_iymed + base;
      } else {
        src = -gradPhi;
      }
      return z0.vz - dt * gradP + dt * src;
    } else {
      if (sph) { // inertial azimuthal velocity v_x + R Omega of the two rings
        const F o0 = (F)(g_ymed * m.g.sinz(p)) * om, o1 = (F)(g_ymed * m.g.sinz(m.kbelow(p))) * om;
        F vt = F(0.25) * ((z0.vx + o0) + (z0.vxp + o0) + (zb.vx + o1) + (zb.vxp + o1));
        src = vt * vt * (F)m.g.cotz(p) * (F)g_iymed;
      }
      return z0.vz - dt * (gradP + gradPhi) + dt * src;
    }
  };
  const bool per = m.zper();
  auto pl = [&](int p) { return per ? m.k0 + (p - m.k0 + 2 * m.nz) % m.nz : p; };

  // The halo zone this thread stages, if any (fixed over the march):
  // role 1, Y halo rows 0, 1, h+2, h+3 over the tile's columns (with v_y and,
  // in spherical geometry, the summed v_theta); role 2, X halo slots 0, 1,
  // w+2, w+3 of the tile rows; role 3, v_x on the X face after the last
  // column, in the Y halo rows.
  int role = 0, ht = 0, hsl = 0;
  if (tid < 256) {
    const int q = tid >> 6;
    ht = q < 2 ? q : h + q;
    hsl = c + 2;
    role = c < w ? 1 : 0;
  } else if (tid < 256 + 4 * TY) {
    const int q = tid - 256, rr = q >> 2, a = q & 3;
    ht = rr + 2;
    hsl = a < 2 ? a : w + a;
    role = rr < h ? 2 : 0;
  } else if (tid < 256 + 4 * TY + 4) {
    const int q = tid - 256 - 4 * TY;
    ht = q < 2 ? q : h + q;
    hsl = w + 2;
    role = 3;
  }
  const unsigned hbase = role ? m.o32(xcol(hsl), yrow(ht), 0) : 0u;
  const bool hvy = role == 1 && ht != 0, hvt = role == 1 && sph;
  // what staging takes from memory besides the window: own v_y and the halo
  struct Halo {
    F vy, hr, hq, hx, hy, ht0, ht1;
    double hp;
  };
  auto load_halo = [&](int kk, Halo &n) {
    if (act) n.vy = s.vy[m.o32(i, j, kk)];
    if (role) {
      const unsigned o = hbase + (unsigned)kk * plane;
      n.hx = s.vx[o];
      if (role != 3) {
        n.hr = s.rho[o];
        n.hq = adi ? s.e[o] : s.cs[o];
        n.hp = s.pot[o];
      }
      if (hvy) n.hy = s.vy[o];
      if (hvt) {
        const int kp = D3 ? m.kabove(kk) : kk;
        n.ht0 = s.vz[o];
        n.ht1 = s.vz[o + (unsigned)(kp - kk) * plane];
      }
    }
  };
  // S: stage plane kk into buffers sb (and rb for the density); interior from
  // the window record z (vt = summed v_theta of the zone), halo from hv
  auto stage = [&](int kk, int sb, int rb, const Zv<F> &z, F vt, const Halo &hv) {
    F(*R)[SX] = L.R[rb];
    if (c == 0 && r < h) L.DX[sb][r] = m.g.inv_dxlen((size_t)kk * m.nyg + jt0 + r);
    if (act) {
      R[r + 2][c + 2] = z.rho;
      L.P[sb][r + 2][c + 2] = pres(z.rho, z.q);
      L.Ph[sb][r + 2][c + 2] = z.pot;
      L.VX[sb][r + 2][c + 2] = z.vx;
      if (sph) L.VT[sb][r + 2][c] = vt;
      L.VY[sb][r + 2][c] = hv.vy;
    }
    if (role) {
      L.VX[sb][ht][hsl] = hv.hx;
      if (role != 3) {
        R[ht][hsl] = hv.hr;
        L.P[sb][ht][hsl] = pres(hv.hr, hv.hq);
        L.Ph[sb][ht][hsl] = hv.hp;
      }
      if (hvy) L.VY[sb][ht][hsl - 2] = hv.hy;
      if (hvt) L.VT[sb][ht][hsl - 2] = hv.ht0 + hv.ht1;
    }
  };
  // F: 7a on the X and Y faces of plane kk (staged in sb, rb) into face buffer sb
  auto faces = [&](int kk, int sb, int rb) {
    F(*R)[SX] = L.R[rb];
    auto xface = [&](int rr, int sl, double idXd) {
      const int t = rr + 2;
      const F inv = (F)idXd / (R[t][sl] + R[t][sl - 1]);
      const F gradP = F(2) * (L.P[sb][t][sl] - L.P[sb][t][sl - 1]) * inv;
      const F gradPhi = (F)((L.Ph[sb][t][sl] - L.Ph[sb][t][sl - 1]) * idXd);
      L.AX[sb][rr][sl] = L.VX[sb][t][sl] - dt * (gradP + gradPhi);
      if constexpr (KI) L.IX[sb][rr][sl] = inv;
    };
    auto yface = [&](int t, int cc) {
      const int f = yrow(t), sl = cc + 2;
      if (!yowned(f)) {
        L.AY[sb][t][cc] = L.VY[sb][t][cc];
        if constexpr (KI) L.IY[sb][t][cc] = F(0);
        return;
      }
      const double ihd = m.g.inv_hy(f);
      const F inv = (F)ihd / (R[t][sl] + R[t - 1][sl]);
      const F gradP = F(2) * (L.P[sb][t][sl] - L.P[sb][t - 1][sl]) * inv;
      const F gradPhi = (F)((L.Ph[sb][t][sl] - L.Ph[sb][t - 1][sl]) * ihd);
      F src = F(0);
      if constexpr (sizeof(F) == 4) {
        // an FP32 v_x is a deviation d from the ring's background: with W the
        // mean background of the two rings, v^2 = W^2 + (2 W + d) d; the W^2
        // part, which gravity cancels to order h^2 in a disk, is formed with
        // the potential gradient in FP64 and rounded once
        if (cyl || sph) {
          const int ya = yrow(t - 1);
          const F W = (F)(0.5 * (m.bg(BG_VT, f, kk) + m.bg(BG_VT, ya, kk)));
          const F d = F(0.25) * ((L.VX[sb][t][sl] + L.VX[sb][t][sl + 1]) + (L.VX[sb][t - 1][sl] + L.VX[sb][t - 1][sl + 1]));
          src = (F(2) * W + d) * d;
          if (sph) {
            const F wv = F(0.25) * (L.VT[sb][t][cc] + L.VT[sb][t - 1][cc]);
            src += wv * wv;
          }
          src = src * (F)m.g.inv_ymin(f) +
                (F)(m.bg(BG_CY, f, kk) - (L.Ph[sb][t][sl] - L.Ph[sb][t - 1][sl]) * ihd);
        } else {
          src = -gradPhi;
        }
        L.AY[sb][t][cc] = L.VY[sb][t][cc] - dt * gradP + dt * src;
      } else {
        if (cyl || sph) {
          const int ya = yrow(t - 1);
          const F ot = (F)(sph ? m.g.ymed(f) * m.g.sinz(kk) : m.g.ymed(f)) * om;
          const F oa = (F)(sph ? m.g.ymed(ya) * m.g.sinz(kk) : m.g.ymed(ya)) * om;
          const F vt0 = (L.VX[sb][t][sl] + ot) + (L.VX[sb][t][sl + 1] + ot);
          const F vt1 = (L.VX[sb][t - 1][sl] + oa) + (L.VX[sb][t - 1][sl + 1] + oa);
          const F v = F(0.25) * (vt0 + vt1);
          src = v * v;
          if (sph) {
            const F wv = F(0.25) * (L.VT[sb][t][cc] + L.VT[sb][t - 1][cc]);
            src += wv * wv;
          }
          src *= (F)m.g.inv_ymin(f);
        }
        L.AY[sb][t][cc] = L.VY[sb][t][cc] - dt * (gradP + gradPhi) + dt * src;
      }
      if constexpr (KI) L.IY[sb][t][cc] = inv;
    };
    if (act) {
      xface(r, c + 2, m.g.inv_dxlen((size_t)kk * m.nyg + jt0 + r));
      yface(r + 2, c);
    }
    // the halo faces: the last three waves take the extra Y-face rows and
    // wave 4 the extra X faces, since waves 0-3 stage the Y-halo rows (the
    // barrier waits for the most loaded wave)
    if (r >= TY - 3) {
      const int e = r - (TY - 3), t = e == 0 ? 1 : h + 1 + e;
      if (c < w) yface(t, c);
    } else if (r == 4 && c < 3 * TY) {
      const int rr = c / 3, a = c % 3, sl = a == 0 ? 1 : w + 1 + a;
      if (rr < h) xface(rr, sl, L.DX[sb][rr]);
    }
  };
  // Z: 7b and 7c for the zones of plane kk (faces in sb, density in rb); zd
  // gives the Z part: bz1/bz2 (v'' of faces kk and above(kk)), qz and dvz
  struct ZPart {
    F bz1, bz2, qz, dvz;
  };
  auto zones = [&](int kk, int sb, int rb, const ZPart &zp, F e_old) {
    F(*R)[SX] = L.R[rb];
    const int t = r + 2, sl = c + 2;
    const unsigned o = m.o32(i, j, kk);
    // X: faces sl-1 .. sl+2, zones sl-1 .. sl+1
    const F a0 = L.AX[sb][r][sl - 1], a1 = L.AX[sb][r][sl], a2 = L.AX[sb][r][sl + 1], a3 = L.AX[sb][r][sl + 2];
    const F r1 = R[t][sl - 1], r2 = R[t][sl], r3 = R[t][sl + 1];
    const F dvx = a2 - a1;
    const F qx = qvisc(c2, r2, dvx), qxm = qvisc(c2, r1, a1 - a0), qxp = qvisc(c2, r3, a3 - a2);
    const double idX = m.g.inv_dxlen((size_t)kk * m.nyg + j);
    // the reciprocals of the two X faces, as the faces' pass forms them
    const F ix1 = KI ? L.IX[sb][r][sl] : (F)idX / (r2 + r1);
    const F ix2 = KI ? L.IX[sb][r][sl + 1] : (F)idX / (r3 + r2);
    const F bx1 = a1 - dt * F(2) * (qx - qxm) * ix1;
    const F bx2 = a2 - dt * F(2) * (qxp - qx) * ix2;
    vx2[o] = bx1;
    F heat = qx * dvx * (F)idX;
    const double syk = m.g.syk(kk);
    F flux = (F)(g_sxj * m.g.sxk(kk)) * (bx2 - bx1);
    // Y: faces t-1 .. t+2, zones t-1 .. t+1
    const F b0 = L.AY[sb][t - 1][c], b1 = L.AY[sb][t][c], b2 = L.AY[sb][t + 1][c], b3 = L.AY[sb][t + 2][c];
    const F s1 = R[t - 1][sl], s3 = R[t + 1][sl];
    const F dvy = b2 - b1;
    const F qy = qvisc(c2, r2, dvy);
    F by1 = b1, by2 = b2;
    if (yowned(j)) {
      const F iy = KI ? L.IY[sb][t][c] : (F)m.g.inv_hy(j) / (r2 + s1);
      by1 = b1 - dt * F(2) * (qy - qvisc(c2, s1, b1 - b0)) * iy;
    }
    const int ju = yrow(t + 1);
    if (yowned(ju)) {
      const F iy = KI ? L.IY[sb][t + 1][c] : (F)m.g.inv_hy(ju) / (s3 + r2);
      by2 = b2 - dt * F(2) * (qvisc(c2, s3, b3 - b2) - qy) * iy;
    }
    vy2[o] = by1;
    heat += qy * dvy * (F)g_invLy;
    flux += (F)(g_syj1 * syk) * by2 - (F)(g_syj * syk) * by1;
    if (D3) {
      vz2[o] = zp.bz1;
      const F iLz = sph ? (F)(m.g.inv_dz(kk) * g_iymed) : (F)m.g.inv_dz(kk);
      heat += zp.qz * zp.dvz * iLz;
      flux += (F)(g_szj * m.g.szk(kk + 1)) * zp.bz2 - (F)(g_szj * m.g.szk(kk)) * zp.bz1;
    }
    if (adi) {
      const F e1 = e_old - dt * heat;
      const F a = F(0.5) * dt * gm1 * ((F)(g_invVj / syk) * flux);
      e2[o] = e1 * (F(1) - a) / (F(1) + a);
    }
  };

  if constexpr (!D3) {
    // a single plane: S, F, Z in turn
    Zv<F> z0{};
    Halo hv{};
    F e_old = F(0);
    if (act) {
      loadz(0, z0);
      e_old = z0.q;
    }
    load_halo(0, hv);
    stage(0, 0, 0, z0, F(0), hv);
    __syncthreads();
    faces(0, 0, 0);
    __syncthreads();
    if (act) zones(0, 0, 0, ZPart{}, e_old);
  } else {
  // ---- 3D march over the active planes k0 .. kn-1
  const int k0 = m.k0, kn = m.kn;
  // Z window of the thread's column at the top of interval kk:
  //   Z1, Z2 = records of planes kk+1, kk+2; vzk = v_z of plane kk;
  //   A[0..2] = v'_z of faces kk .. kk+2, IZ likewise; Q[0..2] = q_z of
  //   zones kk-1 .. kk+1
  Zv<F> Z1{}, Z2{}, Zn{};
  F vzk = F(0), A[3] = {}, IZ[3] = {}, Q[3] = {}, e_cur = F(0);
  Halo hv{}, hn{};
  if (act) {
    Zv<F> a, b, z0;
    F Am1, IZm1, A0, IZ0, A1, IZ1, A2, IZ2;
    loadz(pl(k0 - 2), a);
    loadz(pl(k0 - 1), b);
    loadz(k0, z0);
    loadz(pl(k0 + 1), Z1);
    loadz(pl(k0 + 2), Z2);
    Am1 = vz1(pl(k0 - 1), a, b, IZm1);
    A0 = vz1(k0, b, z0, IZ0);
    A1 = vz1(pl(k0 + 1), z0, Z1, IZ1);
    A2 = vz1(pl(k0 + 2), Z1, Z2, IZ2);
    (void)IZm1;
    A[0] = A0;
    A[1] = A1;
    A[2] = A2;
    IZ[0] = IZ0;
    IZ[1] = IZ1;
    IZ[2] = IZ2;
    Q[0] = qvisc(c2, b.rho, A0 - Am1);
    Q[1] = qvisc(c2, z0.rho, A1 - A0);
    Q[2] = qvisc(c2, Z1.rho, A2 - A1);
    vzk = z0.vz;
    e_cur = z0.q;
    // prologue: S(k0), then F(k0) with S(k0+1)
    load_halo(k0, hv);
    stage(k0, 0, 0, z0, z0.vz + Z1.vz, hv);
  } else {
    load_halo(k0, hv);
    stage(k0, 0, 0, Zv<F>{}, F(0), hv);
  }
  __syncthreads();
  faces(k0, 0, 0);
  load_halo(pl(k0 + 1), hv);
  stage(k0 + 1, 1, 1, Z1, Z1.vz + Z2.vz, hv);
  // prefetch for interval k0: record of plane k0+3, halo of plane k0+2
  if (act) loadz(pl(k0 + 3), Zn);
  if (k0 + 2 < kn) load_halo(k0 + 2, hn);
  __syncthreads();

  int sb = 0, rb = 0; // buffers of plane kk
#pragma unroll 1
  for (int kk = k0; kk < kn; kk++) {
    const int sb1 = sb ^ 1, rb1 = rb == 2 ? 0 : rb + 1, rb2 = rb1 == 2 ? 0 : rb1 + 1;
    // Z(kk)
    if (act) {
      ZPart zp;
      const int ka = pl(kk + 1);
      zp.bz1 = zowned(kk) ? A[0] - dt * F(2) * (Q[1] - Q[0]) * IZ[0] : vzk;
      zp.bz2 = zowned(ka) ? A[1] - dt * F(2) * (Q[2] - Q[1]) * IZ[1] : Z1.vz;
      zp.qz = Q[1];
      zp.dvz = A[1] - A[0];
      zones(kk, sb, rb, zp, e_cur);
    }
    // F(kk+1), S(kk+2)
    if (kk + 1 < kn) faces(kk + 1, sb1, rb1);
    if (kk + 2 < kn) stage(kk + 2, sb, rb2, Z2, Z2.vz + Zn.vz, hn);
    // advance the window and prefetch for interval kk+1
    if (kk + 1 < kn) {
      if (act) {
        F A3, IZ3;
        A3 = vz1(pl(kk + 3), Z2, Zn, IZ3);
        const F Q3 = qvisc(c2, Z2.rho, A3 - A[2]);
        vzk = Z1.vz;
        e_cur = Z1.q;
        Z1 = Z2;
        Z2.rho = vmove(Zn.rho);
        Z2.q = vmove(Zn.q);
        Z2.pot = vmove(Zn.pot);
        Z2.vz = vmove(Zn.vz);
        Z2.vx = vmove(Zn.vx);
        Z2.vxp = sph ? vmove(Zn.vxp) : F(0);
        A[0] = A[1];
        A[1] = A[2];
        A[2] = A3;
        IZ[0] = IZ[1];
        IZ[1] = IZ[2];
        IZ[2] = IZ3;
        Q[0] = Q[1];
        Q[1] = Q[2];
        Q[2] = Q3;
        // unconditional (plane kk+4 <= kn+2 is at worst a ghost plane), so
        // that the load writes the window register itself
        loadz(pl(kk + 4), Zn);
      }
      if (kk + 3 < kn) load_halo(kk + 3, hn);
    }
    __syncthreads();
    sb = sb1;
    rb = rb1;
  }
  }
}
template <typename F, bool D3, int GEO, bool ADI>
__global__ __launch_bounds__((src_threads<F, D3, GEO, ADI>()), (src_waves<F, D3, GEO, ADI>())) void k_source(
    Mesh m, StateT<F> s, const double *__restrict__ dtp, F *__restrict__ vx2, F *__restrict__ vy2,
    F *__restrict__ vz2, F *__restrict__ e2, int nbx, int nby) {
  source_body<F, D3, GEO, ADI>(m, s, dtp, vx2, vy2, vz2, e2, nbx, nby, blockIdx.x, gridDim.x);
}

// Ghost zones (Y ghost rows of every plane, and Z ghost planes of the active
// rows) carry v^n and e into v'' and e''; one block per row.
template <typename F>
__device__ __forceinline__ void source_ghosts_body(Mesh m, StateT<F> s, F *__restrict__ vx2,
                                                       F *__restrict__ vy2, F *__restrict__ vz2,
                                                       F *__restrict__ e2, unsigned bid_, unsigned nbk_) {
  const int b = bid_, ngy = m.nyg - m.ny;
  int j, k;
  if (b < m.nzg * ngy) {
    k = b / ngy;
    const int g = b % ngy;
    j = g < m.j0 ? g : m.jn + (g - m.j0);
  } else {
    const int q = b - m.nzg * ngy, ngz = m.nzg - m.nz;
    j = m.j0 + q % m.ny;
    const int g = q / m.ny;
    k = g < m.k0 ? g : m.kn + (g - m.k0);
    (void)ngz;
  }
  const unsigned row = m.o32(0, j, k);
  for (int i = threadIdx.x; i < m.nx; i += blockDim.x) {
    const unsigned o = row + (unsigned)i;
    vx2[o] = s.vx[o];
    vy2[o] = s.vy[o];
    if (m.d3) vz2[o] = s.vz[o];
    if (m.eos == FARGO_ADIABATIC) e2[o] = s.e[o];
  }
}
template <typename F>
__global__ __launch_bounds__(256) void k_source_ghosts(Mesh m, StateT<F> s, F *__restrict__ vx2,
                                                       F *__restrict__ vy2, F *__restrict__ vz2,
                                                       F *__restrict__ e2) {
  source_ghosts_body<F>(m, s, vx2, vy2, vz2, e2, blockIdx.x, gridDim.x);
}

// multi-mesh forms (ManyGrid)
template <typename F>
struct SourceArgs {
  Mesh m;
  StateT<F> s;
  const double *dt;
  F *vx2, *vy2, *vz2, *e2;
  int nbx, nby;
  unsigned nb;
};
template <typename F, bool D3, int GEO, bool ADI>
__global__ __launch_bounds__((src_threads<F, D3, GEO, ADI>()), (src_waves<F, D3, GEO, ADI>())) void k_source_many(
    const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const SourceArgs<F> a = many_args<SourceArgs<F>>(args, t.x);
  source_body<F, D3, GEO, ADI>(a.m, a.s, a.dt, a.vx2, a.vy2, a.vz2, a.e2, a.nbx, a.nby, t.y, a.nb);
}
template <typename F>
__global__ __launch_bounds__(256) void k_source_ghosts_many(const void *args, const uint2 *tab) {
  const uint2 t = many_block(tab);
  if (t.x == MANY_NONE) return;
  const SourceArgs<F> a = many_args<SourceArgs<F>>(args, t.x);
  source_ghosts_body<F>(a.m, a.s, a.vx2, a.vy2, a.vz2, a.e2, t.y, a.nb);
}

// tile rows of the source step's launch on mesh m
template <typename F>
int src_rows(const Mesh &m) {
  if (!m.d3) return tile_rows<F, false, FARGO_CARTESIAN, false>();
  const bool tall = m.geo != FARGO_SPHERICAL && m.eos != FARGO_ADIABATIC;
  return tall ? tile_rows<F, true, FARGO_CARTESIAN, false>() : tile_rows<F, true, FARGO_SPHERICAL, true>();
}

} // namespace

template <typename F>
void launch_source(Launch &L, const Mesh &m, const StateT<F> &s, const double *dt, F *vx2, F *vy2, F *vz2, F *e2) {
  const int nbx = (m.nx + TX - 1) / TX, nby = (m.ny + src_rows<F>(m) - 1) / src_rows<F>(m);
  const unsigned nb = (unsigned)nbx * (unsigned)nby;
  const unsigned ng = (unsigned)(m.nzg * (m.nyg - m.ny) + (m.d3 ? (m.nzg - m.nz) * m.ny : 0));
  prof_begin(L, K_SRC);
  auto go = [&](auto d3, auto geo, auto adi) {
    constexpr bool D3 = decltype(d3)::value, ADI = decltype(adi)::value;
    constexpr int GEO = decltype(geo)::value;
    k_source<F, D3, GEO, ADI><<<nb, src_threads<F, D3, GEO, ADI>(), 0, L.s>>>(m, s, dt, vx2, vy2, vz2, e2, nbx, nby);
  };
  auto by_eos = [&](auto d3, auto geo) {
    if (m.eos == FARGO_ADIABATIC) go(d3, geo, std::true_type{});
    else go(d3, geo, std::false_type{});
  };
  auto by_geo = [&](auto d3) {
    if (m.geo == FARGO_SPHERICAL) by_eos(d3, std::integral_constant<int, FARGO_SPHERICAL>{});
    else if (m.geo == FARGO_CYLINDRICAL) by_eos(d3, std::integral_constant<int, FARGO_CYLINDRICAL>{});
    else by_eos(d3, std::integral_constant<int, FARGO_CARTESIAN>{});
  };
  if (m.d3) by_geo(std::true_type{});
  else by_geo(std::false_type{});
  prof_end(L, K_SRC);
  prof_begin(L, K_SRC_GHOSTS);
  k_source_ghosts<F><<<ng, 256, 0, L.s>>>(m, s, vx2, vy2, vz2, e2);
  prof_end(L, K_SRC_GHOSTS);
}

template void launch_source<double>(Launch &, const Mesh &, const StateT<double> &, const double *, double *, double *,
                                    double *, double *);
template void launch_source<float>(Launch &, const Mesh &, const StateT<float> &, const double *, float *, float *,
                                   float *, float *);

template <typename F>
size_t source_args_bytes() { return sizeof(SourceArgs<F>); }

template <typename F>
unsigned source_args(const Mesh &m, const StateT<F> &s, const double *dt, F *vx2, F *vy2, F *vz2, F *e2, void *dst) {
  const int nbx = (m.nx + TX - 1) / TX, nby = (m.ny + src_rows<F>(m) - 1) / src_rows<F>(m);
  const unsigned nb = (unsigned)nbx * (unsigned)nby;
  *(SourceArgs<F> *)dst = SourceArgs<F>{m, s, dt, vx2, vy2, vz2, e2, nbx, nby, nb};
  return nb;
}

template <typename F>
unsigned source_ghosts_args(const Mesh &m, const StateT<F> &s, F *vx2, F *vy2, F *vz2, F *e2, void *dst) {
  const unsigned ng = (unsigned)(m.nzg * (m.nyg - m.ny) + (m.d3 ? (m.nzg - m.nz) * m.ny : 0));
  *(SourceArgs<F> *)dst = SourceArgs<F>{m, s, nullptr, vx2, vy2, vz2, e2, 0, 0, ng};
  return ng;
}

// 2D meshes of one geometry and equation of state (those of m0)
template <typename F>
void launch_source_many(Launch &L, const Mesh &m0, const ManyGrid &g, const ManyGrid &ghosts) {
  prof_begin(L, K_SRC);
  auto go = [&](auto geo, auto adi) {
    k_source_many<F, false, decltype(geo)::value, decltype(adi)::value><<<g.nblk, src_threads<F, false, decltype(geo)::value, decltype(adi)::value>(), 0, L.s>>>(g.args, g.tab);
  };
  auto by_eos = [&](auto geo) {
    if (m0.eos == FARGO_ADIABATIC) go(geo, std::true_type{});
    else go(geo, std::false_type{});
  };
  if (m0.geo == FARGO_SPHERICAL) by_eos(std::integral_constant<int, FARGO_SPHERICAL>{});
  else if (m0.geo == FARGO_CYLINDRICAL) by_eos(std::integral_constant<int, FARGO_CYLINDRICAL>{});
  else by_eos(std::integral_constant<int, FARGO_CARTESIAN>{});
  prof_end(L, K_SRC);
  prof_begin(L, K_SRC_GHOSTS);
  k_source_ghosts_many<F><<<ghosts.nblk, 256, 0, L.s>>>(ghosts.args, ghosts.tab);
  prof_end(L, K_SRC_GHOSTS);
}

#define FARGO_SOURCE_MANY(F)                                                                                        \
  template size_t source_args_bytes<F>();                                                                          \
  template unsigned source_args<F>(const Mesh &, const StateT<F> &, const double *, F *, F *, F *, F *, void *);   \
  template unsigned source_ghosts_args<F>(const Mesh &, const StateT<F> &, F *, F *, F *, F *, void *);            \
  template void launch_source_many<F>(Launch &, const Mesh &, const ManyGrid &, const ManyGrid &);
FARGO_SOURCE_MANY(double)
FARGO_SOURCE_MANY(float)
#undef FARGO_SOURCE_MANY

} // namespace fargo
