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
// kept in LDS with the reciprocal of its density sum, then each zone forms q
// on its neighbours and its v'' and e''.  Along Z each thread keeps a sliding
// window of its own column in registers (planes k-1 .. k+2), which also
// supplies the tile's interior values to LDS, so each interior value is read
// from memory once.  Geometric lengths enter through reciprocal tables.
//
// The field type F is double, or float for the FP32-bulk state; arithmetic is
// carried out in F, geometric factors are rounded to F where they are used.
#include "fargo_internal.h"

namespace fargo {

namespace {

constexpr int TX = 64, TY = 8;          // tile; one wave per tile row
constexpr int SX = TX + 4, SY = TY + 4; // with two halo zones on each side
constexpr int NT = TX * TY;

template <typename F>
__device__ inline F qvisc(F c2, F rho, F dv) { return dv < F(0) ? c2 * rho * dv * dv : F(0); }

template <typename F>
struct Lds {
  F R[2][SY][SX];  // density (two planes in flight)
  F P[SY][SX];     // pressure
  double Ph[SY][SX]; // potential (FP64 in every mode)
  F VX[SY][SX];    // v_x on the lower X face of each zone slot
  F VY[SY][TX];    // v_y on the lower Y face of each zone slot
  F VT[SY][TX];    // spherical: v_theta on the zone's two Z faces, summed
  F AX[TY][SX];    // v'_x of X faces of the tile rows
  F IX[TY][SX];    // 1 / ((rho_i + rho_{i-1}) dX) on those faces
  F AY[SY][TX];    // v'_y of Y faces
  F IY[SY][TX];    // 1 / ((rho_j + rho_{j-1}) h_y) on those faces
};

// one zone's values in one plane
template <typename F>
struct Zv {
  F rho, P;
  double pot;
  F vz, vx, vxp; // vxp: v_x on the next X face
};

template <typename F, bool D3>
__global__ __launch_bounds__(NT, sizeof(F) == 8 ? 2 : 4) void k_source(Mesh m, StateT<F> s, const double *__restrict__ dtp,
                                                  F *__restrict__ vx2, F *__restrict__ vy2, F *__restrict__ vz2,
                                                  F *__restrict__ e2, int nbx, int nby) {
  __shared__ Lds<F> L;
  const int tid = threadIdx.x, r = tid >> 6, c = tid & 63;
  const unsigned Lb = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = (int)(Lb % (unsigned)nby), tx = (int)(Lb / (unsigned)nby);
  const int i0 = tx * TX, jt0 = m.j0 + ty * TY;
  const int w = min(TX, m.nx - i0), h = min(TY, m.jn - jt0);
  const bool act = r < h && c < w;
  const int i = i0 + c, j = jt0 + r;
  const bool adi = m.eos == FARGO_ADIABATIC;
  const bool sph = m.geo == FARGO_SPHERICAL, cyl = m.geo == FARGO_CYLINDRICAL;
  const F dt = (F)*dtp, c2 = (F)(m.cvnr * m.cvnr), om = (F)m.omega, gm1 = (F)(m.gamma - 1.0);
  const unsigned plane = (unsigned)m.plane();

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
  auto pres = [&](unsigned o) { return adi ? gm1 * s.e[o] : s.cs[o] * s.cs[o] * s.rho[o]; };
  auto loadz = [&](int k, Zv<F> &z) {
    const unsigned o = m.o32(i, j, k);
    const int ip = i + 1 == m.nx ? 0 : i + 1;
    z.rho = s.rho[o];
    z.P = pres(o);
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
    const F ihz = sph ? (F)(m.g.inv_dzmed[p] * m.g.inv_ymed[j]) : (F)m.g.inv_dzmed[p];
    iz = ihz / (z0.rho + zb.rho);
    F gradP = F(2) * (z0.P - zb.P) * iz;
    F gradPhi = (F)((z0.pot - zb.pot) * (sph ? m.g.inv_dzmed[p] * m.g.inv_ymed[j] : m.g.inv_dzmed[p]));
    F src = F(0);
    if (sph) {
      F R0 = (F)(m.g.ymed[j] * m.g.sinz[p]), R1 = (F)(m.g.ymed[j] * m.g.sinz[m.kbelow(p)]);
      F vt = F(0.25) * ((z0.vx + R0 * om) + (z0.vxp + R0 * om) + (zb.vx + R1 * om) + (zb.vxp + R1 * om));
      src = vt * vt * (F)m.g.cotz[p] * (F)m.g.inv_ymed[j];
    }
    return z0.vz - dt * (gradP + gradPhi) + dt * src;
  };
  const bool per = m.zper();
  auto pl = [&](int p) { return per ? m.k0 + (p - m.k0 + 2 * m.nz) % m.nz : p; };

  // Z window of the thread's column: planes k-1 (rho only), k, k+1, k+2
  Zv<F> Z0{}, Z1{}, Z2{};
  F Rm1 = F(0), A[4] = {}, IZ[4] = {}, Q[3] = {};
  const int kfirst = m.k0, klast = m.kn;
  if (act) {
    if (D3) {
      Zv<F> Zm2, Zm1;
      loadz(pl(kfirst - 2), Zm2);
      loadz(pl(kfirst - 1), Zm1);
      A[0] = vz1(pl(kfirst - 1), Zm2, Zm1, IZ[0]);
      Rm1 = Zm1.rho;
      loadz(kfirst, Z0);
      A[1] = vz1(kfirst, Zm1, Z0, IZ[1]);
      loadz(pl(kfirst + 1), Z1);
      A[2] = vz1(pl(kfirst + 1), Z0, Z1, IZ[2]);
      Q[0] = qvisc(c2, Rm1, A[1] - A[0]);
      Q[1] = qvisc(c2, Z0.rho, A[2] - A[1]);
    } else {
      loadz(0, Z0);
    }
  }

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
  // The values an iteration stages (own v_y, the window's next plane and the
  // halo zone) are loaded one iteration ahead, so that their latency overlaps
  // the previous plane's work.  FP64 fields need more registers than two
  // workgroups per CU leave, so that kernel runs one workgroup per CU.
  constexpr bool PF = true;
  struct Pre {
    Zv<F> z;     // window plane kk + 2
    F vy;        // own v_y at plane kk
    F hr, hP, hx, hy, ht;
    double hp;   // halo: rho, P, v_x, v_y, summed v_theta, potential
  };
  auto fetch_window = [&](int kk, Pre &n) {
    if (act && D3) loadz(pl(kk + 2), n.z);
  };
  auto fetch_stage = [&](int kk, Pre &n) {
    if (act) n.vy = s.vy[m.o32(i, j, kk)];
    if (role) {
      const unsigned o = hbase + (unsigned)kk * plane;
      n.hx = s.vx[o];
      if (role != 3) {
        n.hr = s.rho[o];
        n.hP = pres(o);
        n.hp = s.pot[o];
      }
      if (hvy) n.hy = s.vy[o];
      if (hvt) {
        const int kp = D3 ? m.kabove(kk) : kk;
        n.ht = s.vz[o] + s.vz[o + (unsigned)(kp - kk) * plane];
      }
    }
  };
  auto prefetch = [&](int kk, Pre &n) {
    fetch_window(kk, n);
    fetch_stage(kk, n);
  };
  Pre nx{};
  if (PF) prefetch(kfirst, nx);

  int buf = 0;
#pragma unroll 1
  for (int kk = kfirst; kk < klast; kk++) {
    const int ka = D3 ? pl(kk + 1) : kk;
    Pre cur;
    if (PF) {
      cur = nx;
      if (kk + 1 < klast) prefetch(kk + 1, nx);
    } else {
      fetch_window(kk, cur);
    }
    if (D3 && act) {
      Z2 = cur.z;
      A[3] = vz1(pl(kk + 2), Z1, Z2, IZ[3]);
      Q[2] = qvisc(c2, Z1.rho, A[3] - A[2]);
    }
    F(*R)[SX] = L.R[buf];
    if (!PF) fetch_stage(kk, cur);
    // ---- stage plane kk: interior from the window, halo from the prefetched values
    if (act) {
      R[r + 2][c + 2] = Z0.rho;
      L.P[r + 2][c + 2] = Z0.P;
      L.Ph[r + 2][c + 2] = Z0.pot;
      L.VX[r + 2][c + 2] = Z0.vx;
      if (sph) L.VT[r + 2][c] = Z0.vz + Z1.vz;
      L.VY[r + 2][c] = cur.vy;
    }
    if (role) {
      L.VX[ht][hsl] = cur.hx;
      if (role != 3) {
        R[ht][hsl] = cur.hr;
        L.P[ht][hsl] = cur.hP;
        L.Ph[ht][hsl] = cur.hp;
      }
      if (hvy) L.VY[ht][hsl - 2] = cur.hy;
      if (hvt) L.VT[ht][hsl - 2] = cur.ht;
    }
    __syncthreads();
    // ---- 7a on the X and Y faces of the tile and of the halo faces needed
    auto xface = [&](int rr, int sl) {
      const int t = rr + 2, y = jt0 + rr;
      const double idXd = m.g.inv_dxlen[(size_t)kk * m.nyg + y];
      const F inv = (F)idXd / (R[t][sl] + R[t][sl - 1]);
      const F gradP = F(2) * (L.P[t][sl] - L.P[t][sl - 1]) * inv;
      const F gradPhi = (F)((L.Ph[t][sl] - L.Ph[t][sl - 1]) * idXd);
      L.AX[rr][sl] = L.VX[t][sl] - dt * (gradP + gradPhi);
      L.IX[rr][sl] = inv;
    };
    auto yface = [&](int t, int cc) {
      const int f = yrow(t), sl = cc + 2;
      if (!yowned(f)) {
        L.AY[t][cc] = L.VY[t][cc];
        L.IY[t][cc] = F(0);
        return;
      }
      const double ihd = m.g.inv_hy[f];
      const F inv = (F)ihd / (R[t][sl] + R[t - 1][sl]);
      const F gradP = F(2) * (L.P[t][sl] - L.P[t - 1][sl]) * inv;
      const F gradPhi = (F)((L.Ph[t][sl] - L.Ph[t - 1][sl]) * ihd);
      F src = F(0);
      if (cyl || sph) {
        const int ya = yrow(t - 1);
        const F Rt = (F)(sph ? m.g.ymed[f] * m.g.sinz[kk] : m.g.ymed[f]);
        const F Ra = (F)(sph ? m.g.ymed[ya] * m.g.sinz[kk] : m.g.ymed[ya]);
        const F vt0 = (L.VX[t][sl] + Rt * om) + (L.VX[t][sl + 1] + Rt * om);
        const F vt1 = (L.VX[t - 1][sl] + Ra * om) + (L.VX[t - 1][sl + 1] + Ra * om);
        const F v = F(0.25) * (vt0 + vt1);
        src = v * v;
        if (sph) {
          const F wv = F(0.25) * (L.VT[t][cc] + L.VT[t - 1][cc]);
          src += wv * wv;
        }
        src *= (F)m.g.inv_ymin[f];
      }
      L.AY[t][cc] = L.VY[t][cc] - dt * (gradP + gradPhi) + dt * src;
      L.IY[t][cc] = inv;
    };
    if (act) {
      xface(r, c + 2);
      yface(r + 2, c);
    }
    if (tid < 192) {
      const int q = tid >> 6, t = q == 0 ? 1 : h + 1 + q;
      if (c < w) yface(t, c);
    } else if (tid < 192 + 3 * TY) {
      const int q = tid - 192, rr = q / 3, a = q % 3, sl = a == 0 ? 1 : w + 1 + a;
      if (rr < h) xface(rr, sl);
    }
    __syncthreads();
    // ---- 7b and 7c per zone
    if (act) {
      const int t = r + 2, sl = c + 2;
      const unsigned o = m.o32(i, j, kk);
      // X: faces sl-1 .. sl+2, zones sl-1 .. sl+1
      const F a0 = L.AX[r][sl - 1], a1 = L.AX[r][sl], a2 = L.AX[r][sl + 1], a3 = L.AX[r][sl + 2];
      const F r1 = R[t][sl - 1], r2 = R[t][sl], r3 = R[t][sl + 1];
      const F dvx = a2 - a1;
      const F qx = qvisc(c2, r2, dvx), qxm = qvisc(c2, r1, a1 - a0), qxp = qvisc(c2, r3, a3 - a2);
      const F bx1 = a1 - dt * F(2) * (qx - qxm) * L.IX[r][sl];
      const F bx2 = a2 - dt * F(2) * (qxp - qx) * L.IX[r][sl + 1];
      vx2[o] = bx1;
      F heat = qx * dvx * (F)m.g.inv_dxlen[(size_t)kk * m.nyg + j];
      F flux = (F)m.Sx(j, kk) * (bx2 - bx1);
      // Y: faces t-1 .. t+2, zones t-1 .. t+1
      const F b0 = L.AY[t - 1][c], b1 = L.AY[t][c], b2 = L.AY[t + 1][c], b3 = L.AY[t + 2][c];
      const F s1 = R[t - 1][sl], s3 = R[t + 1][sl];
      const F dvy = b2 - b1;
      const F qy = qvisc(c2, r2, dvy);
      F by1 = b1, by2 = b2;
      if (yowned(j)) by1 = b1 - dt * F(2) * (qy - qvisc(c2, s1, b1 - b0)) * L.IY[t][c];
      if (yowned(yrow(t + 1))) by2 = b2 - dt * F(2) * (qvisc(c2, s3, b3 - b2) - qy) * L.IY[t + 1][c];
      vy2[o] = by1;
      heat += qy * dvy * (F)m.g.inv_Ly[j];
      flux += (F)m.Sy(j + 1, kk) * by2 - (F)m.Sy(j, kk) * by1;
      if (D3) {
        F bz1 = Z0.vz, bz2 = Z1.vz;
        if (zowned(kk)) bz1 = A[1] - dt * F(2) * (Q[1] - Q[0]) * IZ[1];
        if (zowned(ka)) bz2 = A[2] - dt * F(2) * (Q[2] - Q[1]) * IZ[2];
        vz2[o] = bz1;
        const F iLz = sph ? (F)(m.g.inv_dz[kk] * m.g.inv_ymed[j]) : (F)m.g.inv_dz[kk];
        heat += Q[1] * (A[2] - A[1]) * iLz;
        flux += (F)m.Sz(j, kk + 1) * bz2 - (F)m.Sz(j, kk) * bz1;
      }
      if (adi) {
        const F e1 = s.e[o] - dt * heat;
        const F a = F(0.5) * dt * gm1 * ((F)m.Vinv(j, kk) * flux);
        e2[o] = e1 * (F(1) - a) / (F(1) + a);
      }
      if (D3) {
        Rm1 = Z0.rho;
        Z0 = Z1;
        Z1 = Z2;
        A[0] = A[1];
        A[1] = A[2];
        A[2] = A[3];
        IZ[0] = IZ[1];
        IZ[1] = IZ[2];
        IZ[2] = IZ[3];
        Q[0] = Q[1];
        Q[1] = Q[2];
      }
    }
    (void)Rm1;
    buf ^= 1;
  }
}

// Ghost zones (Y ghost rows of every plane, and Z ghost planes of the active
// rows) carry v^n and e into v'' and e''; one block per row.
template <typename F>
__global__ __launch_bounds__(256) void k_source_ghosts(Mesh m, StateT<F> s, F *__restrict__ vx2,
                                                       F *__restrict__ vy2, F *__restrict__ vz2,
                                                       F *__restrict__ e2) {
  const int b = blockIdx.x, ngy = m.nyg - m.ny;
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

} // namespace

template <typename F>
void launch_source(Launch &L, const Mesh &m, const StateT<F> &s, const double *dt, F *vx2, F *vy2, F *vz2, F *e2) {
  const int nbx = (m.nx + TX - 1) / TX, nby = (m.ny + TY - 1) / TY;
  const unsigned nb = (unsigned)nbx * (unsigned)nby;
  const unsigned ng = (unsigned)(m.nzg * (m.nyg - m.ny) + (m.d3 ? (m.nzg - m.nz) * m.ny : 0));
  prof_begin(L, K_SRC);
  if (m.d3) k_source<F, true><<<nb, NT, 0, L.s>>>(m, s, dt, vx2, vy2, vz2, e2, nbx, nby);
  else k_source<F, false><<<nb, NT, 0, L.s>>>(m, s, dt, vx2, vy2, vz2, e2, nbx, nby);
  prof_end(L, K_SRC);
  prof_begin(L, K_SRC_GHOSTS);
  k_source_ghosts<F><<<ng, 256, 0, L.s>>>(m, s, vx2, vy2, vz2, e2);
  prof_end(L, K_SRC_GHOSTS);
}

template void launch_source<double>(Launch &, const Mesh &, const StateT<double> &, const double *, double *, double *,
                                    double *, double *);
template void launch_source<float>(Launch &, const Mesh &, const StateT<float> &, const double *, float *, float *,
                                   float *, float *);

} // namespace fargo
