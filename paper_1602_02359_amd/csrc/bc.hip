// Boxes 2 and 9: boundary conditions in the three ghost layers of Y and Z
// (Sect. 4.1).  X is periodic through index arithmetic and has no ghosts.
//
// Per side: PERIODIC copies the opposite edge; REFLECT mirrors zone-centred
// fields and tangential velocities, makes the normal velocity antisymmetric
// and sets the boundary face to zero; OUTFLOW copies the edge zone and the
// first interior face; FIXED writes nothing.  Boundary faces are set by one
// launch and ghosts by a second one, so that ghost faces mirror final values;
// the Y sides are filled over every Z row before the Z sides over every Y
// column (corners consistent).  An FP32 v_x (a deviation from its ring's
// background) is copied with the difference of the two rings' backgrounds.
#include "fargo_internal.h"

namespace fargo {

namespace {

template <typename R>
struct Cen {
  R *p[4];
  int n;
  int ivx; // index of v_x in p (-1 if absent)
};

__device__ inline size_t at(const Mesh &m, int dir, int i, int a, int b) {
  return dir == 1 ? m.idx(i, a, b) : m.idx(i, b, a);
}

template <typename R>
__global__ __launch_bounds__(256) void k_bc_faces(Mesh m, int dir, int side, int kind, R *vn) {
  int lo = dir == 1 ? m.j0 : m.k0, hi = dir == 1 ? m.jn : m.kn;
  int nb = dir == 1 ? m.nzg : m.nyg;
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)m.nx * nb) return;
  int i = (int)(t % m.nx), b = (int)(t / m.nx);
  int bf = side == 0 ? lo : hi;
  R v;
  if (kind == FARGO_BC_REFLECT) v = R(0);
  else if (kind == FARGO_BC_OUTFLOW) v = vn[at(m, dir, i, side == 0 ? lo + 1 : hi - 1, b)];
  else v = vn[at(m, dir, i, lo, b)]; // periodic image of the lower boundary face (side 1 only)
  vn[at(m, dir, i, bf, b)] = v;
}

template <typename R>
__global__ __launch_bounds__(256) void k_bc_ghosts(Mesh m, int dir, int side, int kind, Cen<R> cen, R *vn) {
  int lo = dir == 1 ? m.j0 : m.k0, hi = dir == 1 ? m.jn : m.kn;
  int nb = dir == 1 ? m.nzg : m.nyg;
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)m.nx * nb * NGH) return;
  int i = (int)(t % m.nx);
  long r = t / m.nx;
  int b = (int)(r % nb), g = (int)(r / nb);
  int dst, src, fdst = -1, fsrc = -1;
  R sgn = R(1);
  if (side == 0) {
    dst = lo - 1 - g;
    fdst = lo - 1 - g;
    if (kind == FARGO_BC_PERIODIC) { src = hi - 1 - g; fsrc = hi - 1 - g; }
    else if (kind == FARGO_BC_REFLECT) { src = lo + g; fsrc = lo + 1 + g; sgn = R(-1); }
    else { src = lo; fsrc = lo; }
  } else {
    dst = hi + g;
    if (g < NGH - 1) fdst = hi + 1 + g;
    if (kind == FARGO_BC_PERIODIC) { src = lo + g; fsrc = lo + 1 + g; }
    else if (kind == FARGO_BC_REFLECT) { src = hi - 1 - g; fsrc = hi - 1 - g; sgn = R(-1); }
    else { src = hi - 1; fsrc = hi; }
  }
  size_t d = at(m, dir, i, dst, b), s = at(m, dir, i, src, b);
  for (int q = 0; q < cen.n; q++) cen.p[q][d] = cen.p[q][s];
  if constexpr (sizeof(R) == 4) {
    // FP32 v_x is a deviation from the ring's background: the ghost takes the
    // source's full velocity, so the two backgrounds' difference is added
    if (cen.ivx >= 0) {
      const int jd = dir == 1 ? dst : b, kd = dir == 1 ? b : dst;
      const int js = dir == 1 ? src : b, ks = dir == 1 ? b : src;
      const double off = m.bg(BG_V, js, ks) - m.bg(BG_V, jd, kd);
      cen.p[cen.ivx][d] = cen.p[cen.ivx][s] + (R)off;
    }
  }
  if (fdst >= 0) vn[at(m, dir, i, fdst, b)] = sgn * vn[at(m, dir, i, fsrc, b)];
}

template <typename R>
void one_dir(Launch &L, const Mesh &m, int dir, const Cen<R> &cen, R *vn) {
  int nb = dir == 1 ? m.nzg : m.nyg;
  int k0 = dir == 1 ? 0 : 2;
  long nf = (long)m.nx * nb;
  for (int side = 0; side < 2; side++) {
    int kind = m.bc[k0 + side];
    if (kind == FARGO_BC_FIXED) continue;
    if (kind == FARGO_BC_PERIODIC && side == 0) continue; // the lower face is owned by the step
    prof_begin(L, K_BC_FACES);
    k_bc_faces<R><<<(unsigned)((nf + 255) / 256), 256, 0, L.s>>>(m, dir, side, kind, vn);
    prof_end(L, K_BC_FACES);
  }
  long ng = nf * NGH;
  for (int side = 0; side < 2; side++) {
    int kind = m.bc[k0 + side];
    if (kind == FARGO_BC_FIXED) continue;
    prof_begin(L, K_BC_GHOSTS);
    k_bc_ghosts<R><<<(unsigned)((ng + 255) / 256), 256, 0, L.s>>>(m, dir, side, kind, cen, vn);
    prof_end(L, K_BC_GHOSTS);
  }
}

} // namespace

template <typename R>
void launch_bc(Launch &L, const Mesh &m, R *rho, R *e, R *vx, R *vy, R *vz) {
  Cen<R> cy{};
  cy.p[cy.n++] = rho;
  if (e) cy.p[cy.n++] = e;
  cy.ivx = cy.n;
  cy.p[cy.n++] = vx;
  if (m.d3) cy.p[cy.n++] = vz;
  one_dir(L, m, 1, cy, vy);
  if (!m.d3) return;
  Cen<R> cz{};
  cz.p[cz.n++] = rho;
  if (e) cz.p[cz.n++] = e;
  cz.ivx = cz.n;
  cz.p[cz.n++] = vx;
  cz.p[cz.n++] = vy;
  one_dir(L, m, 2, cz, vz);
}

template void launch_bc<double>(Launch &, const Mesh &, double *, double *, double *, double *, double *);
template void launch_bc<float>(Launch &, const Mesh &, float *, float *, float *, float *, float *);

} // namespace fargo
