// particles_impl.h -- particle coupling kernels (Sec. 3).
//
// Per step, for the state at time T (post-collision populations f*(T), labels
// G(T), particle state P(T)), two kernels with one workgroup per particle
// bracket the sweep:
//   k_pre    before the sweep: enumerate the exterior pulls crossing the
//            particle's surface inside its bounding box, compact them into an
//            LDS list (deterministic block scan); for each link add the
//            momentum exchange of Eq. MP1 and its torque (Eq. MP4) in FP64
//            and write the moving-wall bounce-back (Eqs. MP7-MP8) into the
//            link's two pull slots, so the sweep pulls unconditionally; sum
//            the repulsion from solid nodes and from the other particles
//            (Eq. MP2, one lane per particle pair); then one lane takes the
//            Newton-Euler step of Eqs. MP5-MP6 into P(T+1).
//   k_post   after the sweep: the covered/uncovered-node force (Eq. MP3) of
//            the nodes whose label changes from G(T) to G(T+1), and G(T+1)
//            written into the label plane.
// All reductions run in a fixed order, so results are bit-reproducible.
#pragma once

#include "lb_device.h"

namespace lbk {

constexpr int LINK_CAP = 6144;
// The host admits no particle whose box side W = 2 reach + 2 has W^2 above
// LINK_CAP (W <= 78), so the box with a one-node rim fits 80 x 80 labels.
constexpr int LAB_BOX = 80 * 80;
constexpr uint8_t LBL_OUT = 0xff;  // rim or box node outside a non-periodic domain

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of NV values over the 256 threads of a block, fixed order; result valid
// in every thread.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*scratch)[NV]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) scratch[w][k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = (scratch[0][k] + scratch[1][k]) + (scratch[2][k] + scratch[3][k]);
  __syncthreads();
}

// Exclusive prefix sum of one int per thread over the block (fixed order).
__device__ __forceinline__ int block_exscan(int v, int *sh, int &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  int base = 0;
  for (int k = 0; k < w; ++k) base += sh[k];
  total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return base + incl - v;
}

// Map a box coordinate into the domain: any integer on a periodic axis (so a
// corrupted particle position can never index outside the planes), rejected
// outside a non-periodic axis.
__device__ __forceinline__ bool wrap_coord(int &v, int n, bool periodic) {
  if (v < 0 || v >= n) {
    if (!periodic) return false;
    v %= n;
    if (v < 0) v += n;
  }
  return true;
}

__device__ __forceinline__ double lj_mag(const DevDomain &D, double gap) {
  const double g = gap < D.lj_floor ? D.lj_floor : gap;
  return D.lj_psi * pow(g / D.lj_rit, -13.0);
}

struct PDisc {
  double x, y, radius;
};

// One of two particle records, chosen field by field (a select of the whole
// record by a runtime condition would go through private memory).
__device__ __forceinline__ PState pick_state(bool second, const PState &a, const PState &b) {
  PState r;
  r.x = second ? b.x : a.x;
  r.y = second ? b.y : a.y;
  r.ux = second ? b.ux : a.ux;
  r.uy = second ? b.uy : a.uy;
  r.omega = second ? b.omega : a.omega;
  r.radius = second ? b.radius : a.radius;
  r.mass = second ? b.mass : a.mass;
  r.inertia = second ? b.inertia : a.inertia;
  r.rho_ratio = second ? b.rho_ratio : a.rho_ratio;
  r.fx = second ? b.fx : a.fx;
  r.fy = second ? b.fy : a.fy;
  r.torque = second ? b.torque : a.torque;
  r.flags = second ? b.flags : a.flags;
  r.pad = 0;
  r.pad2[0] = r.pad2[1] = r.pad2[2] = 0.0;
  return r;
}

// Repulsion on particle p from particle q (Eq. MP2), both from P(T): zero
// for q == p or beyond the interaction range.
__device__ __forceinline__ void pair_repulsion(const DevDomain &D, const PState &P,
                                               const PDisc &Q, double &lx, double &ly) {
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  const double dx = min_image(P.x - Q.x, D.nx, perx), dy = min_image(P.y - Q.y, D.ny, pery);
  const double dist = sqrt(dx * dx + dy * dy);
  const double gap = dist - P.radius - Q.radius;
  if (gap > D.lj_rit || !(dist > 0.0)) return;
  const double m = lj_mag(D, gap);
  lx += m * dx / dist;
  ly += m * dy / dist;
}

// Newton-Euler step (Eqs. MP5-MP6) of particle p from its state P = P(T),
// its link, cover and solid-repulsion forces F and its particle-particle
// repulsion (lx, ly), into P(T+1); with F_FAVG the update takes the mean of
// this step's total force and torque and the previous step's, which P(T)
// holds.
__device__ __forceinline__ void advance_particle(const DevDomain &D, int p, const PState &P,
                                                 PState *nxt, const PForce &F, double lx,
                                                 double ly) {
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  const double fx = F.fx + F.cx_ + (lx + F.ljx);
  const double fy = F.fy + F.cy_ + (ly + F.ljy);
  const double tq = F.torque + F.ctorque;
  // optional: the mean of this and the previous step's totals (kept in P)
  const bool avg = (D.feat & F_FAVG) != 0;
  const double fxu = avg ? 0.5 * (fx + P.fx) : fx;
  const double fyu = avg ? 0.5 * (fy + P.fy) : fy;
  const double tqu = avg ? 0.5 * (tq + P.torque) : tq;
  PState N = P;
  N.fx = fx;
  N.fy = fy;
  N.torque = tq;
  if (!(P.flags & 1)) {
    const double buoy = 1.0 - D.rho0 / (P.rho_ratio * D.rho0);
    N.ux = P.ux + fxu / P.mass + buoy * D.gx;
    N.uy = P.uy + fyu / P.mass + buoy * D.gy;
    N.omega = P.omega + tqu / P.inertia;
    N.x = P.x + P.ux;
    N.y = P.y + P.uy;
    if (perx) { if (N.x >= D.nx) N.x -= D.nx; if (N.x < 0.0) N.x += D.nx; }
    if (pery) { if (N.y >= D.ny) N.y -= D.ny; if (N.y < 0.0) N.y += D.ny; }
    if (!(fabs(N.ux) < 0.5 && fabs(N.uy) < 0.5)) atomicOr(D.health, HEALTH_FAST_PARTICLE);
  }
  nxt[p] = N;
}

// Before the sweep of step T -> T+1, one workgroup per particle p.
//
// Links: an exterior fluid node x and an interior node s = x - e_d of p.  The
// pull into x along d and the pull into s along -e_d both bounce off the
// surface point r_b = x - e_d/2 moving at u_b = U + Omega z x (r_b - r_c):
//   f_d(x)  <- f*_{-d}(x) + M,   f_{-d}(s) <- f*_d(s) - M,   M = 6 rho0 w_d (u_b . e_d).
// The slots those two pulls read -- (d, s) and (-d, x) -- are read by no other
// pull and by no other link (s lies inside one particle only), so each link's
// thread reads f*_{-d}(x) for the force and writes the bounced values there
// in place, and the sweep pulls every direction unconditionally.
template <int ST>
__device__ __forceinline__ void pre_body(const DevDomain *__restrict__ doms,
                                         const PItem *__restrict__ items, int kstep) {
  using S = Store<ST>;
  using T = typename S::T;
  using RS = typename S::R;
  __shared__ uint32_t links[LINK_CAP];
  __shared__ int scan_sh[4];
  __shared__ double red[4][7];
  // labels G(T) of the box and a one-node rim (out of the domain: LBL_OUT)
  __shared__ uint8_t lab[LAB_BOX];
  const PItem it = items[blockIdx.x];
  const DevDomain &D = doms[it.dom];
  // The step counter, this particle's record in both state buffers, its force
  // record (read by the update at the end) and, one per lane, the other
  // particles' records in both buffers are requested together: none depends
  // on another, so choosing the buffer by the step's parity afterwards costs
  // no extra round trip through memory (this kernel is a latency chain).
  const uint64_t T0 = *D.tstep + (uint64_t)kstep;
  const PState Pa = D.pstate[0][it.p], Pb = D.pstate[1][it.p];
  const PForce Fpre = D.pforce[it.p];
  const int qme = (int)threadIdx.x;  // np <= MAX_PARTICLES <= 256: one particle per lane
  const bool pair_lane = D.lj_psi > 0.0 && qme < D.np && qme != it.p;
  PDisc qa{0.0, 0.0, 0.0}, qb{0.0, 0.0, 0.0};
  if (pair_lane) {
    const PState &A = D.pstate[0][qme], &B = D.pstate[1][qme];
    qa = PDisc{A.x, A.y, A.radius};
    qb = PDisc{B.x, B.y, B.radius};
  }
  static_assert(MAX_PARTICLES <= 256, "one particle per lane");
  const PState P = pick_state((T0 & 1) != 0, Pa, Pb);
  T *f = (T *)D.f[T0 & 1];
  const size_t plane = (size_t)D.ny * D.pitch;
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  const uint8_t mine = (uint8_t)(LBL_PART0 + it.p);
  const int reach = max((int)ceil(P.radius) + 2, (int)ceil(P.radius + D.lj_rit) + 1);
  const int W = 2 * reach + 2;
  const int bx0 = (int)floor(P.x) - reach, by0 = (int)floor(P.y) - reach;
  const int nbox = W * W;
  const int chunk = (nbox + 255) / 256;
  const double lim = P.radius + D.lj_rit;

  // stage the labels: box position (i, k) -> lab[(k + 1) * WR + i + 1]
  const int WR = W + 2;
  for (int j = threadIdx.x; j < WR * WR; j += 256) {
    int x = bx0 - 1 + j % WR, y = by0 - 1 + j / WR;
    const bool in = wrap_coord(x, D.nx, perx) && wrap_coord(y, D.ny, pery);
    lab[j] = in ? D.label[(size_t)y * D.pitch + x] : LBL_OUT;
  }
  __syncthreads();
  auto lab_at = [&](int i, int k) { return lab[(k + 1) * WR + i + 1]; };

  // pass 1: count crossing exterior pulls of this thread's contiguous nodes,
  // and sum the repulsion from solid nodes
  int cnt = 0;
  double ljx = 0.0, ljy = 0.0;
  for (int j = threadIdx.x * chunk; j < min(nbox, (threadIdx.x + 1) * chunk); ++j) {
    const int bi = j % W, bk = j / W;
    const uint8_t lx = lab_at(bi, bk);
    if (lx == LBL_OUT) continue;
    if (lx == LBL_SOLID) {
      int x = bx0 + bi, y = by0 + bk;
      wrap_coord(x, D.nx, perx);
      wrap_coord(y, D.ny, pery);
      const double dx = min_image(P.x - x, D.nx, perx), dy = min_image(P.y - y, D.ny, pery);
      const double dist = sqrt(dx * dx + dy * dy);
      if (dist <= lim && dist > 0.0) {
        const double m = lj_mag(D, dist - P.radius);
        ljx += m * dx / dist;
        ljy += m * dy / dist;
      }
      continue;
    }
    if (lx != LBL_FLUID) continue;
    for (int i = 1; i < 9; ++i)
      if (lab_at(bi - cx(i), bk - cy(i)) == mine) ++cnt;
  }
  int total;
  int pos = block_exscan(cnt, scan_sh, total);
  // pass 2: write this thread's links in node order into the LDS list
  for (int j = threadIdx.x * chunk; j < min(nbox, (threadIdx.x + 1) * chunk); ++j) {
    if (!cnt) break;
    const int bi = j % W, bk = j / W;
    if (lab_at(bi, bk) != LBL_FLUID) continue;
    for (int i = 1; i < 9; ++i) {
      if (lab_at(bi - cx(i), bk - cy(i)) == mine) {
        if (pos < LINK_CAP) links[pos] = ((uint32_t)j << 4) | (uint32_t)i;
        ++pos;
      }
    }
  }
  __syncthreads();
  // the host admits no radius whose box could hold more links than the list
  if (total > LINK_CAP && threadIdx.x == 0) atomicOr(D.health, HEALTH_LINK_OVERFLOW);
  const int nl = min(total, LINK_CAP);
  // pass 3: momentum exchange (FP64) and moving-wall bounce-back of each link
  // repulsion from the other particles, one lane per pair
  double plx = 0.0, ply = 0.0;
  if (pair_lane) {
    const bool odd = (T0 & 1) != 0;
    const PDisc Q{odd ? qb.x : qa.x, odd ? qb.y : qa.y, odd ? qb.radius : qa.radius};
    pair_repulsion(D, P, Q, plx, ply);
  }
  double acc[7] = {0.0, 0.0, 0.0, ljx, ljy, plx, ply};
  for (int e = threadIdx.x; e < nl; e += 256) {
    const uint32_t rec = links[e];
    const int j = (int)(rec >> 4), dir = (int)(rec & 15u);
    int x = bx0 + j % W, y = by0 + j / W;
    wrap_coord(x, D.nx, perx);
    wrap_coord(y, D.ny, pery);
    int sx = x - cx(dir), sy = y - cy(dir);
    wrap_coord(sx, D.nx, perx);
    wrap_coord(sy, D.ny, pery);
    const uint32_t here = (uint32_t)y * D.pitch + x, so = (uint32_t)sy * D.pitch + sx;
    const int o = opp(dir);
    const double a = (double)S::load(f + o * plane, here, o);
    const double b = (double)S::load(f + dir * plane, so, dir);
    const double fopp = wgt<double>(o) * D.rho0 + a;
    const double bxr = x - 0.5 * cx(dir), byr = y - 0.5 * cy(dir);
    const double rx = min_image(bxr - P.x, D.nx, perx), ry = min_image(byr - P.y, D.ny, pery);
    const double vx = P.ux - P.omega * ry, vy = P.uy + P.omega * rx;
    const double ue = vx * cx(dir) + vy * cy(dir);
    const double mag = 2.0 * fopp + 6.0 * D.rho0 * wgt<double>(dir) * ue;
    const double dpx = -cx(dir) * mag, dpy = -cy(dir) * mag;
    acc[0] += dpx;
    acc[1] += dpy;
    acc[2] += rx * dpy - ry * dpx;
    const double M = 6.0 * D.rho0 * wgt<double>(dir) * ue;
    S::put(f + dir * plane, so, dir, (RS)(a + M), 0u);
    S::put(f + o * plane, here, o, (RS)(b - M), 0u);
  }
  block_sum<7>(acc, red);
  if (threadIdx.x == 0) {
    PForce F = Fpre;
    F.fx = acc[0];
    F.fy = acc[1];
    F.torque = acc[2];
    F.ljx = acc[3];
    F.ljy = acc[4];
    D.pforce[it.p] = F;
    advance_particle(D, it.p, P, D.pstate[(T0 + 1) & 1], F, acc[5], acc[6]);
  }
}

// Label of node (x, y) from the particle discs Pn (PState, or PDisc staged in
// LDS): first particle (in index order) whose disc strictly contains the
// node, else fluid.
template <class Disc>
__device__ __forceinline__ uint8_t new_label(const DevDomain &D, const Disc *Pn, int x, int y) {
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  for (int q = 0; q < D.np; ++q) {
    const double dx = min_image((double)x - Pn[q].x, D.nx, perx);
    const double dy = min_image((double)y - Pn[q].y, D.ny, pery);
    if (dx * dx + dy * dy < Pn[q].radius * Pn[q].radius) return (uint8_t)(LBL_PART0 + q);
  }
  return LBL_FLUID;
}
// The same rule over the candidate discs cand[0 .. n) (ascending indices):
// the particles that can hold a node of the caller's box.
__device__ __forceinline__ uint8_t label_among(const DevDomain &D, const PDisc *Pn, const int *cand,
                                               int n, int x, int y) {
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  for (int k = 0; k < n; ++k) {
    const int q = cand[k];
    const double dx = min_image((double)x - Pn[q].x, D.nx, perx);
    const double dy = min_image((double)y - Pn[q].y, D.ny, pery);
    if (dx * dx + dy * dy < Pn[q].radius * Pn[q].radius) return (uint8_t)(LBL_PART0 + q);
  }
  return LBL_FLUID;
}

// After the sweep of step T -> T+1, one workgroup per particle p, over a box
// around P(T+1) that holds every node p leaves or enters (particles move less
// than half a node per step).  G(T) and G(T+1) of a non-solid node are the
// first-particle rule applied to P(T) and P(T+1), so no workgroup reads the
// label plane while others rewrite it (overlapping boxes write identical
// values).  Covered node (enters p): F = +rho (u - U_p); uncovered node:
// -rho (u - U_p), with rho and u = j/rho + g/2 the moments of f(T+1)
// (recovered from f*(T+1): j(f*) = j(f) + rho g), applied in the next step
// (Eq. MP3).
template <int ST>
__device__ __forceinline__ void post_body(const DevDomain *__restrict__ doms,
                                          const PItem *__restrict__ items, int kstep) {
  using S = Store<ST>;
  using T = typename S::T;
  __shared__ double red[4][3];
  __shared__ int scan_sh[4];
  // discs of P(T) and P(T+1) that can reach a node of this box, in index
  // order (so the first-particle rule is unchanged)
  __shared__ PDisc disc0[MAX_PARTICLES], disc1[MAX_PARTICLES];
  __shared__ int cand[MAX_PARTICLES];
  const PItem it = items[blockIdx.x];
  const DevDomain &D = doms[it.dom];
  // the step counter and the discs in both state buffers (this particle's
  // record, and one other particle per lane) are requested together, then
  // sorted into old and new by the step's parity: no dependent round trip
  const uint64_t T1 = *D.tstep + (uint64_t)kstep + 1;
  const PState Pa = D.pstate[0][it.p], Pb = D.pstate[1][it.p];
  const int qme = (int)threadIdx.x;  // MAX_PARTICLES <= 256: one disc per lane
  PDisc qa{0.0, 0.0, 0.0}, qb{0.0, 0.0, 0.0};
  if (qme < D.np) {
    const PState &A = D.pstate[0][qme], &B = D.pstate[1][qme];
    qa = PDisc{A.x, A.y, A.radius};
    qb = PDisc{B.x, B.y, B.radius};
  }
  const bool odd = (T1 & 1) != 0;
  const PState P = pick_state(odd, Pa, Pb);  // P(T+1)
  const T *src = (const T *)D.f[T1 & 1];
  const size_t plane = (size_t)D.ny * D.pitch;
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  const uint8_t mine = (uint8_t)(LBL_PART0 + it.p);
  const int reach = (int)ceil(P.radius) + 3;
  const int W = 2 * reach + 2;
  const int bx0 = (int)floor(P.x) - reach, by0 = (int)floor(P.y) - reach;
  int ncand;
  {
    static_assert(MAX_PARTICLES <= 256, "one candidate test per lane");
    // a node of the box lies within (W - 1) / 2 of the box centre on each
    // axis, so a disc holding one has its centre within r + W / 2 + 1
    const int q = qme;
    int hit = 0;
    if (q < D.np) {
      const double bcx = bx0 + 0.5 * (W - 1), bcy = by0 + 0.5 * (W - 1), h = 0.5 * W + 1.0;
      const PDisc A{odd ? qa.x : qb.x, odd ? qa.y : qb.y, odd ? qa.radius : qb.radius};  // P(T)
      const PDisc B{odd ? qb.x : qa.x, odd ? qb.y : qa.y, odd ? qb.radius : qa.radius};  // P(T+1)
      disc0[q] = A;
      disc1[q] = B;
      hit = (fabs(min_image(A.x - bcx, D.nx, perx)) < h + A.radius &&
             fabs(min_image(A.y - bcy, D.ny, pery)) < h + A.radius) ||
            (fabs(min_image(B.x - bcx, D.nx, perx)) < h + B.radius &&
             fabs(min_image(B.y - bcy, D.ny, pery)) < h + B.radius);
    }
    const int pos = block_exscan(hit, scan_sh, ncand);
    if (hit) cand[pos] = q;
    __syncthreads();
  }
  double acc[3] = {0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < W * W; j += 256) {
    int x = bx0 + j % W, y = by0 + j / W;
    if (!wrap_coord(x, D.nx, perx) || !wrap_coord(y, D.ny, pery)) continue;
    const uint32_t here = (uint32_t)y * D.pitch + x;
    if (D.nodew[here] & NODE_SOLID) continue;
    const uint8_t l0 = label_among(D, disc0, cand, ncand, x, y);
    const uint8_t l1 = label_among(D, disc1, cand, ncand, x, y);
    if (l1 != l0) D.label[here] = l1;
    if ((l0 == mine) == (l1 == mine)) continue;
    const double sign = l1 == mine ? 1.0 : -1.0;
    double drho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
      const double v = (double)S::load(src + i * plane, here, i);
      drho += v;
      jx += v * cx(i);
      jy += v * cy(i);
    }
    const double rho = D.rho0 + drho;
    const double ux = jx / rho - 0.5 * D.gx, uy = jy / rho - 0.5 * D.gy;
    const double fx = sign * rho * (ux - P.ux), fy = sign * rho * (uy - P.uy);
    const double rx = min_image(x - P.x, D.nx, perx), ry = min_image(y - P.y, D.ny, pery);
    acc[0] += fx;
    acc[1] += fy;
    acc[2] += rx * fy - ry * fx;
  }
  block_sum<3>(acc, red);
  if (threadIdx.x == 0) {
    PForce &F = D.pforce[it.p];
    F.cx_ = acc[0];
    F.cy_ = acc[1];
    F.ctorque = acc[2];
  }
}

template <int ST>
__global__ __launch_bounds__(256) void k_pre(const DevDomain *__restrict__ doms,
                                             const PItem *__restrict__ items, int kstep) {
  pre_body<ST>(doms, items, kstep);
}

template <int ST>
__global__ __launch_bounds__(256) void k_post(const DevDomain *__restrict__ doms,
                                              const PItem *__restrict__ items, int kstep) {
  post_body<ST>(doms, items, kstep);
}

// k_post of step kstep and k_pre of step kstep + 1 in one launch, for
// launches in which no domain holds more than one particle.  Then each
// workgroup's particle is alone in its domain: no other workgroup touches
// its labels, populations or records, and the barrier between the two
// halves orders everything the second half reads (the labels and the cover
// force just written, the populations the first half read before the
// bounce-back writes).  One launch less per step, the same results.  With
// two or more particles in a domain the halves of different workgroups
// would race (a disc's bounce-back writes can reach nodes a neighbour's
// cover force still reads), so those launches keep the two kernels.
template <int ST>
__global__ __launch_bounds__(256) void k_post_pre(const DevDomain *__restrict__ doms,
                                                  const PItem *__restrict__ items, int kstep) {
  post_body<ST>(doms, items, kstep);
  __syncthreads();
  pre_body<ST>(doms, items, kstep + 1);
}

#ifdef LBK_COMMON_KERNELS
// Labels of the current particle state inside each particle's box, from the
// label plane's own values (used once the particles are added).
__global__ __launch_bounds__(256) void k_relabel(const DevDomain *__restrict__ doms,
                                                 const PItem *__restrict__ items) {
  const PItem it = items[blockIdx.x];
  const DevDomain &D = doms[it.dom];
  const PState *Pn = D.pstate[*D.tstep & 1];
  const PState P = Pn[it.p];
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  const int reach = (int)ceil(P.radius) + 3;
  const int W = 2 * reach + 2;
  const int bx0 = (int)floor(P.x) - reach, by0 = (int)floor(P.y) - reach;
  for (int j = threadIdx.x; j < W * W; j += 256) {
    int x = bx0 + j % W, y = by0 + j / W;
    if (!wrap_coord(x, D.nx, perx) || !wrap_coord(y, D.ny, pery)) continue;
    const size_t here = (size_t)y * D.pitch + x;
    const uint8_t l0 = D.label[here];
    if (l0 == LBL_SOLID) continue;
    const uint8_t l1 = new_label(D, Pn, x, y);
    if (l1 != l0) D.label[here] = l1;
  }
}

// [a0, a1] meets [b0, b1] (inclusive node ranges; b may reach past the
// domain, whose periodic images count on a periodic axis)
__device__ __forceinline__ bool ranges_meet(int a0, int a1, int b0, int b1, int n, bool periodic) {
  if (b0 <= a1 && a0 <= b1) return true;
  if (!periodic) return false;
  return (b0 - n <= a1 && a0 <= b1 - n) || (b0 + n <= a1 && a0 <= b1 + n);
}

// Sweep tiles that the particle coupling around the state T = tstep + kstep
// touches: k_post of the step before (labels in a box of reach ceil(R) + 3
// around P(T)) and k_pre (link slots within one node of a box of reach
// max(ceil(R) + 2, ceil(R + r_it) + 1) around P(T)).  A tile is flagged when
// its nodes or the nodes its pulls read (one-node halo) come within two nodes
// of the larger box, into near_tiles[T & 1].  One thread per tile.
__global__ __launch_bounds__(256) void k_near_tiles(const DevDomain *__restrict__ Dp, int kstep) {
  const DevDomain &D = *Dp;
  const int t = (int)(blockIdx.x * 256 + threadIdx.x);
  if (t >= D.tiles_x * D.tiles_y) return;
  const uint64_t T = *D.tstep + (uint64_t)kstep;
  const PState *P = D.pstate[T & 1];
  const int th = (256 / D.tile_w) * D.rows_per_thread;
  const int ty = t / D.tiles_x, tx = t - ty * D.tiles_x;
  const int x0 = tx * D.tile_w - 1, x1 = min((tx + 1) * D.tile_w, D.nx);
  const int y0 = ty * th - 1, y1 = min((ty + 1) * th, D.ny);
  const bool perx = D.bc_x == BC_PERIODIC, pery = D.bc_y == BC_PERIODIC;
  uint8_t hit = 0;
  for (int p = 0; p < D.np && !hit; ++p) {
    const PState &Q = P[p];
    const int reach =
        max((int)ceil(Q.radius) + 3, (int)ceil(Q.radius + D.lj_rit) + 1) + 2;
    const int cx0 = (int)floor(Q.x), cy0 = (int)floor(Q.y);
    hit = ranges_meet(x0, x1, cx0 - reach, cx0 + reach + 1, D.nx, perx) &&
          ranges_meet(y0, y1, cy0 - reach, cy0 + reach + 1, D.ny, pery);
  }
  D.near_tiles[T & 1][t] = hit;
}
#endif  // LBK_COMMON_KERNELS

}  // namespace lbk
