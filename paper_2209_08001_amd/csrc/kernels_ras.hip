// Restricted additive Schwarz preconditioner with LDS-resident subdomains (Section 4).
//
// z = sum_t R_t^0' A_t^{-1} R_t^delta r: every workgroup owns one tile of T_x x T_y (x T_z)
// nodes, extends it by delta layers on every side (overlap), and solves the restriction
// A_t = J[ext, ext] of the Newton Jacobian to that extended block (zero Dirichlet exterior)
// approximately with symmetric multicolour block Gauss-Seidel sweeps; only the owned nodes
// are written back (the restricted prolongation R_t^0').
//
// The iterate of the whole extended tile lives in LDS with a zero ring: one node wide for the
// eta fields (nearest-neighbour coupling), two with the displacement rows (sigma reaches
// distance 2).  Without them the c iterate is read only at its own node (its couplings to
// the rest of the diamond go through dG, kept in LDS), so it stays in the registers of the
// thread that owns the node.  The Jacobian couples nodes up to distance 2 (the 13-point
// diamond in 2D, 25 points in 3D).
// Colour (i + 2j) mod 5 (2D) or (i + 2j + 3k) mod 7 (3D) separates every pair of nodes
// inside one diamond, so all nodes of a colour update at once, exactly as sequential
// Gauss-Seidel would.  The pieces of each node's diagonal block (formed once per time step by
// k_ras_pack) and the right-hand side stay in registers of the thread that owns the node; the
// c row of the chemical block, which the dG updates need, sits in LDS.
//
// Tile operator, per node (the Jacobian of the residual, written in the kernels_phase notes):
//   dG    = B_c.z + kel z_c - (eps0/2) Ctr div_h z_u - (gamma_c/2) Lap_h z_c   on ext and its ring
//   (Az)_c = z_c/dt - div_h(M grad_h dG)
//   (Az)_e = z_e/dt + L_eta (B_e.z - (gamma_eta/2) Lap_h z_e)
//   (Az)_u = sum_J Dhat_J sigma_IJ(z_u, z_c)                      (only when with_u)
#include "pf_internal.h"

namespace pf {

namespace {

// workgroup sizes of the tile kernel: 512 threads, or 256 when the tile fits four nodes per
// thread and two or more workgroups fit the LDS of one compute unit (they then overlap their
// barriers, and fewer of their waves idle in a colour phase)
constexpr int kRasThreadsMax = 512, kRasThreadsSmall = 256;

// Schwarz variants (Section 4): left-RAS z = sum_t R0_t' A_t^{-1} R_t r (owned part of each
// tile's solution), classical AS z = sum_t R_t' A_t^{-1} R_t r and right-RAS
// z = sum_t R_t' A_t^{-1} R0_t r (whole extended solutions summed where tiles overlap; right-
// RAS restricts r to the owned nodes first).  The summing variants write each tile's
// extended solution to a scratch array and a gather kernel adds, per node, the solutions of
// the tiles covering it in a fixed order (deterministic).
enum { kRasLeft = 0, kRasClassical = 1, kRasRight = 2 };

struct Geo {
  int ex, ey, ez;      // extended tile
  int zx, zy, zz;      // LDS iterate (ext + ring of 2 with u, of 1 without; zz = 1 in 2D)
  int dx, dy, dz;      // dG / mobility arrays (ext + ring of 1; dz = 1 in 2D)
  int ntx, nty;        // tiles per direction
  int tx, ty, tz, ov;
  int sweeps;
  int mode;            // kRasLeft, kRasClassical or kRasRight
  double omega;        // over-relaxation of the block updates (1: plain Gauss-Seidel)
};

__device__ inline int wrapg(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

constexpr int kPackVals = 13;  // per extended-tile node: E^{-1} (9), w = E^{-1} v (3), 1 / (d_cc - u'w)

// Per time step (the preconditioner blocks are lagged): the constant pieces of every extended-
// tile node's diagonal block of the tile operator (the node's own unknowns),
//   [d_cc  u'  ]      d_cc = 1/dt + sc (B_cc + kel + gamma_c (2 DIM + 1) / (2 h^2)),
//   [v     E   ]      u_e = sc B_ce, v_e = L_eta B_ec, E = dee I + L_eta B_ee,
// dee = 1/dt + L_eta gamma_eta DIM / h^2, sc = (sum of the 2 DIM face mobilities
// kappa/2 (g_i + g_j), g = c^n (1 - c^n)) / h^2: E^{-1} by the adjugate, w = E^{-1} v and the
// Schur denominator 1 / (d_cc - u'w).  Stored per tile in colour order (plane k of tile t at
// pack[(t kPackVals + k) ne + pos]), so that the tile kernel's thread for colour position pos
// reads them with coalesced loads.  Here the nodes are taken in natural order (coalesced
// loads) and scattered to their colour positions (iperm).
constexpr int kPackThreads = 1024;
template <int DIM, typename R>
__global__ __launch_bounds__(kPackThreads) void k_ras_pack(Consts K, Geo G, double dt, const R* __restrict__ Bg,
                                                           const double* __restrict__ cn,
                                                           const int* __restrict__ iperm, R* __restrict__ pack,
                                                           Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    Bg = bat_at(Bg, bo);
    cn = bat_at(cn, bo);
    pack = bat_at(pack, bo);
  }
  dt = bat_s(bt, bi, dt);
  const int t = blockIdx.x;
  const int tix = t % G.ntx, tiy = (t / G.ntx) % G.nty, tiz = t / (G.ntx * G.nty);
  const int ox = tix * G.tx - G.ov, oy = tiy * G.ty - G.ov, oz = (DIM == 3) ? tiz * G.tz - G.ov : 0;
  const int ne = G.ex * G.ey * G.ez;
  const long long N = K.N;
  // coefficients in the arithmetic type of the solve (formed in double, rounded once)
  const R idt = (R)(1.0 / dt);
  const R ih2 = (R)K.ih2, Le = (R)K.L_eta, hk = (R)(0.5 * K.kappa);
  const R dcc1 = (R)(K.kel + K.gamma_c * DIM * K.ih2 + 0.5 * K.gamma_c * K.ih2);
  const R dee = (R)(1.0 / dt + K.L_eta * K.gamma_eta * DIM * K.ih2);
  R* out = pack + (long long)t * kPackVals * ne;
  auto gnode = [&](int i, int j, int k) {
    return (long long)wrapg(i, K.nx) + (long long)K.nx * ((long long)wrapg(j, K.ny) + (long long)K.ny * wrapg(k, K.nz));
  };
  auto gval = [&](long long m) {
    const double v = cn[m];
    return (R)(v * (1.0 - v));
  };
  for (int q = threadIdx.x; q < ne; q += blockDim.x) {
    const int pos = iperm[q];
    const int a = q % G.ex, b = (q / G.ex) % G.ey, c = q / (G.ex * G.ey);
    const int gi = ox + a, gj = oy + b, gk = (DIM == 3) ? oz + c : 0;
    const long long n = gnode(gi, gj, gk);
    R bv[12];
#pragma unroll
    for (int f = 0; f < 12; ++f) bv[f] = Bg[(4 + f) * N + n];
    // E^{-1} by the adjugate and w = E^{-1} v
    const R E00 = dee + Le * bv[1], E01 = Le * bv[2], E02 = Le * bv[3];
    const R E10 = Le * bv[5], E11 = dee + Le * bv[6], E12 = Le * bv[7];
    const R E20 = Le * bv[9], E21 = Le * bv[10], E22 = dee + Le * bv[11];
    const R A00 = E11 * E22 - E12 * E21, A01 = E02 * E21 - E01 * E22, A02 = E01 * E12 - E02 * E11;
    const R A10 = E12 * E20 - E10 * E22, A11 = E00 * E22 - E02 * E20, A12 = E02 * E10 - E00 * E12;
    const R A20 = E10 * E21 - E11 * E20, A21 = E01 * E20 - E00 * E21, A22 = E00 * E11 - E01 * E10;
    const R idet = R(1) / (E00 * A00 + E01 * A10 + E02 * A20);
    const R Ai[9] = {A00 * idet, A01 * idet, A02 * idet, A10 * idet, A11 * idet,
                     A12 * idet, A20 * idet, A21 * idet, A22 * idet};
    const R v1 = Le * bv[0], v2 = Le * bv[4], v3 = Le * bv[8];
    R w[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) w[e] = Ai[3 * e] * v1 + Ai[3 * e + 1] * v2 + Ai[3 * e + 2] * v3;
    // Schur denominator of the c row
    const R g0 = gval(n);
    R sumM = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const R gp = gval(gnode(gi + (d == 0), gj + (d == 1), gk + (d == 2)));
      const R gm = gval(gnode(gi - (d == 0), gj - (d == 1), gk - (d == 2)));
      sumM += hk * (g0 + gp) + hk * (g0 + gm);
    }
    const R sc = sumM * ih2;
    const R dcc = idt + sc * (Bg[n] + dcc1);
    const R uw = sc * (Bg[N + n] * w[0] + Bg[2 * N + n] * w[1] + Bg[3 * N + n] * w[2]);
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k * ne + pos] = Ai[k];
#pragma unroll
    for (int e = 0; e < 3; ++e) out[(9 + e) * ne + pos] = w[e];
    out[12 * ne + pos] = R(1) / (dcc - uw);
  }
}

// minimum waves per SIMD the registers are sized for (the second launch bound): two for
// 256-thread workgroups (two or more per compute unit), one for 512 threads (one per unit)
template <int TH>
constexpr int ras_waves_per_eu() {
  return TH == kRasThreadsSmall ? 2 : 1;
}

template <int DIM, bool WU, int NPT, typename R, int TH>
__global__ __launch_bounds__(TH, (ras_waves_per_eu<TH>())) void k_ras(Consts K, Geo G, double dt,
                                                     const R* __restrict__ Bg,
                                                     const double* __restrict__ cn,
                                                     const R* __restrict__ rg,
                                                     R* __restrict__ zg,
                                                     const int* __restrict__ permg,
                                                     const R* __restrict__ pack,
                                                     R* __restrict__ xs, Bat bt) {
  // instance of a lockstep batch (the colour order permg is shared, read from instance 0)
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    Bg = bat_at(Bg, bo);
    cn = bat_at(cn, bo);
    rg = bat_at(rg, bo);
    zg = bat_at(zg, bo);
    pack = bat_at(pack, bo);
    xs = bat_at(xs, bo);
  }
  dt = bat_s(bt, bi, dt);
  constexpr int NFZ = WU ? 4 + DIM : 4;
  constexpr int ZP0 = WU ? 0 : 1;     // first field of the iterate held in LDS
  constexpr int NZL = NFZ - ZP0;      // its LDS planes
  constexpr int NCOL = (DIM == 3) ? 7 : 5;
  extern __shared__ double lds_raw[];
  R* lds = reinterpret_cast<R*>(lds_raw);
  const int zsz = G.zx * G.zy * G.zz;
  const int dsz = G.dx * G.dy * G.dz;
  const int ne = G.ex * G.ey * G.ez;
  R* zs = lds;              // NZL planes of zsz: fields ZP0.. of the iterate with a zero ring
  R* dg = zs + NZL * zsz;   // dsz: dG on ext and a ring of 1
  R* gg = dg + dsz;         // dsz: g = c^n (1 - c^n)
  R* bc = gg + dsz;         // 4 planes of ne: c-row of the chemical block

  // tile of this workgroup: workgroups go to the 8 XCDs round-robin, so each XCD is given a
  // contiguous run of tiles (whole tile rows) and the overlap shared by neighbouring tiles is
  // fetched once into its own L2
  int t = blockIdx.x;
  if ((gridDim.x & 7) == 0) t = (t & 7) * (gridDim.x >> 3) + (t >> 3);
  const int tix = t % G.ntx, tiy = (t / G.ntx) % G.nty, tiz = t / (G.ntx * G.nty);
  const int ox = tix * G.tx - G.ov, oy = tiy * G.ty - G.ov, oz = (DIM == 3) ? tiz * G.tz - G.ov : 0;
  const long long N = K.N;
  const int sy = G.zx, sz = G.zx * G.zy;    // LDS strides of the iterate
  const int ty_ = G.dx, tz_ = G.dx * G.dy;  // strides of dG / g
  const int ring = WU ? 2 : 1;

  // Set-up, one barrier: g and dG = 0 on ext and its ring, the c-row blocks (coalesced), the
  // zero iterate, and each thread's own nodes (right-hand side and eta rows of the blocks,
  // straight into registers).
  for (int q = threadIdx.x; q < dsz; q += TH) {
    const int a = q % G.dx, b = (q / G.dx) % G.dy, c = q / (G.dx * G.dy);
    const int gi = wrapg(ox + a - 1, K.nx), gj = wrapg(oy + b - 1, K.ny);
    const int gk = (DIM == 3) ? wrapg(oz + c - 1, K.nz) : 0;
    const double v = cn[gi + (long long)K.nx * (gj + (long long)K.ny * gk)];
    gg[q] = (R)(v * (1.0 - v));
    dg[q] = R(0);
  }
  for (int q = threadIdx.x; q < ne; q += TH) {
    const int a = q % G.ex, b = (q / G.ex) % G.ey, c = q / (G.ex * G.ey);
    const int gi = wrapg(ox + a, K.nx), gj = wrapg(oy + b, K.ny);
    const int gk = (DIM == 3) ? wrapg(oz + c, K.nz) : 0;
    const long long n = gi + (long long)K.nx * (gj + (long long)K.ny * gk);
#pragma unroll
    for (int f = 0; f < 4; ++f) bc[f * ne + q] = Bg[f * N + n];
  }
  for (int q = threadIdx.x; q < NZL * zsz; q += TH) zs[q] = R(0);

  // Nodes of this thread: positions threadIdx.x + m TH of the colour-sorted order permg (ext
  // nodes grouped by colour, the same for every tile of this shape; formed by the host), so
  // the nodes of one colour sit on consecutive threads.
  R rr[NPT][NFZ];
  // E^{-1}, w and 1 / (d_cc - u'w) of each node (the diagonal block of the tile operator,
  // below), formed once per time step by k_ras_pack in colour order: coalesced loads
  R ai[NPT][9], wq[NPT][3], invd[NPT];
  R zcr_[NPT];  // c iterate of this thread's nodes (without u; LDS plane 0 with u)
  // per node, packed in 16-bit halves (every index is below 2^16): zd = iterate position |
  // dG position << 16; qc = ext index
  int zd_[NPT], qc_[NPT];
  int col_[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int pos = threadIdx.x + m * TH;
    col_[m] = -1;
    zd_[m] = qc_[m] = 0;
    zcr_[m] = R(0);
    if (pos < ne) {
      const int q = permg[pos];
      const int a = q % G.ex, b = (q / G.ex) % G.ey, c = q / (G.ex * G.ey);
      const int zi = (a + ring) + sy * (b + ring) + ((DIM == 3) ? sz * (c + ring) : 0);
      const int di = (a + 1) + ty_ * (b + 1) + ((DIM == 3) ? tz_ * (c + 1) : 0);
      col_[m] = (DIM == 3) ? (a + 2 * b + 3 * c) % 7 : (a + 2 * b) % 5;
      zd_[m] = zi | (di << 16);
      qc_[m] = q;
      const int gi = wrapg(ox + a, K.nx), gj = wrapg(oy + b, K.ny);
      const int gk = (DIM == 3) ? wrapg(oz + c, K.nz) : 0;
      const long long n = gi + (long long)K.nx * (gj + (long long)K.ny * gk);
      // right-RAS restricts the right-hand side to the owned nodes
      const bool owned = a >= G.ov && a < G.ov + G.tx && b >= G.ov && b < G.ov + G.ty &&
                         (DIM == 2 || (c >= G.ov && c < G.ov + G.tz));
      const bool keep = G.mode != kRasRight || owned;
#pragma unroll
      for (int f = 0; f < NFZ; ++f) rr[m][f] = keep ? rg[f * N + n] : R(0);
      const R* pk = pack + (long long)t * kPackVals * ne + pos;
#pragma unroll
      for (int k = 0; k < 9; ++k) ai[m][k] = pk[k * ne];
#pragma unroll
      for (int e = 0; e < 3; ++e) wq[m][e] = pk[(9 + e) * ne];
      invd[m] = pk[12 * ne];
    } else {
#pragma unroll
      for (int f = 0; f < NFZ; ++f) rr[m][f] = R(0);
#pragma unroll
      for (int k = 0; k < 9; ++k) ai[m][k] = R(0);
#pragma unroll
      for (int e = 0; e < 3; ++e) wq[m][e] = R(0);
      invd[m] = R(0);
    }
  }
  __syncthreads();

  // coefficients in the arithmetic type of the solve (formed in double, rounded once)
  const R idt = (R)(1.0 / dt);
  const R ih2 = (R)K.ih2, i2h = (R)K.i2h, eps0 = (R)K.eps0;
  const R C11 = (R)K.C11, C12 = (R)K.C12, C44 = (R)K.C44;
  const R hk = (R)(0.5 * K.kappa);
  const int sdir_z[3] = {1, sy, sz};
  const int sdir_d[3] = {1, ty_, tz_};
  const R a_u = (R)(-0.5 * K.eps0 * K.Ctr * K.i2h);  // coefficient of the difference of z_u in dG
  const R iduu = (R)(-2.0 * K.h * K.h / (K.C11 + (DIM - 1) * K.C44));
  const R cxu = (R)(K.eps0 * K.Ctr * 0.25 * K.ih2 * K.ih);
  const R cge = (R)(0.5 * K.L_eta * K.gamma_eta * K.ih2);  // eta-row neighbour coefficient
  const R dgc = (R)(K.kel + K.gamma_c * DIM * K.ih2);    // d dG / d z_c at the node (besides B_cc)
  const R dgn = (R)(-0.5 * K.gamma_c * K.ih2);           // d dG / d z_c at a neighbour
  const R om = (R)G.omega;
  // Per node, the diagonal block of the tile operator (the node's own unknowns) is
  //   [d_cc  u'  ]      d_cc = 1/dt + sc (B_cc + kel + gamma_c (2 DIM + 1) / (2 h^2)),
  //   [v     E   ]      u_e = sc B_ce, v_e = L_eta B_ec, E = dee I + L_eta B_ee,
  // sc = (sum of the 2 DIM face mobilities) / h^2; constant during the sweeps, its pieces
  // E^{-1}, w = E^{-1} v and 1 / (d_cc - u'w) come from k_ras_pack.

  // Block Gauss-Seidel update of one node.  The eta rows are taken in Gauss-Seidel form:
  // with rhs_e = r_e + (L_eta gamma_eta / (2 h^2)) (sum of the 2 DIM neighbours of z_e) the
  // new values satisfy E z_e' + v z_c' = rhs_e, so z_e' = y - w z_c' with y = E^{-1} rhs_e.
  // The c row is taken in correction form, x_c = (res_c - u'E^{-1} res_e) / (d_cc - u'w) with
  // E^{-1} res_e = y - z_e - w z_c; the displacement rows (with_u) by their diagonal.
  auto update_node = [&](const R* rv, const R* Ai, const R* w, R id, int zi, int di, int q, R& zcr) {
    R zv[NFZ], dgp[DIM], dgm[DIM];
    zv[0] = WU ? zs[zi] : zcr;
#pragma unroll
    for (int f = 1; f < NFZ; ++f) zv[f] = zs[(f - ZP0) * zsz + zi];
    // c row residual: r_c - (z_c/dt - div_h(M grad_h dG)); the dG values at the node and its
    // neighbours are kept for the write-back below
    // (the sums start from their first term: x + 0 is not folded away in floating point)
    R sumM, dM[3] = {R(0), R(0), R(0)};
    R divm;
    const R g0 = gg[di], dg0 = dg[di];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      dgp[d] = dg[di + sdir_d[d]];
      dgm[d] = dg[di - sdir_d[d]];
      const R Mp = hk * (g0 + gg[di + sdir_d[d]]);
      const R Mm = hk * (g0 + gg[di - sdir_d[d]]);
      const R dv = Mp * (dgp[d] - dg0) - Mm * (dg0 - dgm[d]);
      divm = (d == 0) ? dv : divm + dv;
      sumM = (d == 0) ? Mp + Mm : sumM + (Mp + Mm);
      dM[d] = Mm - Mp;
    }
    R xc = rv[0] - (zv[0] * idt - divm * ih2);
    // eta rows: y = E^{-1} rhs_e
    R rh[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const int ze = (1 + e - ZP0) * zsz + zi;
      R nb = zs[ze + 1] + zs[ze - 1];
#pragma unroll
      for (int d = 1; d < DIM; ++d) nb += zs[ze + sdir_z[d]] + zs[ze - sdir_z[d]];
      rh[e] = rv[1 + e] + cge * nb;
    }
    R y[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) y[e] = Ai[3 * e] * rh[0] + Ai[3 * e + 1] * rh[1] + Ai[3 * e + 2] * rh[2];
    // u rows: x_u = (r_u - sum_J Dhat_J sigma_IJ(z_u, z_c)) / d_uu, and their coupling into the c row
    R xu[3] = {R(0), R(0), R(0)};
    if (WU) {
#pragma unroll
      for (int I = 0; I < DIM; ++I) {
        R acc = R(0);
#pragma unroll
        for (int J = 0; J < DIM; ++J) {
#pragma unroll
          for (int sgn = -1; sgn <= 1; sgn += 2) {
            const int pz = zi + sgn * sdir_z[J];
            R sig;
            if (I != J) {
              sig = C44 * ((zs[(4 + J) * zsz + pz + sdir_z[I]] - zs[(4 + J) * zsz + pz - sdir_z[I]]) +
                           (zs[(4 + I) * zsz + pz + sdir_z[J]] - zs[(4 + I) * zsz + pz - sdir_z[J]])) * i2h;
            } else {
              const R ec = eps0 * zs[pz];
              sig = R(0);
#pragma unroll
              for (int L = 0; L < DIM; ++L) {
                const R e = (zs[(4 + L) * zsz + pz + sdir_z[L]] - zs[(4 + L) * zsz + pz - sdir_z[L]]) * i2h - ec;
                sig += (L == I ? C11 : C12) * e;
              }
            }
            acc += (sgn > 0) ? sig : -sig;
          }
        }
        xu[I] = (rv[4 + I] - acc * i2h) * iduu;
        xc -= cxu * dM[I] * xu[I];
      }
    }
    const R sc = sumM * ih2;
    R bcv[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) bcv[f] = bc[f * ne + q];
    R t = bcv[1] * (y[0] - zv[1] - w[0] * zv[0]);
#pragma unroll
    for (int e = 1; e < 3; ++e) t += bcv[1 + e] * (y[e] - zv[1 + e] - w[e] * zv[0]);
    xc = (xc - sc * t) * id;
    // over-relaxed block update: z <- z + omega (z_GS - z), z_GS the block Gauss-Seidel values
    // (c from the Schur form, eta = y - w c_GS)
    const R zcg = zv[0] + xc;
    xc *= om;
    const R zc = zv[0] + xc;
    if (WU) zs[zi] = zc;
    else zcr = zc;
    R dz[4];
    dz[0] = xc;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const R dze = om * (y[e] - w[e] * zcg - zv[1 + e]);
      zs[(1 + e - ZP0) * zsz + zi] = zv[1 + e] + dze;
      dz[1 + e] = dze;
    }
    if (WU) {
#pragma unroll
      for (int I = 0; I < DIM; ++I) {
        xu[I] *= om;
        zs[(4 + I) * zsz + zi] = zv[4 + I] + xu[I];
      }
    }
    // dG follows the change: at the node through B_c, kel and the centre of the Laplacian, at
    // the 2 DIM neighbours through the Laplacian (and the divergence of u).  Nodes of one
    // colour are at least three steps apart, so no other update of this phase reads or writes
    // these five (seven) dG values: the ones read above are still current.
    R dself = dgc * xc;
#pragma unroll
    for (int f = 0; f < 4; ++f) dself += bcv[f] * dz[f];
    dg[di] = dg0 + dself;
    const R dn = dgn * xc;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (WU) {
        const R du = a_u * xu[d];
        dg[di + sdir_d[d]] = dgp[d] + (dn - du);
        dg[di - sdir_d[d]] = dgm[d] + (dn + du);
      } else {
        dg[di + sdir_d[d]] = dgp[d] + dn;
        dg[di - sdir_d[d]] = dgm[d] + dn;
      }
    }
  };

  // Symmetric multicolour sweeps.  dG (zero for the zero initial iterate) is kept current by
  // the updates themselves, so a colour phase is just the update of its nodes.  Where the
  // colour order turns (the last colour of a forward pass, the first of a backward pass) the
  // same colour would be updated twice in a row; the second update solves the same node
  // equations with the same neighbours, so it changes nothing but rounding and is left out:
  // the phases run the colours 0 1 .. NCOL-1 .. 1 0 1 .. with period 2 (NCOL - 1), sweeps
  // times and once more for the final colour 0.
  // The update runs on the active node slot's registers through one branch per slot where the
  // registers allow the copies (tiles without u, up to two nodes per thread or three in 2D);
  // the others select the slot's values into one copy, which keeps their occupancy.
  constexpr bool kBranch = !WU && (NPT <= 2 || (NPT == 3 && DIM == 2));
  const int period = 2 * (NCOL - 1);
  const int nphase = G.sweeps > 0 ? G.sweeps * period + 1 : 0;
  for (int ph = 0; ph < nphase; ++ph) {
    const int pm = ph % period;
    const int col = pm < NCOL ? pm : period - pm;
    // ---- update the nodes of this colour (a contiguous range of threads) -------------
    // A thread's nodes lie in different colour ranges (a range is shorter than the block),
    // so at most one of them is active here.
    int msel = -1;
#pragma unroll
    for (int m = 0; m < NPT; ++m)
      if (col_[m] == col) msel = m;
    if constexpr (kBranch) {
      // one copy of the update per node slot, each on that slot's registers directly; within
      // a wave the active slot is the same for all lanes except at the ends of a colour range
#pragma unroll
      for (int m = 0; m < NPT; ++m)
        if (msel == m) update_node(rr[m], ai[m], wq[m], invd[m], zd_[m] & 0xffff, zd_[m] >> 16, qc_[m], zcr_[m]);
    } else if (msel >= 0) {
      // one copy of the update on the active slot's values, selected into registers
      R rv[NFZ], av[9], wv[3], idv = invd[0], zcv = zcr_[0];
      int zd = zd_[0], q = qc_[0];
#pragma unroll
      for (int f = 0; f < NFZ; ++f) rv[f] = rr[0][f];
#pragma unroll
      for (int k = 0; k < 9; ++k) av[k] = ai[0][k];
#pragma unroll
      for (int e = 0; e < 3; ++e) wv[e] = wq[0][e];
#pragma unroll
      for (int m = 1; m < NPT; ++m) {
        const bool sel = (msel == m);
#pragma unroll
        for (int f = 0; f < NFZ; ++f) rv[f] = sel ? rr[m][f] : rv[f];
#pragma unroll
        for (int k = 0; k < 9; ++k) av[k] = sel ? ai[m][k] : av[k];
#pragma unroll
        for (int e = 0; e < 3; ++e) wv[e] = sel ? wq[m][e] : wv[e];
        idv = sel ? invd[m] : idv;
        zd = sel ? zd_[m] : zd;
        q = sel ? qc_[m] : q;
        zcv = sel ? zcr_[m] : zcv;
      }
      update_node(rv, av, wv, idv, zd & 0xffff, zd >> 16, q, zcv);
      if (!WU) {
#pragma unroll
        for (int m = 0; m < NPT; ++m) zcr_[m] = (msel == m) ? zcv : zcr_[m];
      }
    }
    __syncthreads();
  }
  if (!WU) {
    // the c iterate, held by the threads that own the nodes, goes to LDS in ext order (dG is
    // no longer read: the last phase ended with a barrier)
#pragma unroll
    for (int m = 0; m < NPT; ++m)
      if (col_[m] >= 0) dg[qc_[m]] = zcr_[m];
    __syncthreads();
  }
  if (G.mode != kRasLeft) {
    // the whole extended solution, to be summed by the gather kernel
    R* out = xs + (long long)t * NFZ * ne;
    for (int q = threadIdx.x; q < ne; q += TH) {
      const int a = q % G.ex, b = (q / G.ex) % G.ey, c = q / (G.ex * G.ey);
      const int zi = (a + ring) + sy * (b + ring) + ((DIM == 3) ? sz * (c + ring) : 0);
      out[q] = WU ? zs[zi] : dg[q];
#pragma unroll
      for (int f = 1; f < NFZ; ++f) out[f * ne + q] = zs[(f - ZP0) * zsz + zi];
    }
    return;
  }
  // restricted prolongation: write the owned nodes only (coalesced, row-major)
  for (int q = threadIdx.x; q < ne; q += TH) {
    const int a = q % G.ex, b = (q / G.ex) % G.ey, c = q / (G.ex * G.ey);
    if (a < G.ov || a >= G.ov + G.tx || b < G.ov || b >= G.ov + G.ty) continue;
    if (DIM == 3 && (c < G.ov || c >= G.ov + G.tz)) continue;
    const int gi = wrapg(ox + a, K.nx), gj = wrapg(oy + b, K.ny);
    const int gk = (DIM == 3) ? wrapg(oz + c, K.nz) : 0;
    const long long n = gi + (long long)K.nx * (gj + (long long)K.ny * gk);
    const int zi = (a + ring) + sy * (b + ring) + ((DIM == 3) ? sz * (c + ring) : 0);
    zg[n] = WU ? zs[zi] : dg[q];
#pragma unroll
    for (int f = 1; f < NFZ; ++f) zg[f * N + n] = zs[(f - ZP0) * zsz + zi];
  }
}

// z at every node = sum of the extended solutions of the tiles whose extended block contains
// it, tiles taken in a fixed order (at most two per direction: overlap <= tile / 2)
template <int DIM, int NFZ, typename R>
__global__ __launch_bounds__(256) void k_ras_gather(Consts K, Geo G, const R* __restrict__ xs, R* __restrict__ zg,
                                                    Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  xs = bat_at(xs, bi * bt.stride);
  zg = bat_at(zg, bi * bt.stride);
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= K.N) return;
  const int i = (int)(n % K.nx), j = (int)((n / K.nx) % K.ny), k = (int)(n / ((long long)K.nx * K.ny));
  const int ne = G.ex * G.ey * G.ez;
  const int ntz = (DIM == 3) ? K.nz / G.tz : 1;
  double acc[NFZ];
#pragma unroll
  for (int f = 0; f < NFZ; ++f) acc[f] = 0.0;
  // candidate tiles per direction: the owner and its two neighbours, each taken once (with
  // one or two tiles in a direction the neighbours coincide)
  for (int dk = (DIM == 3 ? -1 : 0); dk <= (DIM == 3 ? 1 : 0); ++dk) {
    if (DIM == 3 && ((dk == 1 && ntz <= 2) || (dk == -1 && ntz <= 1))) continue;
    const int tk = (DIM == 3) ? (k / G.tz + dk + ntz) % ntz : 0;
    const int lc = (DIM == 3) ? wrapg(k - (tk * G.tz - G.ov), K.nz) : 0;
    if (lc >= G.ez) continue;
    for (int dj = -1; dj <= 1; ++dj) {
      if ((dj == 1 && G.nty <= 2) || (dj == -1 && G.nty <= 1)) continue;
      const int tj = (j / G.ty + dj + G.nty) % G.nty;
      const int lb = wrapg(j - (tj * G.ty - G.ov), K.ny);
      if (lb >= G.ey) continue;
      for (int di = -1; di <= 1; ++di) {
        if ((di == 1 && G.ntx <= 2) || (di == -1 && G.ntx <= 1)) continue;
        const int ti = (i / G.tx + di + G.ntx) % G.ntx;
        const int la = wrapg(i - (ti * G.tx - G.ov), K.nx);
        if (la >= G.ex) continue;
        const long long t = ti + (long long)G.ntx * (tj + (long long)G.nty * tk);
        const R* src = xs + t * NFZ * ne + la + G.ex * (lb + G.ey * lc);
#pragma unroll
        for (int f = 0; f < NFZ; ++f) acc[f] += (double)src[(long long)f * ne];
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NFZ; ++f) zg[f * K.N + n] = (R)acc[f];
}

Geo make_geo(const Consts& K, const TileCfg& T) {
  Geo G;
  G.tx = T.tx;
  G.ty = T.ty;
  G.tz = (K.dim == 3) ? T.tz : 1;
  G.ov = T.ov;
  G.sweeps = T.sweeps;
  G.omega = T.omega;
  G.ex = T.tx + 2 * T.ov;
  G.ey = T.ty + 2 * T.ov;
  G.ez = (K.dim == 3) ? T.tz + 2 * T.ov : 1;
  const int ring = T.with_u ? 2 : 1;
  G.zx = G.ex + 2 * ring;
  G.zy = G.ey + 2 * ring;
  G.zz = (K.dim == 3) ? G.ez + 2 * ring : 1;
  G.dx = G.ex + 2;
  G.dy = G.ey + 2;
  G.dz = (K.dim == 3) ? G.ez + 2 : 1;
  G.ntx = K.nx / T.tx;
  G.nty = K.ny / T.ty;
  G.mode = T.mode;
  return G;
}

template <int DIM, bool WU, typename R, int TH>
void launch_npt(const Geo& G, const Consts& K, size_t lds, int ntiles, int npt, double dt, const R* B,
                const double* cn, const R* r, R* z, const int* perm, const R* pack, R* xs, hipStream_t s,
                const Bat& bt) {
  const dim3 grid = bat_grid(dim3(ntiles), bt);
#define PF_RAS_CASE(NPTV)                                                                             \
  case NPTV: {                                                                                        \
    allow_max_lds((const void*)k_ras<DIM, WU, NPTV, R, TH>); \
    hipLaunchKernelGGL((k_ras<DIM, WU, NPTV, R, TH>), grid, dim3(TH), lds, s, K, G, dt, B, cn, r, z, perm, pack, xs, bt); \
  } break;
  if constexpr (TH == kRasThreadsSmall) {
    if (npt == 4) {
      allow_max_lds((const void*)k_ras<DIM, WU, 4, R, TH>);
      hipLaunchKernelGGL((k_ras<DIM, WU, 4, R, TH>), grid, dim3(TH), lds, s, K, G, dt, B, cn, r, z, perm, pack,
                         xs, bt);
      return;
    }
  }
  switch (npt) {
    PF_RAS_CASE(1)
    PF_RAS_CASE(2)
    default:
      PF_RAS_CASE(3)
  }
#undef PF_RAS_CASE
}

template <int DIM, bool WU, typename R>
void launch_dim(const Consts& K, const Geo& G, size_t lds, int ntiles, int th, int npt, double dt,
                const R* B, const double* cn, const R* r, R* z, const int* perm, const R* pack, R* xs,
                hipStream_t s, const Bat& bt) {
  if (!WU && th == kRasThreadsSmall)
    launch_npt<DIM, false, R, kRasThreadsSmall>(G, K, lds, ntiles, npt, dt, B, cn, r, z, perm, pack, xs, s, bt);
  else
    launch_npt<DIM, WU, R, kRasThreadsMax>(G, K, lds, ntiles, npt, dt, B, cn, r, z, perm, pack, xs, s, bt);
  if (G.mode != kRasLeft) {
    constexpr int NFZ = WU ? 4 + DIM : 4;
    hipLaunchKernelGGL((k_ras_gather<DIM, NFZ, R>), bat_grid(dim3((unsigned)((K.N + 255) / 256)), bt), dim3(256), 0,
                       s, K, G, (const R*)xs, z, bt);
  }
}

// nodes of the extended tile per thread at th threads: up to four with 256 threads, three
// with 512; 0 beyond
int npt_for(const Geo& G, int th) {
  const int ne = G.ex * G.ey * G.ez;
  const int npt = (ne + th - 1) / th;
  return npt <= (th == kRasThreadsSmall ? 4 : 3) ? npt : 0;
}

// largest number of extended-tile nodes of one colour (a colour's nodes sit on consecutive
// threads, so that each thread has at most one active node per phase: at most th of them)
int max_colour_nodes(int dim, const Geo& G) {
  int cnt[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int c = 0; c < G.ez; ++c)
    for (int b = 0; b < G.ey; ++b)
      for (int a = 0; a < G.ex; ++a) ++cnt[(dim == 3) ? (a + 2 * b + 3 * c) % 7 : (a + 2 * b) % 5];
  int m = 0;
  for (int k = 0; k < 7; ++k) m = cnt[k] > m ? cnt[k] : m;
  return m;
}

}  // namespace

size_t ras_lds_bytes(const Consts& K, const TileCfg& T, size_t real_bytes) {
  const Geo G = make_geo(K, T);
  const int nzl = T.with_u ? 4 + K.dim : 3;  // LDS planes of the iterate
  const size_t ne = (size_t)G.ex * G.ey * G.ez;
  return real_bytes * ((size_t)nzl * G.zx * G.zy * G.zz + 2 * (size_t)G.dx * G.dy * G.dz + 4 * ne);
}

int ras_ext_nodes(const Consts& K, const TileCfg& T) {
  const Geo G = make_geo(K, T);
  return G.ex * G.ey * G.ez;
}

void ras_colour_order(const Consts& K, const TileCfg& T, int* perm) {
  const Geo G = make_geo(K, T);
  const int ncol = (K.dim == 3) ? 7 : 5;
  int pos = 0;
  for (int col = 0; col < ncol; ++col)
    for (int c = 0; c < G.ez; ++c)
      for (int b = 0; b < G.ey; ++b)
        for (int a = 0; a < G.ex; ++a) {
          const int ca = (K.dim == 3) ? (a + 2 * b + 3 * c) % 7 : (a + 2 * b) % 5;
          if (ca == col) perm[pos++] = a + G.ex * (b + G.ey * c);
        }
}

int ras_threads(const Consts& K, const TileCfg& T, size_t real_bytes, int* npt) {
  const Geo G = make_geo(K, T);
  const int ns = npt_for(G, kRasThreadsSmall);
  if (!T.with_u && ns > 0 && max_colour_nodes(K.dim, G) <= kRasThreadsSmall &&
      2 * ras_lds_bytes(K, T, real_bytes) <= 160 * 1024) {
    if (npt) *npt = ns;
    return kRasThreadsSmall;
  }
  const int nm = npt_for(G, kRasThreadsMax);
  if (nm > 0 && max_colour_nodes(K.dim, G) > kRasThreadsMax) return 0;
  if (npt) *npt = nm;
  return nm > 0 ? kRasThreadsMax : 0;
}

template <typename R>
void launch_ras(const Consts& K, const TileCfg& T, double dt, const R* B, const double* cn,
                const R* r, R* z, hipStream_t s, const Bat& bt) {
  const Geo G = make_geo(K, T);
  const int ntiles = G.ntx * G.nty * ((K.dim == 3) ? K.nz / T.tz : 1);
  const size_t lds = ras_lds_bytes(K, T, sizeof(R));
  int npt = 0;
  const int th = ras_threads(K, T, sizeof(R), &npt);
  R* xs = static_cast<R*>(T.scratch);
  const R* pk = static_cast<const R*>(T.pack);
  if (K.dim == 2) {
    if (T.with_u) launch_dim<2, true, R>(K, G, lds, ntiles, th, npt, dt, B, cn, r, z, T.perm, pk, xs, s, bt);
    else launch_dim<2, false, R>(K, G, lds, ntiles, th, npt, dt, B, cn, r, z, T.perm, pk, xs, s, bt);
  } else {
    if (T.with_u) launch_dim<3, true, R>(K, G, lds, ntiles, th, npt, dt, B, cn, r, z, T.perm, pk, xs, s, bt);
    else launch_dim<3, false, R>(K, G, lds, ntiles, th, npt, dt, B, cn, r, z, T.perm, pk, xs, s, bt);
  }
}

template <typename R>
void launch_ras_pack(const Consts& K, const TileCfg& T, double dt, const R* B, const double* cn, hipStream_t s,
                     const Bat& bt) {
  const Geo G = make_geo(K, T);
  const int ntiles = G.ntx * G.nty * ((K.dim == 3) ? K.nz / T.tz : 1);
  R* pk = static_cast<R*>(T.pack);
  const int* iperm = T.perm + G.ex * G.ey * G.ez;
  if (K.dim == 2)
    hipLaunchKernelGGL((k_ras_pack<2, R>), bat_grid(dim3(ntiles), bt), dim3(kPackThreads), 0, s, K, G, dt, B, cn,
                       iperm, pk, bt);
  else
    hipLaunchKernelGGL((k_ras_pack<3, R>), bat_grid(dim3(ntiles), bt), dim3(kPackThreads), 0, s, K, G, dt, B, cn,
                       iperm, pk, bt);
}
template void launch_ras_pack<double>(const Consts&, const TileCfg&, double, const double*, const double*,
                                      hipStream_t, const Bat&);
template void launch_ras_pack<float>(const Consts&, const TileCfg&, double, const float*, const double*,
                                     hipStream_t, const Bat&);

size_t ras_pack_values(const Consts& K, const TileCfg& T) {
  const Geo G = make_geo(K, T);
  const size_t ntiles = (size_t)G.ntx * G.nty * ((K.dim == 3) ? K.nz / T.tz : 1);
  return ntiles * kPackVals * (size_t)G.ex * G.ey * G.ez;
}
template void launch_ras<double>(const Consts&, const TileCfg&, double, const double*, const double*,
                                 const double*, double*, hipStream_t, const Bat&);
template void launch_ras<float>(const Consts&, const TileCfg&, double, const float*, const double*,
                                const float*, float*, hipStream_t, const Bat&);

}  // namespace pf
