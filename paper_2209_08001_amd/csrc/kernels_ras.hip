// Restricted additive Schwarz preconditioner with LDS-resident subdomains (Section 4).
//
// z = sum_t R_t^0' A_t^{-1} R_t^delta r: every workgroup owns one tile of T_x x T_y (x T_z)
// nodes, extends it by delta layers on every side (overlap), and solves the restriction
// A_t = J[ext, ext] of the Newton Jacobian to that extended block (zero Dirichlet exterior)
// approximately with symmetric multicolour block Gauss-Seidel sweeps; only the owned nodes
// are written back (the restricted prolongation R_t^0').
//
// The iterate of the whole extended tile lives in LDS with a zero ring two nodes wide (the
// Jacobian couples nodes up to distance 2: the 13-point diamond in 2D, 25 points in 3D).
// Colour (i + 2j) mod 5 (2D) or (i + 2j + 3k) mod 7 (3D) separates every pair of nodes
// inside one diamond, so all nodes of a colour update at once, exactly as sequential
// Gauss-Seidel would.  The per-node 4 x 4 chemical block B and the right-hand side stay in
// registers of the thread that owns the node.
//
// Tile operator, per node (the Jacobian of the residual, written in the kernels_phase notes):
//   dG    = B_c.z + kel z_c - (eps0/2) Ctr div_h z_u - (gamma_c/2) Lap_h z_c   on ext and its ring
//   (Az)_c = z_c/dt - div_h(M grad_h dG)
//   (Az)_e = z_e/dt + L_eta (B_e.z - (gamma_eta/2) Lap_h z_e)
//   (Az)_u = sum_J Dhat_J sigma_IJ(z_u, z_c)                      (only when with_u)
#include "pf_internal.h"

namespace pf {

namespace {

constexpr int kRasThreads = 512;

struct Geo {
  int ex, ey, ez;      // extended tile
  int zx, zy, zz;      // LDS iterate (ext + ring of 2; zz = 1 in 2D)
  int dx, dy, dz;      // dG / mobility arrays (ext + ring of 1; dz = 1 in 2D)
  int ntx, nty;        // tiles per direction
  int tx, ty, tz, ov;
  int sweeps;
};

template <int NF>
__device__ inline void solve_small(double (&D)[NF][NF], double (&x)[NF]) {
  // Gauss elimination with partial pivoting (NF <= 4)
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    int piv = k;
    double best = fabs(D[k][k]);
#pragma unroll
    for (int i = k + 1; i < NF; ++i) {
      if (fabs(D[i][k]) > best) {
        best = fabs(D[i][k]);
        piv = i;
      }
    }
    if (piv != k) {
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        const double t = D[k][j];
        D[k][j] = D[piv][j];
        D[piv][j] = t;
      }
      const double t = x[k];
      x[k] = x[piv];
      x[piv] = t;
    }
    const double inv = 1.0 / D[k][k];
#pragma unroll
    for (int i = k + 1; i < NF; ++i) {
      const double f = D[i][k] * inv;
#pragma unroll
      for (int j = k; j < NF; ++j) D[i][j] -= f * D[k][j];
      x[i] -= f * x[k];
    }
  }
#pragma unroll
  for (int k = NF - 1; k >= 0; --k) {
    double s = x[k];
#pragma unroll
    for (int j = k + 1; j < NF; ++j) s -= D[k][j] * x[j];
    x[k] = s / D[k][k];
  }
}

__device__ inline int wrapg(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

template <int DIM, bool WU, int NPT>
__global__ __launch_bounds__(kRasThreads) void k_ras(Consts K, Geo G, double dt,
                                                     const double* __restrict__ Bg,
                                                     const double* __restrict__ cn,
                                                     const double* __restrict__ rg,
                                                     double* __restrict__ zg) {
  constexpr int NFZ = WU ? 4 + DIM : 4;
  extern __shared__ double lds[];
  const int zsz = G.zx * G.zy * G.zz;
  const int dsz = G.dx * G.dy * G.dz;
  double* zs = lds;              // NFZ planes of zsz
  double* dg = zs + NFZ * zsz;   // dsz
  double* gg = dg + dsz;         // dsz: g = c^n (1 - c^n)

  const int t = blockIdx.x;
  const int tix = t % G.ntx, tiy = (t / G.ntx) % G.nty, tiz = t / (G.ntx * G.nty);
  const int ox = tix * G.tx - G.ov, oy = tiy * G.ty - G.ov, oz = (DIM == 3) ? tiz * G.tz - G.ov : 0;
  const long long N = K.N;
  const int sy = G.zx, sz = G.zx * G.zy;  // LDS strides of the iterate
  const int ty_ = G.dx, tz_ = G.dx * G.dy; // strides of dG / g
  const int ring = 2;

  for (int q = threadIdx.x; q < NFZ * zsz; q += kRasThreads) zs[q] = 0.0;
  for (int q = threadIdx.x; q < dsz; q += kRasThreads) {
    const int a = q % G.dx, b = (q / G.dx) % G.dy, c = q / (G.dx * G.dy);
    const int gi = wrapg(ox + a - 1, K.nx), gj = wrapg(oy + b - 1, K.ny);
    const int gk = (DIM == 3) ? wrapg(oz + c - 1, K.nz) : 0;
    const double v = cn[gi + (long long)K.nx * (gj + (long long)K.ny * gk)];
    gg[q] = v * (1.0 - v);
    dg[q] = 0.0;
  }

  // owned nodes: rhs and chemical block in registers
  const int ne = G.ex * G.ey * G.ez;
  double rr[NPT][NFZ];
  double bb[NPT][16];
  int zi_[NPT], di_[NPT], col_[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int q = threadIdx.x + m * kRasThreads;
    col_[m] = -1;
    zi_[m] = 0;
    di_[m] = 0;
    if (q < ne) {
      const int a = q % G.ex, b = (q / G.ex) % G.ey, c = q / (G.ex * G.ey);
      const int gi = wrapg(ox + a, K.nx), gj = wrapg(oy + b, K.ny);
      const int gk = (DIM == 3) ? wrapg(oz + c, K.nz) : 0;
      const long long n = gi + (long long)K.nx * (gj + (long long)K.ny * gk);
      for (int f = 0; f < NFZ; ++f) rr[m][f] = rg[f * N + n];
      for (int f = 0; f < 16; ++f) bb[m][f] = Bg[f * N + n];
      zi_[m] = (a + ring) + sy * (b + ring) + ((DIM == 3) ? sz * (c + ring) : 0);
      di_[m] = (a + 1) + ty_ * (b + 1) + ((DIM == 3) ? tz_ * (c + 1) : 0);
      col_[m] = (DIM == 3) ? (a + 2 * b + 3 * c) % 7 : (a + 2 * b) % 5;
    } else {
#pragma unroll
      for (int f = 0; f < NFZ; ++f) rr[m][f] = 0.0;
#pragma unroll
      for (int f = 0; f < 16; ++f) bb[m][f] = 0.0;
    }
  }
  __syncthreads();

  const int ncol = (DIM == 3) ? 7 : 5;
  const double idt = 1.0 / dt;
  const double lapc = -2.0 * DIM * K.ih2;
  const int sdir_z[3] = {1, sy, sz};
  const int sdir_d[3] = {1, ty_, tz_};
  const double a_u = -0.5 * K.eps0 * K.Ctr;  // coefficient of div_h z_u in dG
  bool first = true;

  for (int sw = 0; sw < G.sweeps; ++sw) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int cc = 0; cc < ncol; ++cc) {
        const int col = pass == 0 ? cc : ncol - 1 - cc;
        // ---- dG on ext (owned) and on the ring of width 1 ------------------------------
        if (!first) {
#pragma unroll
          for (int m = 0; m < NPT; ++m) {
            if (col_[m] < 0) continue;
            const int zi = zi_[m];
            double s = K.kel * zs[zi];
#pragma unroll
            for (int f = 0; f < 4; ++f) s += bb[m][f] * zs[f * zsz + zi];
            double l = lapc * zs[zi];
#pragma unroll
            for (int d = 0; d < DIM; ++d) l += (zs[zi + sdir_z[d]] + zs[zi - sdir_z[d]]) * K.ih2;
            s -= 0.5 * K.gamma_c * l;
            if (WU) {
              double dv = 0.0;
#pragma unroll
              for (int d = 0; d < DIM; ++d)
                dv += zs[(4 + d) * zsz + zi + sdir_z[d]] - zs[(4 + d) * zsz + zi - sdir_z[d]];
              s += a_u * dv * K.i2h;
            }
            dg[di_[m]] = s;
          }
          // ring positions (no chemical block there: the iterate is zero outside ext)
          for (int q = threadIdx.x; q < dsz; q += kRasThreads) {
            const int a = q % G.dx, b = (q / G.dx) % G.dy, c = q / (G.dx * G.dy);
            const bool inside = a >= 1 && a <= G.ex && b >= 1 && b <= G.ey &&
                                (DIM == 2 || (c >= 1 && c <= G.ez));
            if (inside) continue;
            const int zi = (a - 1 + ring) + sy * (b - 1 + ring) + ((DIM == 3) ? sz * (c - 1 + ring) : 0);
            double l = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) l += (zs[zi + sdir_z[d]] + zs[zi - sdir_z[d]]) * K.ih2;
            double s = -0.5 * K.gamma_c * l;
            if (WU) {
              double dv = 0.0;
#pragma unroll
              for (int d = 0; d < DIM; ++d)
                dv += zs[(4 + d) * zsz + zi + sdir_z[d]] - zs[(4 + d) * zsz + zi - sdir_z[d]];
              s += a_u * dv * K.i2h;
            }
            dg[q] = s;
          }
          __syncthreads();
        }
        first = false;
        // ---- update the nodes of this colour -------------------------------------------
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
          if (col_[m] != col) continue;
          const int zi = zi_[m], di = di_[m];
          double zv[NFZ];
#pragma unroll
          for (int f = 0; f < NFZ; ++f) zv[f] = zs[f * zsz + zi];
          double res[NFZ];
          // c row
          double sumM = 0.0, dM[3] = {0.0, 0.0, 0.0};
          double divm = 0.0;
          const double g0 = gg[di], dg0 = dg[di];
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            const double Mp = 0.5 * K.kappa * (g0 + gg[di + sdir_d[d]]);
            const double Mm = 0.5 * K.kappa * (g0 + gg[di - sdir_d[d]]);
            divm += Mp * (dg[di + sdir_d[d]] - dg0) - Mm * (dg0 - dg[di - sdir_d[d]]);
            sumM += Mp + Mm;
            dM[d] = Mm - Mp;
          }
          res[0] = rr[m][0] - (zv[0] * idt - divm * K.ih2);
          // eta rows
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            const int ze = (1 + e) * zsz + zi;
            double l = lapc * zs[ze];
#pragma unroll
            for (int d = 0; d < DIM; ++d) l += (zs[ze + sdir_z[d]] + zs[ze - sdir_z[d]]) * K.ih2;
            double s = -0.5 * K.gamma_eta * l;
#pragma unroll
            for (int f = 0; f < 4; ++f) s += bb[m][4 * (1 + e) + f] * zv[f];
            res[1 + e] = rr[m][1 + e] - (zv[1 + e] * idt + K.L_eta * s);
          }
          // u rows
          if (WU) {
#pragma unroll
            for (int I = 0; I < DIM; ++I) {
              double acc = 0.0;
#pragma unroll
              for (int J = 0; J < DIM; ++J) {
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                  const int pz = zi + sgn * sdir_z[J];
                  double sig;
                  if (I != J) {
                    sig = K.C44 * ((zs[(4 + J) * zsz + pz + sdir_z[I]] - zs[(4 + J) * zsz + pz - sdir_z[I]]) +
                                   (zs[(4 + I) * zsz + pz + sdir_z[J]] - zs[(4 + I) * zsz + pz - sdir_z[J]])) * K.i2h;
                  } else {
                    const double ec = K.eps0 * zs[pz];
                    sig = 0.0;
#pragma unroll
                    for (int L = 0; L < DIM; ++L) {
                      const double e = (zs[(4 + L) * zsz + pz + sdir_z[L]] - zs[(4 + L) * zsz + pz - sdir_z[L]]) * K.i2h - ec;
                      sig += (L == I ? K.C11 : K.C12) * e;
                    }
                  }
                  acc += sgn * sig;
                }
              }
              res[4 + I] = rr[m][4 + I] - acc * K.i2h;
            }
          }
          // diagonal block and its solve
          double Dw[4][4];
          const double sc = sumM * K.ih2;
          Dw[0][0] = idt + sc * (bb[m][0] + K.kel + K.gamma_c * DIM * K.ih2 + 0.5 * K.gamma_c * K.ih2);
          for (int q = 1; q < 4; ++q) Dw[0][q] = sc * bb[m][q];
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            Dw[1 + e][0] = K.L_eta * bb[m][4 * (1 + e)];
#pragma unroll
            for (int q = 1; q < 4; ++q)
              Dw[1 + e][q] = K.L_eta * bb[m][4 * (1 + e) + q] + ((q == 1 + e) ? idt + K.L_eta * K.gamma_eta * DIM * K.ih2 : 0.0);
          }
          double x[4] = {res[0], res[1], res[2], res[3]};
          double xu[3] = {0.0, 0.0, 0.0};
          if (WU) {
            const double duu = -(K.C11 + (DIM - 1) * K.C44) * 0.5 * K.ih2;
#pragma unroll
            for (int I = 0; I < DIM; ++I) {
              xu[I] = res[4 + I] / duu;
              x[0] -= (K.eps0 * K.Ctr * 0.25 * K.ih2 * K.ih) * dM[I] * xu[I];
            }
          }
          solve_small<4>(Dw, x);
#pragma unroll
          for (int f = 0; f < 4; ++f) zs[f * zsz + zi] = zv[f] + x[f];
          if (WU) {
#pragma unroll
            for (int I = 0; I < DIM; ++I) zs[(4 + I) * zsz + zi] = zv[4 + I] + xu[I];
          }
        }
        __syncthreads();
      }
    }
  }
  // restricted prolongation: write the owned nodes only
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    if (col_[m] < 0) continue;
    const int q = threadIdx.x + m * kRasThreads;
    const int a = q % G.ex, b = (q / G.ex) % G.ey, c = q / (G.ex * G.ey);
    if (a < G.ov || a >= G.ov + G.tx || b < G.ov || b >= G.ov + G.ty) continue;
    if (DIM == 3 && (c < G.ov || c >= G.ov + G.tz)) continue;
    const int gi = wrapg(ox + a, K.nx), gj = wrapg(oy + b, K.ny);
    const int gk = (DIM == 3) ? wrapg(oz + c, K.nz) : 0;
    const long long n = gi + (long long)K.nx * (gj + (long long)K.ny * gk);
    for (int f = 0; f < NFZ; ++f) zg[f * N + n] = zs[f * zsz + zi_[m]];
  }
}

Geo make_geo(const Consts& K, const TileCfg& T) {
  Geo G;
  G.tx = T.tx;
  G.ty = T.ty;
  G.tz = (K.dim == 3) ? T.tz : 1;
  G.ov = T.ov;
  G.sweeps = T.sweeps;
  G.ex = T.tx + 2 * T.ov;
  G.ey = T.ty + 2 * T.ov;
  G.ez = (K.dim == 3) ? T.tz + 2 * T.ov : 1;
  G.zx = G.ex + 4;
  G.zy = G.ey + 4;
  G.zz = (K.dim == 3) ? G.ez + 4 : 1;
  G.dx = G.ex + 2;
  G.dy = G.ey + 2;
  G.dz = (K.dim == 3) ? G.ez + 2 : 1;
  G.ntx = K.nx / T.tx;
  G.nty = K.ny / T.ty;
  return G;
}

template <int DIM, bool WU>
void launch_dim(const Consts& K, const Geo& G, size_t lds, int ntiles, int npt, double dt,
                const double* B, const double* cn, const double* r, double* z, hipStream_t s) {
#define PF_RAS_CASE(NPTV)                                                                          \
  case NPTV:                                                                                       \
    (void)hipFuncSetAttribute((const void*)k_ras<DIM, WU, NPTV>,                                      \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                    \
    hipLaunchKernelGGL((k_ras<DIM, WU, NPTV>), dim3(ntiles), dim3(kRasThreads), lds, s, K, G, dt, \
                       B, cn, r, z);                                                               \
    break;
  switch (npt) {
    PF_RAS_CASE(1)
    PF_RAS_CASE(2)
    PF_RAS_CASE(3)
    default:
      PF_RAS_CASE(4)
  }
#undef PF_RAS_CASE
}

}  // namespace

size_t ras_lds_bytes(const Consts& K, const TileCfg& T) {
  const Geo G = make_geo(K, T);
  const int nfz = T.with_u ? 4 + K.dim : 4;
  return sizeof(double) * ((size_t)nfz * G.zx * G.zy * G.zz + 2 * (size_t)G.dx * G.dy * G.dz);
}

// nodes of the extended tile per thread (1..4), 0 if the tile does not fit
int ras_npt(const Consts& K, const TileCfg& T) {
  const Geo G = make_geo(K, T);
  const int ne = G.ex * G.ey * G.ez;
  const int npt = (ne + kRasThreads - 1) / kRasThreads;
  return npt <= 4 ? npt : 0;
}

void launch_ras(const Consts& K, const TileCfg& T, double dt, const double* B, const double* cn,
                const double* r, double* z, hipStream_t s) {
  const Geo G = make_geo(K, T);
  const int ntiles = G.ntx * G.nty * ((K.dim == 3) ? K.nz / T.tz : 1);
  const size_t lds = ras_lds_bytes(K, T);
  const int npt = ras_npt(K, T);
  if (K.dim == 2) {
    if (T.with_u) launch_dim<2, true>(K, G, lds, ntiles, npt, dt, B, cn, r, z, s);
    else launch_dim<2, false>(K, G, lds, ntiles, npt, dt, B, cn, r, z, s);
  } else {
    if (T.with_u) launch_dim<3, true>(K, G, lds, ntiles, npt, dt, B, cn, r, z, s);
    else launch_dim<3, false>(K, G, lds, ntiles, npt, dt, B, cn, r, z, s);
  }
}

}  // namespace pf
