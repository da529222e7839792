// Stencil kernels of the NSOA-1 step: residual F, local linearisation, matrix-free J v, energy.
//
// Scheme (NSOA-1) of Section 3 in d dimensions (tensor-product operators on a periodic grid):
//   G_c   = G_chem,c(V^{n+1}, V^n) - eps0 sum_I sigma_bar_II - gamma_c Lap_h c_bar
//   G_eta = G_chem,eta_p(V^{n+1}, V^n)                     - gamma_eta Lap_h eta_bar_p
//   F_c   = (c^{n+1} - c^n)/dt - div_h(M grad_h G_c),  M_{i+1/2} = kappa (g_i + g_{i+1})/2,
//           g = c^n (1 - c^n)                     (face mobility at t_n, Section 3)
//   F_eta = (eta^{n+1} - eta^n)/dt + L_eta G_eta
//   F_u_I = sum_J Dhat_J sigma_IJ(u^{n+1}, c^{n+1})  (mechanicalequilibrium-dis)
// G_chem is the discrete variational derivative of the Appendix-A chemical energy:
// G^1 by product-rule quotients (Appendix B, generalised to eta_1..3) and G^{2,S} from the
// Taylor-stabilised quotient Psi_S of eq. (D2-1), evaluated in closed form:
//   Psi_S[a, b] = ln(ybar/(1-ybar)) + P(rho^2) - P(tau^2),  P(x) = sum_{j=1}^{S-1} x^j/(2j(2j+1)),
//   ybar = (a+b)/2, delta = (a-b)/2, rho = delta/(1-ybar), tau = delta/ybar
// (the odd Taylor terms Psi^(2j+1)(ybar) delta^(2j) / (2j+1)! summed by derivative order).
//
// Layout: SoA planes of N doubles, x fastest; fields c, eta_1..3, u_1..u_d.
#include "pf_internal.h"

namespace pf {

namespace {

constexpr int kBX = 64, kBY = 4;  // stencil launches: one wave along x, four rows

// ---------------------------------------------------------------------------------
// indexing
// ---------------------------------------------------------------------------------
struct Pt {
  int i, j, k;
};

// Periodic indices.  P2 (every side a power of two): a mask, exact for any offset.  Otherwise
// two selects, exact for a in [-n, 2n) (a grid point plus a stencil offset, or a block's halo
// on grids wider than the block), or the remainder for any a (FAR: halos of grids narrower
// than the block).  The stencil kernels are instantiated for both P2 values.
template <bool P2>
__device__ inline int wrap(int a, int n) {
  if (P2) return a & (n - 1);
  a += (a < 0) ? n : 0;
  a -= (a >= n) ? n : 0;
  return a;
}
__device__ inline int wrap_far(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}
template <bool P2, bool FAR>
__device__ inline int wrap_t(int a, int n) {
  return (FAR && !P2) ? wrap_far(a, n) : wrap<P2>(a, n);
}

template <bool P2>
__device__ inline long long at(const Consts& K, Pt p, int di, int dj, int dk) {
  const int i = wrap<P2>(p.i + di, K.nx), j = wrap<P2>(p.j + dj, K.ny), k = wrap<P2>(p.k + dk, K.nz);
  return (long long)i + (long long)K.nx * ((long long)j + (long long)K.ny * k);
}

template <bool P2>
__device__ inline long long at_dir(const Consts& K, Pt p, int dir, int s) {
  return at<P2>(K, p, dir == 0 ? s : 0, dir == 1 ? s : 0, dir == 2 ? s : 0);
}

__device__ inline Pt shift(Pt p, int dir, int s) {
  if (dir == 0) p.i += s;
  else if (dir == 1) p.j += s;
  else p.k += s;
  return p;
}

__device__ inline long long lin(const Consts& K, Pt p) {
  return (long long)p.i + (long long)K.nx * ((long long)p.j + (long long)K.ny * p.k);
}

// Block coordinates of a stencil launch, reordered for the 8 XCDs: workgroups go to the XCDs
// round-robin by linear id, so linear id b is given block b' = (b mod 8) * (nb / 8) + b / 8
// (when nb is a multiple of 8).  Each XCD then sweeps a contiguous band of rows and the halo
// lines shared by neighbouring blocks are fetched once into its own L2.  The instance of a
// lockstep batch is the slowest part of z; returns it.
__device__ inline int xcd_block(const Bat& bt, int& bx, int& by, int& bz) {
  const int gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const int nb = gx * gy * gz;
  int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
  bx = b % gx;
  by = (b / gx) % gy;
  const int zt = b / (gx * gy), nzl = gz / bt.count;
  bz = zt % nzl;
  return bt.map[zt / nzl];
}

__device__ inline Pt coords(const Consts& K, long long n) {
  Pt p;
  p.i = (int)(n % K.nx);
  const long long t = n / K.nx;
  p.j = (int)(t % K.ny);
  p.k = (int)(t / K.ny);
  return p;
}

// The stencil helpers read planes of element type T (double, or the float of a mixed-precision
// Krylov vector) and compute in double.

// 2*d+1 point Laplacian of one plane
template <bool P2, typename T>
__device__ inline double lap(const Consts& K, const T* __restrict__ f, Pt p, double fc) {
  double s = 0.0;
  for (int dir = 0; dir < K.dim; ++dir) s += (double)f[at_dir<P2>(K, p, dir, 1)] + (double)f[at_dir<P2>(K, p, dir, -1)];
  return (s - 2.0 * K.dim * fc) * K.ih2;
}

// Dhat_dir of one plane at p (p may be an unwrapped neighbour)
template <bool P2, typename T>
__device__ inline double dhat(const Consts& K, const T* __restrict__ f, Pt p, int dir) {
  return ((double)f[at_dir<P2>(K, p, dir, 1)] - (double)f[at_dir<P2>(K, p, dir, -1)]) * K.i2h;
}

// sigma_IJ at point p from displacement planes u (d planes) and composition c.
// xi = 1 includes the eigenstrain -eps0 (c - cbar0) delta_IJ; for a perturbation (J v) the
// composition enters as -eps0 dc (xi = 1, cref = 0).
template <bool P2, typename T>
__device__ inline double sigma(const Consts& K, const T* __restrict__ u, long long N,
                               const T* __restrict__ c, double cref, Pt p, int I, int J) {
  if (I != J) {
    return K.C44 * (dhat<P2>(K, u + (long long)J * N, p, I) + dhat<P2>(K, u + (long long)I * N, p, J));
  }
  const double ec = K.eps0 * ((double)c[at<P2>(K, p, 0, 0, 0)] - cref);
  double s = 0.0;
  for (int L = 0; L < K.dim; ++L) {
    const double e = dhat<P2>(K, u + (long long)L * N, p, L) - ec;
    s += (L == I ? K.C11 : K.C12) * e;
  }
  return s;
}

// sum_J Dhat_J sigma_IJ at p
template <bool P2, typename T>
__device__ inline double div_sigma(const Consts& K, const T* __restrict__ u, long long N,
                                   const T* __restrict__ c, double cref, Pt p, int I) {
  double s = 0.0;
  for (int J = 0; J < K.dim; ++J) {
    s += sigma<P2>(K, u, N, c, cref, shift(p, J, 1), I, J) - sigma<P2>(K, u, N, c, cref, shift(p, J, -1), I, J);
  }
  return s * K.i2h;
}

// ---------------------------------------------------------------------------------
// Taylor-stabilised quotient Psi_S[a, b] and its derivative in a
// ---------------------------------------------------------------------------------
template <bool D>
__device__ inline double psi_quot(const Consts& K, double a, double b, double& dq) {
  const double yb = 0.5 * (a + b), de = 0.5 * (a - b);
  const double iy = 1.0 / yb, iz = 1.0 / (1.0 - yb);
  const double rho = de * iz, tau = de * iy;
  const double x1 = rho * rho, x2 = tau * tau;
  double p1 = 0.0, p2 = 0.0, d1 = 0.0, d2 = 0.0;
  for (int j = K.S - 2; j >= 0; --j) {
    p1 = p1 * x1 + K.qs[j];
    p2 = p2 * x2 + K.qs[j];
    if (D) {
      d1 = d1 * x1 + K.qd[j];
      d2 = d2 * x2 + K.qd[j];
    }
  }
  if (D) dq = 0.5 * (iy + iz) + d1 * (rho * iz) * (1.0 + rho) - d2 * (tau * iy) * (1.0 - tau);
  return log(yb * iz) + x1 * p1 - x2 * p2;
}

// divided difference g[a, b] of g = sum_{m=1}^{deg} co[m] c^m and its derivative in a,
// via q_1 = 1, q_{m+1} = a q_m + b^m (expanded form: finite at a = b)
__device__ inline double poly_dd(const double* co, int deg, double a, double b, double& dval) {
  double q = 1.0, dq = 0.0, bm = b;
  double val = co[1];
  dval = 0.0;
  for (int m = 1; m < deg; ++m) {
    const double qn = a * q + bm;
    const double dqn = q + a * dq;
    q = qn;
    dq = dqn;
    bm *= b;
    val += co[m + 1] * q;
    dval += co[m + 1] * dq;
  }
  return val;
}

// eta_p appears in phi_k: phi_1 = 1 - (eta_1 + eta_2)/2, phi_2 = 1 - (eta_1 + eta_3)/2,
// phi_3 = 1 - (eta_2 + eta_3)/2  (Appendix A)
__device__ inline bool in_phi(int k, int p) {
  return (k == 0 && p < 2) || (k == 1 && p != 1) || (k == 2 && p > 0);
}

// Chemical discrete gradient (G_c, G_eta_1..3) and, if JAC, B = d G / d (c, eta_1..3)^{n+1}
// (row-major 4 x 4).
template <bool JAC>
__device__ inline void chem_dg(const Consts& K, double c1, const double* e1, double c0,
                               const double* e0, double& Gc, double* Ge, double* B) {
  double f1[3], f0[3];
  f1[0] = 1.0 - 0.5 * (e1[0] + e1[1]);
  f1[1] = 1.0 - 0.5 * (e1[0] + e1[2]);
  f1[2] = 1.0 - 0.5 * (e1[1] + e1[2]);
  f0[0] = 1.0 - 0.5 * (e0[0] + e0[1]);
  f0[1] = 1.0 - 0.5 * (e0[0] + e0[2]);
  f0[2] = 1.0 - 0.5 * (e0[1] + e0[2]);
  const double S2b = 0.5 * (f1[0] * f1[0] + f1[1] * f1[1] + f1[2] * f1[2] + f0[0] * f0[0] +
                            f0[1] * f0[1] + f0[2] * f0[2]);
  const double P3b = 0.5 * (f1[0] * f1[1] * f1[2] + f0[0] * f0[1] * f0[2]);
  const double Aco[4] = {0.0, 0.0, K.A2, K.A3};
  const double Bco[4] = {0.0, 0.0, 0.0, K.B3};
  double dp, dA, dB;
  const double pq = poly_dd(K.pc, 5, c1, c0, dp);
  const double Aq = poly_dd(Aco, 3, c1, c0, dA);
  const double Bq = poly_dd(Bco, 3, c1, c0, dB);
  const double A1 = (K.A2 + K.A3 * c1) * c1 * c1, A0 = (K.A2 + K.A3 * c0) * c0 * c0;
  const double Ab = 0.5 * (A1 + A0), Bb = 0.5 * K.B3 * (c1 * c1 * c1 + c0 * c0 * c0);
  // G^1: product-rule quotients
  Gc = pq + S2b * Aq + P3b * Bq;
  double T[3], Gphi[3];
  for (int k = 0; k < 3; ++k) {
    const int a = (k == 0) ? 1 : 0, b = (k == 2) ? 1 : 2;
    T[k] = (f0[a] * f0[b] + f1[a] * f1[b]) * (1.0 / 3.0) + (f0[a] * f1[b] + f1[a] * f0[b]) * (1.0 / 6.0);
    Gphi[k] = Ab * (f1[k] + f0[k]) + Bb * T[k];
  }
  for (int p = 0; p < 3; ++p) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k)
      if (in_phi(k, p)) s += Gphi[k];
    Ge[p] = -0.5 * s;
  }
  // G^{2,S}: y_i = c eta_i, eta_4 = 4 - eta_1 - eta_2 - eta_3
  double y1[4], y0[4], eb[4], Q[4], dQ[4];
  const double e14 = 4.0 - e1[0] - e1[1] - e1[2], e04 = 4.0 - e0[0] - e0[1] - e0[2];
  for (int i = 0; i < 4; ++i) {
    const double a1 = (i < 3) ? e1[i] : e14, a0 = (i < 3) ? e0[i] : e04;
    y1[i] = c1 * a1;
    y0[i] = c0 * a0;
    eb[i] = 0.5 * (a1 + a0);
    Q[i] = psi_quot<JAC>(K, y1[i], y0[i], dQ[i]);
  }
  double dQc = 0.0;
  const double Qc = (K.w_c != 0.0) ? psi_quot<JAC>(K, c1, c0, dQc) : 0.0;
  const double cb = 0.5 * (c1 + c0);
  Gc += K.theta * (K.w_c * Qc + 0.25 * (eb[0] * Q[0] + eb[1] * Q[1] + eb[2] * Q[2] + eb[3] * Q[3]));
  for (int p = 0; p < 3; ++p) Ge[p] += 0.25 * K.theta * cb * (Q[p] - Q[3]);

  if (JAC) {
    const double a1[4] = {e1[0], e1[1], e1[2], e14};
    // row c
    B[0] = dp + S2b * dA + P3b * dB +
           K.theta * (K.w_c * dQc + 0.25 * (eb[0] * dQ[0] * a1[0] + eb[1] * dQ[1] * a1[1] +
                                            eb[2] * dQ[2] * a1[2] + eb[3] * dQ[3] * a1[3]));
    for (int p = 0; p < 3; ++p) {
      double dS2 = 0.0, dP3 = 0.0;
      for (int k = 0; k < 3; ++k) {
        if (!in_phi(k, p)) continue;
        const int a = (k == 0) ? 1 : 0, b = (k == 2) ? 1 : 2;
        dS2 += -f1[k];               // d(phi_k^2)/d eta_p /2 ... times 1/2 from the average: see below
        dP3 += -0.5 * f1[a] * f1[b];
      }
      // S2b = (S2^1 + S2^0)/2: d S2b/d eta_p = (1/2) sum_k 2 phi_k^1 (-1/2) = -(1/2) sum_k phi_k^1
      // P3b: d P3b / d eta_p = (1/2) sum_k (-1/2) prod_{l != k} phi_l^1
      B[1 + p] = 0.5 * dS2 * Aq + 0.5 * dP3 * Bq +
                 0.25 * K.theta * (0.5 * Q[p] + eb[p] * dQ[p] * c1 - 0.5 * Q[3] - eb[3] * dQ[3] * c1);
    }
    // rows eta_p
    const double dA1 = (2.0 * K.A2 + 3.0 * K.A3 * c1) * c1;  // A'(c^{n+1})
    const double dB1 = 3.0 * K.B3 * c1 * c1;                  // B'(c^{n+1})
    for (int p = 0; p < 3; ++p) {
      double sc = 0.0;
      for (int k = 0; k < 3; ++k)
        if (in_phi(k, p)) sc += 0.5 * dA1 * (f1[k] + f0[k]) + 0.5 * dB1 * T[k];
      B[4 * (1 + p)] = -0.5 * sc + 0.25 * K.theta * (0.5 * (Q[p] - Q[3]) + cb * (dQ[p] * a1[p] - dQ[3] * e14));
      for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
          if (!in_phi(k, p)) continue;
          const int a = (k == 0) ? 1 : 0, b = (k == 2) ? 1 : 2;
          // d phi_k / d eta_q = -1/2 if eta_q in phi_k
          double dT = 0.0;
          if (in_phi(a, q)) dT += -0.5 * (f1[b] * (1.0 / 3.0) + f0[b] * (1.0 / 6.0));
          if (in_phi(b, q)) dT += -0.5 * (f1[a] * (1.0 / 3.0) + f0[a] * (1.0 / 6.0));
          s += Ab * (in_phi(k, q) ? -0.5 : 0.0) + Bb * dT;
        }
        B[4 * (1 + p) + 1 + q] = -0.5 * s + 0.25 * K.theta * cb * ((p == q ? dQ[p] * c1 : 0.0) + dQ[3] * c1);
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// residual
// ---------------------------------------------------------------------------------
// pass 1: G_c, G_eta (4 planes) and F_u
template <bool P2>
__global__ __launch_bounds__(kBX* kBY) void k_residual_g(Consts K, const double* __restrict__ X,
                                                         const double* __restrict__ Xn,
                                                         double* __restrict__ G4,
                                                         double* __restrict__ F, Bat bt) {
  int bx, by, bz;
  const int bi = xcd_block(bt, bx, by, bz);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    X = bat_at(X, bo);
    Xn = bat_at(Xn, bo);
    G4 = bat_at(G4, bo);
    F = bat_at(F, bo);
  }
  const double cb = bt.cb[bi];
  Pt p{bx * kBX + (int)threadIdx.x, by * kBY + (int)threadIdx.y, bz};
  if (p.i >= K.nx || p.j >= K.ny) return;
  const long long N = K.N, n = lin(K, p);
  const double c1 = X[n], c0 = Xn[n];
  double e1[3], e0[3], Gc, Ge[3];
  for (int q = 0; q < 3; ++q) {
    e1[q] = X[(1 + q) * N + n];
    e0[q] = Xn[(1 + q) * N + n];
  }
  chem_dg<false>(K, c1, e1, c0, e0, Gc, Ge, nullptr);
  // elastic part of G_c: -eps0 * (sum_I sigma_II^{n+1} + sum_I sigma_II^n) / 2
  if (K.elastic) {
    double div1 = 0.0, div0 = 0.0;
    for (int I = 0; I < K.dim; ++I) {
      div1 += dhat<P2>(K, X + (4 + I) * N, p, I);
      div0 += dhat<P2>(K, Xn + (4 + I) * N, p, I);
    }
    const double tr1 = K.Ctr * (div1 - K.dim * K.eps0 * (c1 - cb));
    const double tr0 = K.Ctr * (div0 - K.dim * K.eps0 * (c0 - cb));
    Gc -= K.eps0 * 0.5 * (tr1 + tr0);
  }
  Gc -= K.gamma_c * 0.5 * (lap<P2>(K, X, p, c1) + lap<P2>(K, Xn, p, c0));
  G4[n] = Gc;
  for (int q = 0; q < 3; ++q) {
    Ge[q] -= K.gamma_eta * 0.5 * (lap<P2>(K, X + (1 + q) * N, p, e1[q]) + lap<P2>(K, Xn + (1 + q) * N, p, e0[q]));
    G4[(1 + q) * N + n] = Ge[q];
  }
  for (int I = 0; I < K.dim; ++I) {
    F[(4 + I) * N + n] = K.elastic ? div_sigma<P2>(K, X + 4 * N, N, X, cb, p, I) : X[(4 + I) * N + n];
  }
}

__device__ inline double block_sum(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += lds[w];
  return r;
}

// div_h (M grad_h g) at p with face mobilities from g_n = c^n (1 - c^n)
template <bool P2>
__device__ inline double div_M_grad(const Consts& K, const double* __restrict__ g,
                                    const double* __restrict__ cn, Pt p, long long n) {
  const double gc = g[n];
  const double mc = cn[n] * (1.0 - cn[n]);
  double s = 0.0;
  for (int dir = 0; dir < K.dim; ++dir) {
    const long long np = at_dir<P2>(K, p, dir, 1), nm = at_dir<P2>(K, p, dir, -1);
    const double Mp = 0.5 * K.kappa * (mc + cn[np] * (1.0 - cn[np]));
    const double Mm = 0.5 * K.kappa * (mc + cn[nm] * (1.0 - cn[nm]));
    s += Mp * (g[np] - gc) - Mm * (gc - g[nm]);
  }
  return s * K.ih2;
}

// pass 2: F_c, F_eta; partial[0] = ||F||^2, partial[1] = number of nodes outside the log domain
template <bool P2>
__global__ __launch_bounds__(256) void k_residual_f(Consts K, double dt, const double* __restrict__ X,
                                                    const double* __restrict__ Xn,
                                                    const double* __restrict__ G4,
                                                    double* __restrict__ F,
                                                    double* __restrict__ partial, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    X = bat_at(X, bo);
    Xn = bat_at(Xn, bo);
    G4 = bat_at(G4, bo);
    F = bat_at(F, bo);
    partial = bat_at(partial, bo);
  }
  dt = bat_s(bt, bi, dt);
  __shared__ double lds[4];
  const long long N = K.N;
  const double idt = 1.0 / dt;
  double nrm = 0.0, bad = 0.0;
  for (long long n = (long long)blockIdx.x * 256 + threadIdx.x; n < N; n += (long long)gridDim.x * 256) {
    const Pt p = coords(K, n);
    const double c1 = X[n];
    const double fc = (c1 - Xn[n]) * idt - div_M_grad<P2>(K, G4, Xn, p, n);
    F[n] = fc;
    nrm += fc * fc;
    bool ok = (c1 > 0.0 && c1 < 1.0);
    double esum = 0.0;
    for (int q = 0; q < 3; ++q) {
      const double e1 = X[(1 + q) * N + n];
      const double fe = (e1 - Xn[(1 + q) * N + n]) * idt + K.L_eta * G4[(1 + q) * N + n];
      F[(1 + q) * N + n] = fe;
      nrm += fe * fe;
      esum += e1;
      const double y = c1 * e1;
      ok = ok && (y > 0.0 && y < 1.0);
    }
    const double y4 = c1 * (4.0 - esum);
    ok = ok && (y4 > 0.0 && y4 < 1.0);
    for (int I = 0; I < K.dim; ++I) {
      const double fu = F[(4 + I) * N + n];
      nrm += fu * fu;
    }
    bad += ok ? 0.0 : 1.0;
  }
  const double s0 = block_sum(nrm, lds);
  const double s1 = block_sum(bad, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s0;
    partial[kRedBlocks + blockIdx.x] = s1;
  }
}

// ---------------------------------------------------------------------------------
// linearisation: B = d G_chem / d V^{n+1}, 16 planes (row-major 4 x 4 per node)
// ---------------------------------------------------------------------------------
// B: the 16 block planes in double; Bf (optional): the same rounded to float, for a
// mixed-precision preconditioner
__global__ __launch_bounds__(256) void k_linearise(Consts K, const double* __restrict__ X,
                                                   const double* __restrict__ Xn,
                                                   double* __restrict__ B, float* __restrict__ Bf, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    X = bat_at(X, bo);
    Xn = bat_at(Xn, bo);
    B = bat_at(B, bo);
    Bf = bat_at(Bf, bo);
  }
  const long long N = K.N;
  for (long long n = (long long)blockIdx.x * 256 + threadIdx.x; n < N; n += (long long)gridDim.x * 256) {
    double e1[3], e0[3], Ge[3], Gc, b[16];
    for (int q = 0; q < 3; ++q) {
      e1[q] = X[(1 + q) * N + n];
      e0[q] = Xn[(1 + q) * N + n];
    }
    chem_dg<true>(K, X[n], e1, Xn[n], e0, Gc, Ge, b);
    for (int q = 0; q < 16; ++q) B[q * N + n] = b[q];
    if (Bf)
      for (int q = 0; q < 16; ++q) Bf[q * N + n] = (float)b[q];
  }
}

// ---------------------------------------------------------------------------------
// matrix-free Jacobian-vector product
//   dG_c   = B_c. v + kel v_c - (eps0/2) Ctr div_h v_u - (gamma_c/2) Lap_h v_c
//   (Jv)_c = v_c/dt - div_h(M grad_h dG_c)
//   (Jv)_e = v_e/dt + L_eta (B_e. v - (gamma_eta/2) Lap_h v_e)
//   (Jv)_u = sum_J Dhat_J sigma_IJ(v_u, v_c)   (composition enters through -eps0 v_c)
// ---------------------------------------------------------------------------------
// J v in 2D, one pass: a block of kBX x kJY2 nodes stages v in LDS, computes dG on the block
// and a halo of one node into LDS, and forms the c, eta and u rows from LDS.  v has element
// type Tv (double, or float for a mixed-precision Krylov vector); the arithmetic and w are
// double.
constexpr int kJY2 = 8;
template <typename Tv, bool P2, bool FAR>
__global__ __launch_bounds__(kBX* kJY2) void k_jv2(Consts K, double dt, const double* __restrict__ B,
                                                   const double* __restrict__ cn, const Tv* __restrict__ v,
                                                   double* __restrict__ w, Bat bt) {
  // v (all six fields, as double) with a halo of 2 (sigma of the u rows reaches distance 2),
  // g = c^n (1 - c^n) and dG with a halo of 1; every stencil below reads LDS, only B comes
  // from global memory
  constexpr int SX = kBX + 4, SY = kJY2 + 4, SP = SX * SY;
  constexpr int HX = kBX + 2, HY = kJY2 + 2, HP = HX * HY;
  __shared__ double sv[6 * SP];
  __shared__ double sg[HP], sdg[HP];
  int bx, by, bz;
  const int bi = xcd_block(bt, bx, by, bz);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    B = bat_at(B, bo);
    cn = bat_at(cn, bo);
    v = bat_at(v, bo);
    w = bat_at(w, bo);
  }
  dt = bat_s(bt, bi, dt);
  const int i0 = bx * kBX, j0 = by * kJY2;
  const int tid = threadIdx.x + kBX * threadIdx.y;
  const long long N = K.N;
  for (int q = tid; q < 6 * SP; q += kBX * kJY2) {
    const int f = q / SP, r = q - f * SP, a = r % SX, b = r / SX;
    sv[q] = (double)v[f * N + wrap_t<P2, FAR>(i0 + a - 2, K.nx) + (long long)K.nx * wrap_t<P2, FAR>(j0 + b - 2, K.ny)];
  }
  for (int q = tid; q < HP; q += kBX * kJY2) {
    const int a = q % HX, b = q / HX;
    const double c = cn[wrap_t<P2, FAR>(i0 + a - 1, K.nx) + (long long)K.nx * wrap_t<P2, FAR>(j0 + b - 1, K.ny)];
    sg[q] = c * (1.0 - c);
  }
  __syncthreads();
  const int st[2] = {1, SX};
  auto lap_s = [&](const double* F, int ci, double fc) {
    double s = 0.0;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) s += F[ci + st[dir]] + F[ci - st[dir]];
    return (s - 4.0 * fc) * K.ih2;
  };
  auto dhat_s = [&](const double* F, int ci, int dir) { return (F[ci + st[dir]] - F[ci - st[dir]]) * K.i2h; };
  const double* su = sv + 4 * SP;
  // sigma_IJ of u with the eigenstrain of v_c (reference 0), at LDS position ci
  auto sigma_s = [&](int ci, int I, int J) {
    if (I != J) return K.C44 * (dhat_s(su + J * SP, ci, I) + dhat_s(su + I * SP, ci, J));
    const double ec = K.eps0 * (sv[ci] - 0.0);
    double s = 0.0;
#pragma unroll
    for (int L = 0; L < 2; ++L) s += (L == I ? K.C11 : K.C12) * (dhat_s(su + L * SP, ci, L) - ec);
    return s;
  };
  // dG on the block and its halo of 1 (halo point (a, b) sits at v position (a + 1, b + 1))
  for (int q = tid; q < HP; q += kBX * kJY2) {
    const int a = q % HX, b = q / HX, ci = (a + 1) + SX * (b + 1);
    const long long n = wrap_t<P2, FAR>(i0 + a - 1, K.nx) + (long long)K.nx * wrap_t<P2, FAR>(j0 + b - 1, K.ny);
    double vv[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) vv[f] = sv[f * SP + ci];
    double g = K.kel * vv[0] - 0.5 * K.gamma_c * lap_s(sv, ci, vv[0]);
#pragma unroll
    for (int f = 0; f < 4; ++f) g += B[f * N + n] * vv[f];
    if (K.elastic) {
      double div = 0.0;
#pragma unroll
      for (int I = 0; I < 2; ++I) div += dhat_s(su + I * SP, ci, I);
      g += -0.5 * K.eps0 * K.Ctr * div;
    }
    sdg[q] = g;
  }
  __syncthreads();
  const int pi = i0 + (int)threadIdx.x, pj = j0 + (int)threadIdx.y;
  if (pi >= K.nx || pj >= K.ny) return;
  const long long n = pi + (long long)K.nx * pj;
  const int ci = (threadIdx.x + 2) + SX * (threadIdx.y + 2);
  const int hq = (threadIdx.x + 1) + HX * (threadIdx.y + 1);
  const int hs[2] = {1, HX};
  const double idt = 1.0 / dt;
  {
    // c row: v_c / dt - div_h(M grad_h dG), face mobility M = kappa/2 (g_i + g_j)
    const double mc = sg[hq], g0 = sdg[hq];
    double s = 0.0;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const double Mp = 0.5 * K.kappa * (mc + sg[hq + hs[dir]]);
      const double Mm = 0.5 * K.kappa * (mc + sg[hq - hs[dir]]);
      s += Mp * (sdg[hq + hs[dir]] - g0) - Mm * (g0 - sdg[hq - hs[dir]]);
    }
    w[n] = sv[ci] * idt - s * K.ih2;
  }
  double vv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) vv[q] = sv[q * SP + ci];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    double s = -0.5 * K.gamma_eta * lap_s(sv + (1 + e) * SP, ci, vv[1 + e]);
#pragma unroll
    for (int q = 0; q < 4; ++q) s += B[(4 * (1 + e) + q) * N + n] * vv[q];
    w[(1 + e) * N + n] = vv[1 + e] * idt + K.L_eta * s;
  }
#pragma unroll
  for (int I = 0; I < 2; ++I) {
    double d = 0.0;
    if (K.elastic) {
#pragma unroll
      for (int J = 0; J < 2; ++J) d += sigma_s(ci + st[J], I, J) - sigma_s(ci - st[J], I, J);
    }
    w[(4 + I) * N + n] = K.elastic ? d * K.i2h : su[I * SP + ci];
  }
}

// J v in 3D in two passes over blocks of kBX x kJY3 columns marching through a chunk of planes.
// Each thread keeps its column's values at z - 1, z and z + 1 in registers; the x and y
// neighbours come from the current plane, staged in LDS with a ring of one node (the in-plane
// stencils are five-point crosses, so the ring's corners are never read).
//   pass A (k_jv3_dg):   dG of the c row and the stress sigma_IJ(v_u, v_c) at every node, into
//                        seven scratch planes: dG, s_xx, s_yy, s_zz, s_xy, s_xz, s_yz;
//   pass B (k_jv3_rows): the c row from dG and g = c^n (1 - c^n), the eta rows, and the u rows
//                        as sum_J Dhat_J sigma_IJ of the stored stress.
// Each pass reads every input plane once (plus the ring, shared with the neighbouring blocks
// through L2, and two planes per chunk in z), so neither re-reads the 3 x 3 x 3 neighbourhood
// the single-pass stencil needs for sigma at distance two.
constexpr int kJY3 = 4;   // block rows
constexpr int kJZ3 = 8;   // planes per chunk
constexpr int kRX3 = kBX + 2, kRP3 = kRX3 * (kJY3 + 2);
constexpr int kRing3 = 2 * kBX + 2 * kJY3;

// ring slot r of the staged plane: its offset (a, b) from the block origin and LDS index
__device__ inline int ring_slot(int r, int& a, int& b) {
  if (r < kBX) {
    a = r;
    b = -1;
  } else if (r < 2 * kBX) {
    a = r - kBX;
    b = kJY3;
  } else if (r < 2 * kBX + kJY3) {
    a = -1;
    b = r - 2 * kBX;
  } else {
    a = kBX;
    b = r - 2 * kBX - kJY3;
  }
  return (a + 1) + kRX3 * (b + 1);
}

// the column of a thread and, for the first kRing3 threads, of a ring slot (wrapped: threads
// outside a ragged grid stage the periodic image their neighbours read)
struct Cols3 {
  long long col, rcol;
  int slot, rslot;
};
template <bool P2, bool FAR>
__device__ inline Cols3 cols3(const Consts& K, int i0, int j0) {
  Cols3 c;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + kBX * ty;
  c.col = wrap_t<P2, FAR>(i0 + tx, K.nx) + (long long)K.nx * wrap_t<P2, FAR>(j0 + ty, K.ny);
  c.slot = (tx + 1) + kRX3 * (ty + 1);
  c.rslot = -1;
  c.rcol = 0;
  if (tid < kRing3) {
    int a, b;
    c.rslot = ring_slot(tid, a, b);
    c.rcol = wrap_t<P2, FAR>(i0 + a, K.nx) + (long long)K.nx * wrap_t<P2, FAR>(j0 + b, K.ny);
  }
  return c;
}

template <typename Tv, bool P2, bool FAR>
__global__ __launch_bounds__(kBX* kJY3) void k_jv3_dg(Consts K, const double* __restrict__ B,
                                                      const Tv* __restrict__ v, double* __restrict__ scr,
                                                      int zc, Bat bt) {
  // staged fields: v_c, u_x, u_y, u_z (field f of v at plane offset fo[f] * N)
  __shared__ Tv sp[4 * kRP3];
  int bx, by, bz;
  const int bi = xcd_block(bt, bx, by, bz);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    B = bat_at(B, bo);
    v = bat_at(v, bo);
    scr = bat_at(scr, bo);
  }
  const long long N = K.N, NP = (long long)K.nx * K.ny;
  const int i0 = bx * kBX, j0 = by * kJY3, z0 = bz * zc;
  const int z1 = (z0 + zc < K.nz) ? z0 + zc : K.nz;
  const Cols3 c = cols3<P2, FAR>(K, i0, j0);
  const bool live = (i0 + (int)threadIdx.x < K.nx) && (j0 + (int)threadIdx.y < K.ny);
  const int fo[4] = {0, 4, 5, 6};
  auto plane = [&](int z) { return NP * wrap_t<P2, FAR>(z, K.nz); };
  double prv[4], cur[4], nxt[4];
  {
    const long long pm = plane(z0 - 1) + c.col, p0 = plane(z0) + c.col;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      prv[f] = (double)v[fo[f] * N + pm];
      cur[f] = (double)v[fo[f] * N + p0];
    }
  }
  for (int z = z0; z < z1; ++z) {
    const long long pz = plane(z), n = pz + c.col, np = plane(z + 1) + c.col;
#pragma unroll
    for (int f = 0; f < 4; ++f) nxt[f] = (double)v[fo[f] * N + np];
    Tv ring[4];
    if (c.rslot >= 0) {
#pragma unroll
      for (int f = 0; f < 4; ++f) ring[f] = v[fo[f] * N + pz + c.rcol];
    }
    double ve[3], bc[4];
#pragma unroll
    for (int e = 0; e < 3; ++e) ve[e] = (double)v[(1 + e) * N + n];
#pragma unroll
    for (int f = 0; f < 4; ++f) bc[f] = B[f * N + n];
    __syncthreads();  // every thread is done reading the previous plane
#pragma unroll
    for (int f = 0; f < 4; ++f) sp[f * kRP3 + c.slot] = (Tv)cur[f];
    if (c.rslot >= 0) {
#pragma unroll
      for (int f = 0; f < 4; ++f) sp[f * kRP3 + c.rslot] = ring[f];
    }
    __syncthreads();
    if (live) {
      const int q = c.slot;
      // Dhat_K u_L at the node: du[K][L]
      double du[3][3];
#pragma unroll
      for (int L = 0; L < 3; ++L) {
        const Tv* s = sp + (1 + L) * kRP3;
        du[0][L] = ((double)s[q + 1] - (double)s[q - 1]) * K.i2h;
        du[1][L] = ((double)s[q + kRX3] - (double)s[q - kRX3]) * K.i2h;
        du[2][L] = (nxt[1 + L] - prv[1 + L]) * K.i2h;
      }
      const double vc = cur[0];
      double lp = 0.0;
      lp += (double)sp[q + 1] + (double)sp[q - 1];
      lp += (double)sp[q + kRX3] + (double)sp[q - kRX3];
      lp += nxt[0] + prv[0];
      lp = (lp - 6.0 * vc) * K.ih2;
      double g = K.kel * vc - 0.5 * K.gamma_c * lp;
      g += bc[0] * vc;
#pragma unroll
      for (int e = 0; e < 3; ++e) g += bc[1 + e] * ve[e];
      if (K.elastic) {
        g += -0.5 * K.eps0 * K.Ctr * (du[0][0] + du[1][1] + du[2][2]);
        const double ec = K.eps0 * vc;
        double sd[3];
#pragma unroll
        for (int I = 0; I < 3; ++I) {
          double s = 0.0;
#pragma unroll
          for (int L = 0; L < 3; ++L) s += (L == I ? K.C11 : K.C12) * (du[L][L] - ec);
          sd[I] = s;
        }
        scr[1 * N + n] = sd[0];
        scr[2 * N + n] = sd[1];
        scr[3 * N + n] = sd[2];
        scr[4 * N + n] = K.C44 * (du[0][1] + du[1][0]);
        scr[5 * N + n] = K.C44 * (du[0][2] + du[2][0]);
        scr[6 * N + n] = K.C44 * (du[1][2] + du[2][1]);
      }
      scr[n] = g;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      prv[f] = cur[f];
      cur[f] = nxt[f];
    }
  }
}

template <typename Tv, bool P2, bool FAR>
__global__ __launch_bounds__(kBX* kJY3) void k_jv3_rows(Consts K, double dt, const double* __restrict__ B,
                                                        const double* __restrict__ cn,
                                                        const Tv* __restrict__ v,
                                                        const double* __restrict__ scr,
                                                        double* __restrict__ w, int zc, Bat bt) {
  // staged fields: 0 dG, 1 g, 2..4 v_eta, 5 s_xx, 6 s_yy, 7 s_xy, 8 s_xz, 9 s_yz
  // z-queued fields (registers): 0 dG, 1 g, 2..4 v_eta, 5 s_xz, 6 s_yz, 7 s_zz
  __shared__ double sp[10 * kRP3];
  int bx, by, bz;
  const int bi = xcd_block(bt, bx, by, bz);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    B = bat_at(B, bo);
    cn = bat_at(cn, bo);
    v = bat_at(v, bo);
    scr = bat_at(scr, bo);
    w = bat_at(w, bo);
  }
  dt = bat_s(bt, bi, dt);
  const long long N = K.N, NP = (long long)K.nx * K.ny;
  const int i0 = bx * kBX, j0 = by * kJY3, z0 = bz * zc;
  const int z1 = (z0 + zc < K.nz) ? z0 + zc : K.nz;
  const Cols3 c = cols3<P2, FAR>(K, i0, j0);
  const bool live = (i0 + (int)threadIdx.x < K.nx) && (j0 + (int)threadIdx.y < K.ny);
  const bool el = K.elastic != 0;
  auto plane = [&](int z) { return NP * wrap_t<P2, FAR>(z, K.nz); };
  // the z-queued values at node n
  auto ldq = [&](long long n, double* r) {
    r[0] = scr[n];
    const double cc = cn[n];
    r[1] = cc * (1.0 - cc);
#pragma unroll
    for (int e = 0; e < 3; ++e) r[2 + e] = (double)v[(1 + e) * N + n];
    if (el) {
      r[5] = scr[5 * N + n];
      r[6] = scr[6 * N + n];
      r[7] = scr[3 * N + n];
    }
  };
  // the staged values at node n (into a register set of 10)
  auto lds10 = [&](long long n, double* r) {
    r[0] = scr[n];
    const double cc = cn[n];
    r[1] = cc * (1.0 - cc);
#pragma unroll
    for (int e = 0; e < 3; ++e) r[2 + e] = (double)v[(1 + e) * N + n];
    if (el) {
      r[5] = scr[1 * N + n];
      r[6] = scr[2 * N + n];
      r[7] = scr[4 * N + n];
      r[8] = scr[5 * N + n];
      r[9] = scr[6 * N + n];
    }
  };
  double prv[8] = {}, cur[8] = {}, nxt[8] = {};
  ldq(plane(z0 - 1) + c.col, prv);
  ldq(plane(z0) + c.col, cur);
  const double idt = 1.0 / dt;
  const int nst = el ? 10 : 5;
  for (int z = z0; z < z1; ++z) {
    const long long pz = plane(z), n = pz + c.col;
    ldq(plane(z + 1) + c.col, nxt);
    double ring[10] = {};
    if (c.rslot >= 0) lds10(pz + c.rcol, ring);
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    if (el) {
      sxx = scr[1 * N + n];
      syy = scr[2 * N + n];
      sxy = scr[4 * N + n];
    }
    const double vc = (double)v[n];
    __syncthreads();  // every thread is done reading the previous plane
    const int q = c.slot;
#pragma unroll
    for (int f = 0; f < 5; ++f) sp[f * kRP3 + q] = cur[f];
    if (el) {
      sp[5 * kRP3 + q] = sxx;
      sp[6 * kRP3 + q] = syy;
      sp[7 * kRP3 + q] = sxy;
      sp[8 * kRP3 + q] = cur[5];
      sp[9 * kRP3 + q] = cur[6];
    }
    if (c.rslot >= 0) {
      for (int f = 0; f < nst; ++f) sp[f * kRP3 + c.rslot] = ring[f];
    }
    __syncthreads();
    if (live) {
      const double* sdg = sp;
      const double* sg = sp + kRP3;
      {
        // c row: v_c / dt - div_h(M grad_h dG), face mobility M = kappa/2 (g_i + g_j)
        const double mc = cur[1], g0 = cur[0];
        double s = 0.0;
        s += 0.5 * K.kappa * (mc + sg[q + 1]) * (sdg[q + 1] - g0) - 0.5 * K.kappa * (mc + sg[q - 1]) * (g0 - sdg[q - 1]);
        s += 0.5 * K.kappa * (mc + sg[q + kRX3]) * (sdg[q + kRX3] - g0) -
             0.5 * K.kappa * (mc + sg[q - kRX3]) * (g0 - sdg[q - kRX3]);
        s += 0.5 * K.kappa * (mc + nxt[1]) * (nxt[0] - g0) - 0.5 * K.kappa * (mc + prv[1]) * (g0 - prv[0]);
        w[n] = vc * idt - s * K.ih2;
      }
      const double vv[4] = {vc, cur[2], cur[3], cur[4]};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const double* se = sp + (2 + e) * kRP3;
        const double fc = cur[2 + e];
        double lp = 0.0;
        lp += se[q + 1] + se[q - 1];
        lp += se[q + kRX3] + se[q - kRX3];
        lp += nxt[2 + e] + prv[2 + e];
        lp = (lp - 6.0 * fc) * K.ih2;
        double s = -0.5 * K.gamma_eta * lp;
#pragma unroll
        for (int f = 0; f < 4; ++f) s += B[(4 * (1 + e) + f) * N + n] * vv[f];
        w[(1 + e) * N + n] = fc * idt + K.L_eta * s;
      }
      if (el) {
        const double* sxxp = sp + 5 * kRP3;
        const double* syyp = sp + 6 * kRP3;
        const double* sxyp = sp + 7 * kRP3;
        const double* sxzp = sp + 8 * kRP3;
        const double* syzp = sp + 9 * kRP3;
        // sum_J (sigma_IJ(p + e_J) - sigma_IJ(p - e_J)), J = x, y, z
        double d = 0.0;
        d += sxxp[q + 1] - sxxp[q - 1];
        d += sxyp[q + kRX3] - sxyp[q - kRX3];
        d += nxt[5] - prv[5];
        w[4 * N + n] = d * K.i2h;
        d = 0.0;
        d += sxyp[q + 1] - sxyp[q - 1];
        d += syyp[q + kRX3] - syyp[q - kRX3];
        d += nxt[6] - prv[6];
        w[5 * N + n] = d * K.i2h;
        d = 0.0;
        d += sxzp[q + 1] - sxzp[q - 1];
        d += syzp[q + kRX3] - syzp[q - kRX3];
        d += nxt[7] - prv[7];
        w[6 * N + n] = d * K.i2h;
      } else {
#pragma unroll
        for (int I = 0; I < 3; ++I) w[(4 + I) * N + n] = (double)v[(4 + I) * N + n];
      }
    }
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      prv[f] = cur[f];
      cur[f] = nxt[f];
    }
  }
}

// The first residual stage in 3D, in two passes over the same z-marching column blocks:
//   pass A (k_res3_g):   G_c and G_eta (the laps of c and eta at both levels, the trace of
//                        sigma at both levels, the chemical discrete gradient) into G4, and the
//                        stress sigma_IJ(X) (eigenstrain about cbar0) into six scratch planes
//                        s_xx, s_yy, s_zz, s_xy, s_xz, s_yz (without elasticity F_u = X_u instead);
//   pass B (k_res3_fu):  F_u = sum_J Dhat_J sigma_IJ from the stored stress.
// The arithmetic is that of k_residual_g term by term.
template <bool P2, bool FAR>
__global__ __launch_bounds__(kBX* kJY3) void k_res3_g(Consts K, const double* __restrict__ X,
                                                      const double* __restrict__ Xn, double* __restrict__ G4,
                                                      double* __restrict__ F, double* __restrict__ sig,
                                                      int zc, Bat bt) {
  // staged fields (in-plane neighbours): 0 c, 1..3 eta, 4..6 u of X; 7 c, 8..10 eta, 11, 12
  // u_x, u_y of Xn.  z-queued fields: 0..6 those of X, 7..10 c and eta of Xn, 11 u_z of Xn.
  constexpr int NS = 13, NQ = 12;
  __shared__ double sp[NS * kRP3];
  int bx, by, bz;
  const int bi = xcd_block(bt, bx, by, bz);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    X = bat_at(X, bo);
    Xn = bat_at(Xn, bo);
    G4 = bat_at(G4, bo);
    F = bat_at(F, bo);
    sig = bat_at(sig, bo);
  }
  const double cb = bt.cb[bi];
  const long long N = K.N, NP = (long long)K.nx * K.ny;
  const int i0 = bx * kBX, j0 = by * kJY3, z0 = bz * zc;
  const int z1 = (z0 + zc < K.nz) ? z0 + zc : K.nz;
  const Cols3 c = cols3<P2, FAR>(K, i0, j0);
  const bool live = (i0 + (int)threadIdx.x < K.nx) && (j0 + (int)threadIdx.y < K.ny);
  const bool el = K.elastic != 0;
  auto plane = [&](int z) { return NP * wrap_t<P2, FAR>(z, K.nz); };
  auto ldq = [&](long long n, double* r) {
#pragma unroll
    for (int f = 0; f < 7; ++f) r[f] = X[f * N + n];
#pragma unroll
    for (int f = 0; f < 4; ++f) r[7 + f] = Xn[f * N + n];
    r[11] = Xn[6 * N + n];
  };
  double prv[NQ], cur[NQ], nxt[NQ];
  ldq(plane(z0 - 1) + c.col, prv);
  ldq(plane(z0) + c.col, cur);
  for (int z = z0; z < z1; ++z) {
    const long long pz = plane(z), n = pz + c.col;
    ldq(plane(z + 1) + c.col, nxt);
    double ring[NS];
    if (c.rslot >= 0) {
      const long long m = pz + c.rcol;
#pragma unroll
      for (int f = 0; f < 7; ++f) ring[f] = X[f * N + m];
#pragma unroll
      for (int f = 0; f < 6; ++f) ring[7 + f] = Xn[f * N + m];
    }
    const double u0x = Xn[4 * N + n], u0y = Xn[5 * N + n];
    __syncthreads();  // every thread is done reading the previous plane
    const int q = c.slot;
#pragma unroll
    for (int f = 0; f < 11; ++f) sp[f * kRP3 + q] = cur[f];
    sp[11 * kRP3 + q] = u0x;
    sp[12 * kRP3 + q] = u0y;
    if (c.rslot >= 0) {
#pragma unroll
      for (int f = 0; f < NS; ++f) sp[f * kRP3 + c.rslot] = ring[f];
    }
    __syncthreads();
    if (live) {
      // 2 d + 1 point Laplacian of staged field f (z neighbours from queue slot fq)
      auto lap = [&](int f, int fq) {
        const double* s = sp + f * kRP3;
        double l = 0.0;
        l += s[q + 1] + s[q - 1];
        l += s[q + kRX3] + s[q - kRX3];
        l += nxt[fq] + prv[fq];
        return (l - 6.0 * s[q]) * K.ih2;
      };
      auto dx = [&](int f) { return (sp[f * kRP3 + q + 1] - sp[f * kRP3 + q - 1]) * K.i2h; };
      auto dy = [&](int f) { return (sp[f * kRP3 + q + kRX3] - sp[f * kRP3 + q - kRX3]) * K.i2h; };
      const double c1 = cur[0], c0 = cur[7];
      const double e1[3] = {cur[1], cur[2], cur[3]}, e0[3] = {cur[8], cur[9], cur[10]};
      double Gc, Ge[3];
      chem_dg<false>(K, c1, e1, c0, e0, Gc, Ge, nullptr);
      if (el) {
        double div1 = 0.0, div0 = 0.0;
        div1 += dx(4);
        div0 += dx(11);
        div1 += dy(5);
        div0 += dy(12);
        div1 += (nxt[6] - prv[6]) * K.i2h;
        div0 += (nxt[11] - prv[11]) * K.i2h;
        const double tr1 = K.Ctr * (div1 - 3 * K.eps0 * (c1 - cb));
        const double tr0 = K.Ctr * (div0 - 3 * K.eps0 * (c0 - cb));
        Gc -= K.eps0 * 0.5 * (tr1 + tr0);
      }
      Gc -= K.gamma_c * 0.5 * (lap(0, 0) + lap(7, 7));
      G4[n] = Gc;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        Ge[e] -= K.gamma_eta * 0.5 * (lap(1 + e, 1 + e) + lap(8 + e, 8 + e));
        G4[(1 + e) * N + n] = Ge[e];
      }
      if (el) {
        // Dhat_K u_L of X at the node: du[K][L]
        double du[3][3];
#pragma unroll
        for (int L = 0; L < 3; ++L) {
          du[0][L] = dx(4 + L);
          du[1][L] = dy(4 + L);
          du[2][L] = (nxt[4 + L] - prv[4 + L]) * K.i2h;
        }
        const double ec = K.eps0 * (c1 - cb);
        double sd[3];
#pragma unroll
        for (int I = 0; I < 3; ++I) {
          double s = 0.0;
#pragma unroll
          for (int L = 0; L < 3; ++L) s += (L == I ? K.C11 : K.C12) * (du[L][L] - ec);
          sd[I] = s;
        }
        sig[n] = sd[0];
        sig[1 * N + n] = sd[1];
        sig[2 * N + n] = sd[2];
        sig[3 * N + n] = K.C44 * (du[0][1] + du[1][0]);
        sig[4 * N + n] = K.C44 * (du[0][2] + du[2][0]);
        sig[5 * N + n] = K.C44 * (du[1][2] + du[2][1]);
      } else {
#pragma unroll
        for (int I = 0; I < 3; ++I) F[(4 + I) * N + n] = cur[4 + I];
      }
    }
#pragma unroll
    for (int f = 0; f < NQ; ++f) {
      prv[f] = cur[f];
      cur[f] = nxt[f];
    }
  }
}

template <bool P2, bool FAR>
__global__ __launch_bounds__(kBX* kJY3) void k_res3_fu(Consts K, const double* __restrict__ sig,
                                                       double* __restrict__ F, int zc, Bat bt) {
  // staged: 0 s_xx, 1 s_yy, 2 s_xy, 3 s_xz, 4 s_yz; z-queued: 0 s_xz, 1 s_yz, 2 s_zz
  __shared__ double sp[5 * kRP3];
  int bx, by, bz;
  const int bi = xcd_block(bt, bx, by, bz);
  if (bat_skip(bt, bi)) return;
  {
    const long long bo = bi * bt.stride;
    sig = bat_at(sig, bo);
    F = bat_at(F, bo);
  }
  const long long N = K.N, NP = (long long)K.nx * K.ny;
  const int i0 = bx * kBX, j0 = by * kJY3, z0 = bz * zc;
  const int z1 = (z0 + zc < K.nz) ? z0 + zc : K.nz;
  const Cols3 c = cols3<P2, FAR>(K, i0, j0);
  const bool live = (i0 + (int)threadIdx.x < K.nx) && (j0 + (int)threadIdx.y < K.ny);
  auto plane = [&](int z) { return NP * wrap_t<P2, FAR>(z, K.nz); };
  auto ldq = [&](long long n, double* r) {
    r[0] = sig[4 * N + n];
    r[1] = sig[5 * N + n];
    r[2] = sig[2 * N + n];
  };
  double prv[3], cur[3], nxt[3];
  ldq(plane(z0 - 1) + c.col, prv);
  ldq(plane(z0) + c.col, cur);
  const int so[5] = {0, 1, 3, 4, 5};  // scratch plane of each staged field
  for (int z = z0; z < z1; ++z) {
    const long long pz = plane(z), n = pz + c.col;
    ldq(plane(z + 1) + c.col, nxt);
    double ring[5];
    if (c.rslot >= 0) {
#pragma unroll
      for (int f = 0; f < 5; ++f) ring[f] = sig[so[f] * N + pz + c.rcol];
    }
    const double sxx = sig[n], syy = sig[1 * N + n], sxy = sig[3 * N + n];
    __syncthreads();  // every thread is done reading the previous plane
    const int q = c.slot;
    sp[q] = sxx;
    sp[kRP3 + q] = syy;
    sp[2 * kRP3 + q] = sxy;
    sp[3 * kRP3 + q] = cur[0];
    sp[4 * kRP3 + q] = cur[1];
    if (c.rslot >= 0) {
#pragma unroll
      for (int f = 0; f < 5; ++f) sp[f * kRP3 + c.rslot] = ring[f];
    }
    __syncthreads();
    if (live) {
      const double *pxx = sp, *pyy = sp + kRP3, *pxy = sp + 2 * kRP3, *pxz = sp + 3 * kRP3,
                   *pyz = sp + 4 * kRP3;
      // sum_J (sigma_IJ(p + e_J) - sigma_IJ(p - e_J)), J = x, y, z
      double d = 0.0;
      d += pxx[q + 1] - pxx[q - 1];
      d += pxy[q + kRX3] - pxy[q - kRX3];
      d += nxt[0] - prv[0];
      F[4 * N + n] = d * K.i2h;
      d = 0.0;
      d += pxy[q + 1] - pxy[q - 1];
      d += pyy[q + kRX3] - pyy[q - kRX3];
      d += nxt[1] - prv[1];
      F[5 * N + n] = d * K.i2h;
      d = 0.0;
      d += pxz[q + 1] - pxz[q - 1];
      d += pyz[q + kRX3] - pyz[q - kRX3];
      d += nxt[2] - prv[2];
      F[6 * N + n] = d * K.i2h;
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      prv[f] = cur[f];
      cur[f] = nxt[f];
    }
  }
}

// ---------------------------------------------------------------------------------
// energy (eqs. (relations)/(freeenergy)) and mass; partial: chem, elastic, interfacial, sum c
// ---------------------------------------------------------------------------------
__device__ inline double psi(double z) { return z * log(z) + (1.0 - z) * log(1.0 - z); }

template <bool P2>
__global__ __launch_bounds__(256) void k_energy(Consts K, const double* __restrict__ X,
                                                double* __restrict__ partial, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  X = bat_at(X, bi * bt.stride);
  partial = bat_at(partial, bi * bt.stride);
  const double cb = bt.cb[bi];
  __shared__ double lds[4];
  const long long N = K.N;
  double ech = 0.0, eel = 0.0, ein = 0.0, mc = 0.0;
  for (long long n = (long long)blockIdx.x * 256 + threadIdx.x; n < N; n += (long long)gridDim.x * 256) {
    const Pt p = coords(K, n);
    const double c = X[n];
    double e[4], f[3];
    e[0] = X[N + n];
    e[1] = X[2 * N + n];
    e[2] = X[3 * N + n];
    e[3] = 4.0 - e[0] - e[1] - e[2];
    f[0] = 1.0 - 0.5 * (e[0] + e[1]);
    f[1] = 1.0 - 0.5 * (e[0] + e[2]);
    f[2] = 1.0 - 0.5 * (e[1] + e[2]);
    double pv = 0.0;
    for (int m = 5; m >= 0; --m) pv = pv * c + K.pc[m];
    const double Av = (K.A2 + K.A3 * c) * c * c, Bv = K.B3 * c * c * c;
    double ideal = K.w_c * psi(c);
    for (int i = 0; i < 4; ++i) ideal += 0.25 * psi(c * e[i]);
    ech += pv + Av * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2]) + Bv * f[0] * f[1] * f[2] + K.theta * ideal;
    // elastic: eps^el : sigma / 2
    if (K.elastic) {
      double s = 0.0;
      for (int I = 0; I < K.dim; ++I)
        for (int J = 0; J < K.dim; ++J) {
          double eij = 0.5 * (dhat<P2>(K, X + (4 + I) * N, p, J) + dhat<P2>(K, X + (4 + J) * N, p, I));
          if (I == J) eij -= K.eps0 * (c - cb);
          s += eij * sigma<P2>(K, X + 4 * N, N, X, cb, p, I, J);
        }
      eel += 0.5 * s;
    }
    // interfacial: gamma/2 sum_k ((D+ w)^2 + (D- w)^2)/2
    for (int fld = 0; fld < 4; ++fld) {
      const double* w = X + fld * N;
      const double gam = (fld == 0) ? K.gamma_c : K.gamma_eta;
      const double wc = w[n];
      double s = 0.0;
      for (int dir = 0; dir < K.dim; ++dir) {
        const double dp = (w[at_dir<P2>(K, p, dir, 1)] - wc) * K.ih, dm = (wc - w[at_dir<P2>(K, p, dir, -1)]) * K.ih;
        s += 0.5 * (dp * dp + dm * dm);
      }
      ein += 0.5 * gam * s;
    }
    mc += c;
  }
  const double a = block_sum(ech, lds), b = block_sum(eel, lds), cc = block_sum(ein, lds),
               d = block_sum(mc, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a;
    partial[kRedBlocks + blockIdx.x] = b;
    partial[2 * kRedBlocks + blockIdx.x] = cc;
    partial[3 * kRedBlocks + blockIdx.x] = d;
  }
}

dim3 stencil_grid(const Consts& K) {
  return dim3((K.nx + kBX - 1) / kBX, (K.ny + kBY - 1) / kBY, K.nz);
}

}  // namespace

bool pow2_sides(const Consts& K) {
  auto p2 = [](int n) { return (n & (n - 1)) == 0; };
  return p2(K.nx) && p2(K.ny) && p2(K.nz);
}

// the mean composition of each instance (a single problem's from K)
static Bat with_cbar0(const Consts& K, const Bat& bt) {
  Bat b = bt;
  if (!b.per) b.cb[0] = K.cbar0;
  return b;
}

void launch_residual(const Consts& K, double dt, const double* X, const double* Xn, double* G4,
                     double* F, double* partial, hipStream_t s, const Bat& bt_, double* sig) {
  const Bat bt = with_cbar0(K, bt_);
  const dim3 gg = bat_grid(stencil_grid(K), bt), gf = bat_grid(dim3(kRedBlocks), bt);
  if (K.dim == 3 && sig) {
    // the first stage in two passes over z-marching column blocks (as the 3D J v)
    const int zc = K.nz < kJZ3 ? K.nz : kJZ3;
    const dim3 g((K.nx + kBX - 1) / kBX, (K.ny + kJY3 - 1) / kJY3, (K.nz + zc - 1) / zc);
    const bool far = !((int)g.x * kBX < 2 * K.nx && (int)g.y * kJY3 < 2 * K.ny);
    const dim3 gb = bat_grid(g, bt), tb(kBX, kJY3);
    const bool p2 = pow2_sides(K);
    if (p2) {
      hipLaunchKernelGGL((k_res3_g<true, false>), gb, tb, 0, s, K, X, Xn, G4, F, sig, zc, bt);
      if (K.elastic) hipLaunchKernelGGL((k_res3_fu<true, false>), gb, tb, 0, s, K, sig, F, zc, bt);
      hipLaunchKernelGGL(k_residual_f<true>, gf, dim3(256), 0, s, K, dt, X, Xn, G4, F, partial, bt);
    } else if (far) {
      hipLaunchKernelGGL((k_res3_g<false, true>), gb, tb, 0, s, K, X, Xn, G4, F, sig, zc, bt);
      if (K.elastic) hipLaunchKernelGGL((k_res3_fu<false, true>), gb, tb, 0, s, K, sig, F, zc, bt);
      hipLaunchKernelGGL(k_residual_f<false>, gf, dim3(256), 0, s, K, dt, X, Xn, G4, F, partial, bt);
    } else {
      hipLaunchKernelGGL((k_res3_g<false, false>), gb, tb, 0, s, K, X, Xn, G4, F, sig, zc, bt);
      if (K.elastic) hipLaunchKernelGGL((k_res3_fu<false, false>), gb, tb, 0, s, K, sig, F, zc, bt);
      hipLaunchKernelGGL(k_residual_f<false>, gf, dim3(256), 0, s, K, dt, X, Xn, G4, F, partial, bt);
    }
    return;
  }
  if (pow2_sides(K)) {
    hipLaunchKernelGGL(k_residual_g<true>, gg, dim3(kBX, kBY), 0, s, K, X, Xn, G4, F, bt);
    hipLaunchKernelGGL(k_residual_f<true>, gf, dim3(256), 0, s, K, dt, X, Xn, G4, F, partial, bt);
  } else {
    hipLaunchKernelGGL(k_residual_g<false>, gg, dim3(kBX, kBY), 0, s, K, X, Xn, G4, F, bt);
    hipLaunchKernelGGL(k_residual_f<false>, gf, dim3(256), 0, s, K, dt, X, Xn, G4, F, partial, bt);
  }
}

void launch_linearise(const Consts& K, const double* X, const double* Xn, double* B, float* Bf,
                      hipStream_t s, const Bat& bt) {
  long long nb = (K.N + 255) / 256;
  hipLaunchKernelGGL(k_linearise, bat_grid(dim3((unsigned)(nb < 4096 ? nb : 4096)), bt), dim3(256), 0, s, K, X,
                     Xn, B, Bf, bt);
}

template <typename Tv>
void launch_jv(const Consts& K, double dt, const double* B, const double* cn, const Tv* v, double* w,
               double* scr, hipStream_t s, const Bat& bt) {
  const bool p2 = pow2_sides(K);
  if (K.dim == 2) {
    const dim3 g((K.nx + kBX - 1) / kBX, (K.ny + kJY2 - 1) / kJY2, 1);
    // halo positions run from -2 to (blocks x block side) + 1: the two-select wrap holds while
    // that stays below 2n (sides are >= 4)
    const bool far = !((int)g.x * kBX + 1 < 2 * K.nx && (int)g.y * kJY2 + 1 < 2 * K.ny);
    const dim3 gb = bat_grid(g, bt);
    if (p2) hipLaunchKernelGGL((k_jv2<Tv, true, false>), gb, dim3(kBX, kJY2), 0, s, K, dt, B, cn, v, w, bt);
    else if (far) hipLaunchKernelGGL((k_jv2<Tv, false, true>), gb, dim3(kBX, kJY2), 0, s, K, dt, B, cn, v, w, bt);
    else hipLaunchKernelGGL((k_jv2<Tv, false, false>), gb, dim3(kBX, kJY2), 0, s, K, dt, B, cn, v, w, bt);
  } else {
    const int zc = K.nz < kJZ3 ? K.nz : kJZ3;
    const dim3 g((K.nx + kBX - 1) / kBX, (K.ny + kJY3 - 1) / kJY3, (K.nz + zc - 1) / zc);
    // staged columns run from -1 to (blocks x block side); planes from z0 - 1 to z0 + zc stay
    // within [-1, nz]
    const bool far = !((int)g.x * kBX < 2 * K.nx && (int)g.y * kJY3 < 2 * K.ny);
    const dim3 gb = bat_grid(g, bt), tb(kBX, kJY3);
    if (p2) {
      hipLaunchKernelGGL((k_jv3_dg<Tv, true, false>), gb, tb, 0, s, K, B, v, scr, zc, bt);
      hipLaunchKernelGGL((k_jv3_rows<Tv, true, false>), gb, tb, 0, s, K, dt, B, cn, v, scr, w, zc, bt);
    } else if (far) {
      hipLaunchKernelGGL((k_jv3_dg<Tv, false, true>), gb, tb, 0, s, K, B, v, scr, zc, bt);
      hipLaunchKernelGGL((k_jv3_rows<Tv, false, true>), gb, tb, 0, s, K, dt, B, cn, v, scr, w, zc, bt);
    } else {
      hipLaunchKernelGGL((k_jv3_dg<Tv, false, false>), gb, tb, 0, s, K, B, v, scr, zc, bt);
      hipLaunchKernelGGL((k_jv3_rows<Tv, false, false>), gb, tb, 0, s, K, dt, B, cn, v, scr, w, zc, bt);
    }
  }
}
template void launch_jv<double>(const Consts&, double, const double*, const double*, const double*, double*,
                                double*, hipStream_t, const Bat&);
template void launch_jv<float>(const Consts&, double, const double*, const double*, const float*, double*,
                               double*, hipStream_t, const Bat&);

void launch_energy(const Consts& K, const double* X, double* partial, hipStream_t s, const Bat& bt_) {
  const Bat bt = with_cbar0(K, bt_);
  const dim3 g = bat_grid(dim3(kRedBlocks), bt);
  if (pow2_sides(K)) hipLaunchKernelGGL(k_energy<true>, g, dim3(256), 0, s, K, X, partial, bt);
  else hipLaunchKernelGGL(k_energy<false>, g, dim3(256), 0, s, K, X, partial, bt);
}

}  // namespace pf
