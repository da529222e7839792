// Exact solve of the displacement block of the NSOA-1 Jacobian by discrete Fourier transform.
//
// The displacement rows of scheme (NSOA-1) are the discrete equilibrium
// (mechanicalequilibrium-dis) sum_J Dhat_J sigma_IJ = 0 with sigma = Lscale C : eps and
// eps_IJ = (Dhat_J u_I + Dhat_I u_J)/2.  On a periodic grid with homogeneous cubic C that
// operator is diagonalised by the DFT: Dhat_J -> i S_J, S_J = sin(2 pi m_J / n_J) / h, and
//   Khat_IK = - sum_{J,L} C_IJKL S_J S_L
//           = -[C11 S_I^2 + C44 sum_{J != I} S_J^2]     (I = K)
//           = -(C12 + C44) S_I S_K                      (I != K).
// Modes with every S_J = 0 (the parity-class constants that Dhat annihilates) get u = 0, which
// is the zero-mean-per-parity-class gauge.
//
// Transforms: in-LDS decimation-in-time FFTs along one direction at a time (radix-4 stage
// pairs, a last radix-2 stage when log2 n is odd), several lines per workgroup, complex double.  Two real fields travel as one complex field
// (q_1 + i q_2); their spectra are separated with the conjugate-symmetric mirror k -> -k.
#include "pf_internal.h"

namespace pf {

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftLds = 4096;  // complex doubles of line data per workgroup (64 KiB; twiddles extra)

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// LDS position of line element i: one pad slot after every 8 elements, which spreads the
// power-of-two strides of the bit-reversed stores and the first butterfly stages over all LDS
// banks (unpadded, the 16-byte elements of a wave landed on the same banks); lp_size(len)
// slots hold elements 0 .. len - 1.
__host__ __device__ constexpr int lp(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lp_size(int len) { return len + (len >> 3) + 1; }

// ---- fused 2D pipeline ------------------------------------------------------------------
// In-LDS transform of one line of n = 2^logn complex points stored in bit-reversed order at
// padded positions lp(base + l n + k), k < n, of buf; radix-4 stage pairs (two radix-2 stages
// per thread, 4 points in registers) and a final radix-2 stage when logn is odd.  All threads
// of the block take part; nl lines l are transformed together.
__device__ inline void fft_lds(double2* buf, int n, int logn, int nl, const double2* __restrict__ tw,
                               int inverse, int base = 0) {
  int s = 1;
  for (; s + 1 <= logn; s += 2) {
    const int half = 1 << (s - 1);
    const int nq = n >> 2;  // quads per line
    for (int t = threadIdx.x; t < nl * nq; t += blockDim.x) {
      const int l = t / nq, r = t - l * nq;
      const int grp = r / half, pos = r - grp * half;
      const int i0 = base + l * n + grp * 4 * half + pos;
      double2 w1 = tw[pos * (n >> s)];                 // W_{2 half}^pos
      double2 w2 = tw[pos * (n >> (s + 1))];           // W_{4 half}^pos
      double2 w3 = tw[(pos + half) * (n >> (s + 1))];  // W_{4 half}^(pos + half)
      if (inverse) {
        w1.y = -w1.y;
        w2.y = -w2.y;
        w3.y = -w3.y;
      }
      const double2 a0 = buf[lp(i0)], a1 = cmul(buf[lp(i0 + half)], w1), a2 = buf[lp(i0 + 2 * half)],
                    a3 = cmul(buf[lp(i0 + 3 * half)], w1);
      const double2 c0 = make_double2(a0.x + a1.x, a0.y + a1.y), c1 = make_double2(a0.x - a1.x, a0.y - a1.y);
      const double2 c2 = make_double2(a2.x + a3.x, a2.y + a3.y), c3 = make_double2(a2.x - a3.x, a2.y - a3.y);
      const double2 d2 = cmul(c2, w2), d3 = cmul(c3, w3);
      buf[lp(i0)] = make_double2(c0.x + d2.x, c0.y + d2.y);
      buf[lp(i0 + 2 * half)] = make_double2(c0.x - d2.x, c0.y - d2.y);
      buf[lp(i0 + half)] = make_double2(c1.x + d3.x, c1.y + d3.y);
      buf[lp(i0 + 3 * half)] = make_double2(c1.x - d3.x, c1.y - d3.y);
    }
    __syncthreads();
  }
  if (s == logn) {
    const int half = 1 << (s - 1);
    const int nh = n >> 1;
    for (int t = threadIdx.x; t < nl * nh; t += blockDim.x) {
      const int l = t / nh, r = t - l * nh;
      const int grp = r / half, pos = r - grp * half;
      const int i0 = base + l * n + grp * 2 * half + pos;
      double2 w = tw[pos * (n >> s)];
      if (inverse) w.y = -w.y;
      const double2 a0 = buf[lp(i0)], a1 = cmul(buf[lp(i0 + half)], w);
      buf[lp(i0)] = make_double2(a0.x + a1.x, a0.y + a1.y);
      buf[lp(i0 + half)] = make_double2(a0.x - a1.x, a0.y - a1.y);
    }
    __syncthreads();
  }
}

// The twiddles W_n^k, k < n/2, copied into LDS (tws) once per workgroup: every stage of the
// in-LDS transforms reads three per butterfly, which would otherwise wait on global loads.
// Visible after the workgroup's next barrier.
__device__ inline void stage_twiddles(double2* tws, const double2* __restrict__ tw, int n) {
  for (int e = threadIdx.x; e < n / 2; e += blockDim.x) tws[e] = tw[e];
}

// Lines of length n (power of two), points pstride apart; line l starts at
// (l % la) * lb + (l / la) * lc.  contiguous = 1 when pstride == 1 (threads walk along a line),
// else consecutive threads take consecutive lines (la lines adjacent in memory).
__global__ __launch_bounds__(kFftThreads) void k_fft_lines(double2* __restrict__ data, int n, int logn,
                                                           long long pstride, long long la,
                                                           long long lb, long long lc, long long nlines,
                                                           int lpb, const double2* __restrict__ tw,
                                                           int inverse, int contiguous, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  data = bat_at(data, bo);
  extern __shared__ double2 sm[];  // lpb lines of n (padded), then n/2 twiddles
  double2* tws = sm + lp_size(lpb * n);
  stage_twiddles(tws, tw, n);
  const long long line0 = (long long)blockIdx.x * lpb;
  const int total = lpb * n;
  for (int e = threadIdx.x; e < total; e += kFftThreads) {
    int l, p;
    if (contiguous) {
      l = e / n;
      p = e - l * n;
    } else {
      l = e % lpb;
      p = e / lpb;
    }
    const long long line = line0 + l;
    if (line < nlines) {
      const long long off = (line % la) * lb + (line / la) * lc;
      const int rp = (int)(__brev((unsigned)p) >> (32 - logn));
      sm[lp(l * n + rp)] = data[off + p * pstride];
    }
  }
  __syncthreads();
  fft_lds(sm, n, logn, lpb, tws, inverse);
  for (int e = threadIdx.x; e < total; e += kFftThreads) {
    int l, p;
    if (contiguous) {
      l = e / n;
      p = e - l * n;
    } else {
      l = e % lpb;
      p = e / lpb;
    }
    const long long line = line0 + l;
    if (line < nlines) {
      const long long off = (line % la) * lb + (line / la) * lc;
      data[off + p * pstride] = sm[lp(l * n + p)];
    }
  }
}

__device__ inline int brev(int p, int logn) { return (int)(__brev((unsigned)p) >> (32 - logn)); }

// Workgroups go to the 8 XCDs round-robin by id: block b < nb (nb a multiple of 8) is given
// index (b mod 8) * (nb / 8) + b / 8, so that each XCD works on a contiguous band; other
// blocks keep their id.
__device__ inline int xcd_band(int b, int nb) {
  if ((nb & 7) != 0 || b >= nb) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// pass 1: rows j0 .. j0+nl-1: q = r_u + a Dhat z_c packed as q_x + i q_y, forward FFT along x
template <typename T>
__global__ __launch_bounds__(256) void k_fft2_rows_fwd(Consts K, const T* __restrict__ r, double a,
                                                       const T* __restrict__ zc, int logn, int nl,
                                                       const double2* __restrict__ tw,
                                                       double2* __restrict__ out, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  r = bat_at(r, bo);
  zc = bat_at(zc, bo);
  out = bat_at(out, bo);
  extern __shared__ double2 sm[];  // nl * n (padded), then n/2 twiddles
  const int n = K.nx;
  double2* tws = sm + lp_size(nl * n);
  stage_twiddles(tws, tw, n);
  const int j0 = xcd_band(blockIdx.x, gridDim.x) * nl;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    const int l = e / n, i = e - l * n, j = j0 + l;
    const long long m = (long long)i + (long long)n * j;
    double qx = r ? (double)r[m] : 0.0, qy = r ? (double)r[K.N + m] : 0.0;
    if (zc && a != 0.0) {
      const int ip = (i + 1 == n) ? 0 : i + 1, im = (i == 0) ? n - 1 : i - 1;
      const int jp = (j + 1 == K.ny) ? 0 : j + 1, jm = (j == 0) ? K.ny - 1 : j - 1;
      qx += a * ((double)zc[ip + (long long)n * j] - (double)zc[im + (long long)n * j]) * K.i2h;
      qy += a * ((double)zc[i + (long long)n * jp] - (double)zc[i + (long long)n * jm]) * K.i2h;
    }
    sm[lp(l * n + brev(i, logn))] = make_double2(qx, qy);
  }
  __syncthreads();
  fft_lds(sm, n, logn, nl, tws, 0);
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    const int l = e / n, i = e - l * n;
    out[(long long)i + (long long)n * (j0 + l)] = sm[lp(e)];
  }
}

// The 2D symbol solve at wave numbers (S0, S1) = (S_kx, S_ky): the spectra av = Z(k) and
// bv = Z(-k) of z = q_x + i q_y give Q_x = (Z(k) + conj Z(-k)) / 2 and Q_y = (Z(k) -
// conj Z(-k)) / (2i); Khat U = Q (U = 0 where S0 = S1 = 0: the gauge; U = Q without
// elasticity); returns the spectrum of u_x + i u_y, U_x + i U_y.
__device__ inline double2 symbol_solve2(const Consts& K, double2 av, double2 bv, double S0, double S1) {
  const double2 Q0 = make_double2(0.5 * (av.x + bv.x), 0.5 * (av.y - bv.y));
  const double2 Q1 = make_double2(0.5 * (av.y + bv.y), -0.5 * (av.x - bv.x));
  double2 U0 = make_double2(0.0, 0.0), U1 = make_double2(0.0, 0.0);
  const double s2 = S0 * S0 + S1 * S1;
  if (!K.elastic) {
    U0 = Q0;
    U1 = Q1;
  } else if (s2 != 0.0) {
    const double A00 = -(K.C11 * S0 * S0 + K.C44 * S1 * S1), A11 = -(K.C11 * S1 * S1 + K.C44 * S0 * S0);
    const double A01 = -(K.C12 + K.C44) * S0 * S1;
    const double id = 1.0 / (A00 * A11 - A01 * A01);
    U0 = make_double2((A11 * Q0.x - A01 * Q1.x) * id, (A11 * Q0.y - A01 * Q1.y) * id);
    U1 = make_double2((A00 * Q1.x - A01 * Q0.x) * id, (A00 * Q1.y - A01 * Q0.y) * id);
  }
  return make_double2(U0.x - U1.y, U0.y + U1.x);
}

// pass 2: the column pair (kx, -kx): forward FFT along y, pointwise solve of the 2 x 2
// symbol system (needs Z(k) and Z(-k), both in this block), inverse FFT along y.  Block kx
// (0 .. nx/2 - 1) takes columns kx and nx - kx; block 0 takes the two columns that are
// their own mirrors, 0 and nx/2, so that nx/2 blocks cover the spectrum.
__global__ __launch_bounds__(256) void k_fft2_cols_solve(Consts K, int logn, const double2* __restrict__ tw,
                                                         const double* __restrict__ sx,
                                                         const double* __restrict__ syt,
                                                         double2* __restrict__ data, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  data = bat_at(data, bo);
  // 2 lines of n, then the 2 lines of output spectra (elements 2n .. 4n; padded), then n/2
  // twiddles
  extern __shared__ double2 sm[];
  const int n = K.ny, nx = K.nx;
  double2* tws = sm + lp_size(4 * n);
  stage_twiddles(tws, tw, n);
  // XCD-band order, so that the columns one XCD reads are adjacent and share cache lines
  const int kx = xcd_band(blockIdx.x, gridDim.x);
  const bool self = (kx == 0);
  const int kxm = self ? nx / 2 : nx - kx;
  constexpr int ncol = 2;
  for (int e = threadIdx.x; e < ncol * n; e += blockDim.x) {
    const int l = e / n, j = e - l * n;
    const int col = l ? kxm : kx;
    sm[lp(l * n + brev(j, logn))] = data[(long long)col + (long long)nx * j];
  }
  __syncthreads();
  fft_lds(sm, n, logn, ncol, tws, 0);
  for (int e = threadIdx.x; e < ncol * n; e += blockDim.x) {
    const int l = e / n, j = e - l * n;
    const int col = l ? kxm : kx;
    const int lm = self ? l : 1 - l;   // the mirror column's line
    const int jm = (j == 0) ? 0 : n - j;
    const double2 av = sm[lp(l * n + j)], bv = sm[lp(lm * n + jm)];
    const double2 Uv = symbol_solve2(K, av, bv, sx[col], syt[j]);
    // spectrum of u_x + i u_y, written in bit-reversed order for the inverse transform
    sm[lp(2 * n + l * n + brev(j, logn))] = Uv;
  }
  __syncthreads();
  fft_lds(sm, n, logn, ncol, tws, 1, 2 * n);
  for (int e = threadIdx.x; e < ncol * n; e += blockDim.x) {
    const int l = e / n, j = e - l * n;
    const int col = l ? kxm : kx;
    data[(long long)col + (long long)nx * j] = sm[lp(2 * n + e)];
  }
}

// pass 3: inverse FFT along x, unpack u_x = Re / N, u_y = Im / N
template <typename T>
__global__ __launch_bounds__(256) void k_fft2_rows_inv(Consts K, int logn, int nl, const double2* __restrict__ tw,
                                                       const double2* __restrict__ in, T* __restrict__ u, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  in = bat_at(in, bo);
  u = bat_at(u, bo);
  extern __shared__ double2 sm[];  // nl * n (padded), then n/2 twiddles
  const int n = K.nx;
  double2* tws = sm + lp_size(nl * n);
  stage_twiddles(tws, tw, n);
  const int j0 = xcd_band(blockIdx.x, gridDim.x) * nl;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    const int l = e / n, i = e - l * n;
    sm[lp(l * n + brev(i, logn))] = in[(long long)i + (long long)n * (j0 + l)];
  }
  __syncthreads();
  fft_lds(sm, n, logn, nl, tws, 1);
  const double inv = 1.0 / (double)K.N;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    const int l = e / n, i = e - l * n;
    const long long m = (long long)i + (long long)n * (j0 + l);
    u[m] = (T)(sm[lp(e)].x * inv);
    u[K.N + m] = (T)(sm[lp(e)].y * inv);
  }
}

// ---- 3D pipeline with real-to-complex transforms along x ---------------------------
// The three displacement fields are real, so along x only the half spectrum kx <= nx/2 is
// kept (nxh = nx/2 + 1 columns; the rest follows by conjugation).  Half spectra are stored
// as Qh[f][k][j][kx] (f = 0..2, one plane of nxh * ny * nz complex each; 1.52 N complex in
// all at nx = 128).  Five passes: x (real to complex, fused with forming q = r + a Dhat zc),
// y (all three fields in one launch), z fused with the pointwise solve, y inverse, x inverse
// (complex to real, scaled by 1/N).  In the x passes y and z are still physical, so every
// x line is real and its spectrum is Hermitian in kx alone.

// x pass.  A block takes rp row pairs (j0, j0 + 1) of plane k and transforms three complex
// lines per pair: q1 + i q2 of each row and q3(j0) + i q3(j0 + 1); the two real spectra in
// each line are separated with kx <-> nx - kx.
template <typename T>
__global__ __launch_bounds__(256) void k_r2c_x(Consts K, const T* __restrict__ r, double a,
                                               const T* __restrict__ zc, int logn, int rp,
                                               const double2* __restrict__ tw, double2* __restrict__ Qh, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  r = bat_at(r, bo);
  zc = bat_at(zc, bo);
  Qh = bat_at(Qh, bo);
  extern __shared__ double2 sm[];  // 3 rp lines of nx (padded), then nx/2 twiddles
  const int n = K.nx, nxh = n / 2 + 1, hb = K.ny / (2 * rp);
  double2* tws = sm + lp_size(3 * rp * n);
  stage_twiddles(tws, tw, n);
  const int b = xcd_band((int)blockIdx.x, (int)gridDim.x);
  const int jb = (b % hb) * 2 * rp, k = b / hb;
  const long long NN = K.N;
  for (int e = threadIdx.x; e < 2 * rp * n; e += blockDim.x) {
    const int rr = e / n, i = e - rr * n, j = jb + rr;
    const int q = rr >> 1, l = rr & 1;
    const long long row = (long long)n * ((long long)j + (long long)K.ny * k);
    const long long m = row + i;
    double q0 = r ? (double)r[m] : 0.0, q1 = r ? (double)r[NN + m] : 0.0, q2 = r ? (double)r[2 * NN + m] : 0.0;
    if (zc && a != 0.0) {
      const int jp = (j + 1) & (K.ny - 1), jm = (j - 1) & (K.ny - 1);
      const int kp = (k + 1) & (K.nz - 1), km = (k - 1) & (K.nz - 1);
      q0 += a * ((double)zc[row + ((i + 1) & (n - 1))] - (double)zc[row + ((i - 1) & (n - 1))]) * K.i2h;
      q1 += a * ((double)zc[i + (long long)n * (jp + (long long)K.ny * k)] -
                 (double)zc[i + (long long)n * (jm + (long long)K.ny * k)]) * K.i2h;
      q2 += a * ((double)zc[i + (long long)n * (j + (long long)K.ny * kp)] -
                 (double)zc[i + (long long)n * (j + (long long)K.ny * km)]) * K.i2h;
    }
    const int bi = brev(i, logn);
    sm[lp((3 * q + l) * n + bi)] = make_double2(q0, q1);
    reinterpret_cast<double*>(&sm[lp((3 * q + 2) * n + bi)])[l] = q2;
  }
  __syncthreads();
  fft_lds(sm, n, logn, 3 * rp, tws, 0);
  const long long plane = (long long)nxh * K.ny * K.nz;
  for (int e = threadIdx.x; e < 3 * rp * nxh; e += blockDim.x) {
    const int line = e / nxh, kx = e - line * nxh;
    const int q = line / 3, t = line - 3 * q, j0 = jb + 2 * q;
    const double2 av = sm[lp(line * n + kx)], bv = sm[lp(line * n + ((n - kx) & (n - 1)))];
    const double2 A = make_double2(0.5 * (av.x + bv.x), 0.5 * (av.y - bv.y));   // real part's spectrum
    const double2 B = make_double2(0.5 * (av.y + bv.y), -0.5 * (av.x - bv.x));  // imaginary part's
    if (t < 2) {
      const long long o = kx + (long long)nxh * ((long long)(j0 + t) + (long long)K.ny * k);
      Qh[o] = A;
      Qh[plane + o] = B;
    } else {
      const long long o = 2 * plane + kx + (long long)nxh * ((long long)j0 + (long long)K.ny * k);
      Qh[o] = A;
      Qh[o + nxh] = B;
    }
  }
}

// z pass with the solve: lpb adjacent kx columns at one ky, all three fields.  Forward FFT
// along z, Khat U = Q at every mode (U = 0 where every S_J = 0: the gauge; U = Q without
// elasticity), the bit-reversal permutation in place, inverse FFT along z.
__global__ __launch_bounds__(256) void k_z_solve(Consts K, int logn, int lpb, const double2* __restrict__ tw,
                                                 const double* __restrict__ sx, const double* __restrict__ sy,
                                                 const double* __restrict__ szt, double2* __restrict__ Qh, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  Qh = bat_at(Qh, bo);
  extern __shared__ double2 sm[];  // 3 lpb lines of nz: line (f lpb + l) (padded), then nz/2 twiddles
  const int n = K.nz, nxh = K.nx / 2 + 1;
  double2* tws = sm + lp_size(3 * lpb * n);
  stage_twiddles(tws, tw, n);
  const int nxb = (nxh + lpb - 1) / lpb;
  const int b = xcd_band((int)blockIdx.x, (int)gridDim.x);
  const int kx0 = (b % nxb) * lpb, ky = b / nxb;
  const long long plane = (long long)nxh * K.ny * K.nz;
  const long long zs = (long long)nxh * K.ny;
  const long long base = kx0 + (long long)nxh * ky;
  const int nl = 3 * lpb;
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    const int l = e % lpb, rest = e / lpb, p = rest % n, f = rest / n;
    double2 v = make_double2(0.0, 0.0);
    if (kx0 + l < nxh) v = Qh[f * plane + base + l + zs * p];
    sm[lp((f * lpb + l) * n + brev(p, logn))] = v;
  }
  __syncthreads();
  fft_lds(sm, n, logn, nl, tws, 0);
  for (int e = threadIdx.x; e < lpb * n; e += blockDim.x) {
    const int l = e % lpb, p = e / lpb, kx = kx0 + l;
    if (kx >= nxh) continue;
    const double S0 = sx[kx], S1 = sy[ky], S2 = szt[p];
    const double s2 = S0 * S0 + S1 * S1 + S2 * S2;
    double2 Q[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) Q[f] = sm[lp((f * lpb + l) * n + p)];
    if (K.elastic) {
      double2 U[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
      if (s2 != 0.0) {
        const double S[3] = {S0, S1, S2};
        double A[3][3];
#pragma unroll
        for (int I = 0; I < 3; ++I)
#pragma unroll
          for (int L = 0; L < 3; ++L)
            A[I][L] = (I == L) ? -(K.C11 * S[I] * S[I] + K.C44 * (s2 - S[I] * S[I])) : -(K.C12 + K.C44) * S[I] * S[L];
        // symmetric 3 x 3 inverse by the adjugate
        const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        const double c01 = A[0][2] * A[2][1] - A[0][1] * A[2][2];
        const double c02 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
        const double c11 = A[0][0] * A[2][2] - A[0][2] * A[2][0];
        const double c12 = A[0][2] * A[1][0] - A[0][0] * A[1][2];
        const double c22 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        const double id = 1.0 / (A[0][0] * c00 + A[0][1] * (A[1][2] * A[2][0] - A[1][0] * A[2][2]) +
                                 A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]));
        const double Ai[3][3] = {{c00 * id, c01 * id, c02 * id}, {c01 * id, c11 * id, c12 * id},
                                 {c02 * id, c12 * id, c22 * id}};
#pragma unroll
        for (int I = 0; I < 3; ++I)
          U[I] = make_double2(Ai[I][0] * Q[0].x + Ai[I][1] * Q[1].x + Ai[I][2] * Q[2].x,
                              Ai[I][0] * Q[0].y + Ai[I][1] * Q[1].y + Ai[I][2] * Q[2].y);
      }
#pragma unroll
      for (int f = 0; f < 3; ++f) sm[lp((f * lpb + l) * n + p)] = U[f];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    const int line = e / n, p = e - line * n, q = brev(p, logn);
    if (p < q) {
      const double2 t = sm[lp(line * n + p)];
      sm[lp(line * n + p)] = sm[lp(line * n + q)];
      sm[lp(line * n + q)] = t;
    }
  }
  __syncthreads();
  fft_lds(sm, n, logn, nl, tws, 1);
  for (int e = threadIdx.x; e < nl * n; e += blockDim.x) {
    const int l = e % lpb, rest = e / lpb, p = rest % n, f = rest / n;
    if (kx0 + l < nxh) Qh[f * plane + base + l + zs * p] = sm[lp((f * lpb + l) * n + p)];
  }
}

// x pass back: rp row pairs of plane k.  Each line is rebuilt over the full kx range from
// the half spectra (conjugates above nx/2) as U1 + i U2 of one row, or U3(j0) + i U3(j0 + 1);
// one inverse FFT per line gives the real fields, u = result / N.
template <typename T>
__global__ __launch_bounds__(256) void k_c2r_x(Consts K, int logn, int rp, const double2* __restrict__ tw,
                                               const double2* __restrict__ Qh, T* __restrict__ u, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  Qh = bat_at(Qh, bo);
  u = bat_at(u, bo);
  extern __shared__ double2 sm[];  // 3 rp lines of nx (padded), then nx/2 twiddles
  const int n = K.nx, nxh = n / 2 + 1, hb = K.ny / (2 * rp);
  double2* tws = sm + lp_size(3 * rp * n);
  stage_twiddles(tws, tw, n);
  const int b = xcd_band((int)blockIdx.x, (int)gridDim.x);
  const int jb = (b % hb) * 2 * rp, k = b / hb;
  const long long plane = (long long)nxh * K.ny * K.nz;
  for (int e = threadIdx.x; e < 3 * rp * n; e += blockDim.x) {
    const int line = e / n, kx = e - line * n;
    const int q = line / 3, t = line - 3 * q, j0 = jb + 2 * q;
    const bool mirror = kx >= nxh;
    const int kk = mirror ? n - kx : kx;
    long long o1, o2;
    if (t < 2) {
      o1 = kk + (long long)nxh * ((long long)(j0 + t) + (long long)K.ny * k);
      o2 = plane + o1;
    } else {
      o1 = 2 * plane + kk + (long long)nxh * ((long long)j0 + (long long)K.ny * k);
      o2 = o1 + nxh;
    }
    double2 P = Qh[o1], Q = Qh[o2];
    if (mirror) {
      P.y = -P.y;
      Q.y = -Q.y;
    }
    sm[lp(line * n + brev(kx, logn))] = make_double2(P.x - Q.y, P.y + Q.x);  // P + i Q
  }
  __syncthreads();
  fft_lds(sm, n, logn, 3 * rp, tws, 1);
  const double inv = 1.0 / (double)K.N;
  const long long NN = K.N;
  for (int e = threadIdx.x; e < 2 * rp * n; e += blockDim.x) {
    const int rr = e / n, i = e - rr * n, j = jb + rr;
    const int q = rr >> 1, l = rr & 1;
    const long long m = (long long)i + (long long)n * ((long long)j + (long long)K.ny * k);
    const double2 z = sm[lp((3 * q + l) * n + i)];
    const double2 z3 = sm[lp((3 * q + 2) * n + i)];
    u[m] = (T)(z.x * inv);
    u[NN + m] = (T)(z.y * inv);
    u[2 * NN + m] = (T)((l == 0 ? z3.x : z3.y) * inv);
  }
}

__device__ inline int wrapi(int a, int n) {
  a += (a < 0) ? n : 0;
  a -= (a >= n) ? n : 0;
  return a;
}

// ---- mixed-radix lines (sides that are not powers of two) --------------------------------
// Self-sorting (Stockham) transform of lines of any length n = 4^a 2^b 3^c 5^d 7^e 11^f 13^g:
// stage s of radix R takes the R points j + t n/R (t < R) of butterfly j, multiplies point t
// by W_{pR}^{t k} (k = j mod p, p = product of the radices before s), forms their R-point DFT
// and writes output u to (j - k) R + k + u p, ping-ponging between two LDS buffers; after the
// last stage the line is in natural order.  W_m^e = tw[e n/m] from the table of W_n^e, e < n,
// kept in LDS.
struct MrPlan {
  int nst;     // stages
  int r[16];   // radix of each stage
};

// One stage of radix R over the lpb lines of the block (src -> dst).  The R-th roots of unity
// W_R^u of the butterflies' DFTs are loaded into registers once per stage; the stage twiddles
// W_{pR}^{t k} come from the LDS table per butterfly.
template <int R>
__device__ inline void mr_stage(const double2* __restrict__ src, double2* __restrict__ dst,
                                const double2* __restrict__ tws, int n, int p, int lpb, int inverse) {
  const int m = n / R;
  const int tstep = n / (p * R);  // W_{pR}^{t k} = W_n^{t k n/(pR)}
  double2 wr[R];                  // W_R^u = W_n^{u n/R}
#pragma unroll
  for (int u = 0; u < R; ++u) {
    double2 w = tws[u * m];
    if (inverse) w.y = -w.y;
    wr[u] = w;
  }
  for (int b = threadIdx.x; b < lpb * m; b += kFftThreads) {
    const int l = b / m, j = b - l * m;
    const int k = j % p;
    const double2* sl = src + l * n;
    double2* dl = dst + l * n;
    double2 x[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      double2 v = sl[j + t * m];
      if (t > 0 && k > 0) {
        double2 w = tws[t * k * tstep];
        if (inverse) w.y = -w.y;
        v = cmul(v, w);
      }
      x[t] = v;
    }
    const int base = (j - k) * R + k;
    if constexpr (R == 2) {
      dl[base] = make_double2(x[0].x + x[1].x, x[0].y + x[1].y);
      dl[base + p] = make_double2(x[0].x - x[1].x, x[0].y - x[1].y);
    } else if constexpr (R == 4) {
      // W_4 = -i (forward) or +i (inverse)
      const double2 a = make_double2(x[0].x + x[2].x, x[0].y + x[2].y);
      const double2 c0 = make_double2(x[0].x - x[2].x, x[0].y - x[2].y);
      const double2 c = make_double2(x[1].x + x[3].x, x[1].y + x[3].y);
      const double2 d = make_double2(x[1].x - x[3].x, x[1].y - x[3].y);
      // -i d (forward), +i d (inverse)
      const double2 e = inverse ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);
      dl[base] = make_double2(a.x + c.x, a.y + c.y);
      dl[base + p] = make_double2(c0.x + e.x, c0.y + e.y);
      dl[base + 2 * p] = make_double2(a.x - c.x, a.y - c.y);
      dl[base + 3 * p] = make_double2(c0.x - e.x, c0.y - e.y);
    } else {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        double2 y = x[0];
#pragma unroll
        for (int t = 1; t < R; ++t) {
          const double2 z = cmul(x[t], wr[(t * u) % R]);
          y.x += z.x;
          y.y += z.y;
        }
        dl[base + u * p] = y;
      }
    }
  }
}

// All stages of the mixed-radix transform of lpb contiguous lines of n points held in LDS (b0),
// ping-ponging with b1; returns the buffer that holds the result, in natural order.  MAXR: the
// largest radix the kernel is built for (5, 7 or 13: the registers of the largest butterfly
// bound the kernel's occupancy, so lines without radices 7, 11, 13 use a smaller build).
template <int MAXR>
__device__ inline double2* mr_lines(double2* b0, double2* b1, const double2* tws, int n, int lpb, const MrPlan& pl,
                                    int inverse) {
  double2 *src = b0, *dst = b1;
  int p = 1;
  for (int st = 0; st < pl.nst; ++st) {
    const int R = pl.r[st];
    if (R == 2) mr_stage<2>(src, dst, tws, n, p, lpb, inverse);
    else if (R == 3) mr_stage<3>(src, dst, tws, n, p, lpb, inverse);
    else if (R == 4) mr_stage<4>(src, dst, tws, n, p, lpb, inverse);
    else if (R == 5) mr_stage<5>(src, dst, tws, n, p, lpb, inverse);
    else if constexpr (MAXR >= 7) {
      if (R == 7) mr_stage<7>(src, dst, tws, n, p, lpb, inverse);
      else if constexpr (MAXR >= 13) {
        if (R == 11) mr_stage<11>(src, dst, tws, n, p, lpb, inverse);
        else mr_stage<13>(src, dst, tws, n, p, lpb, inverse);
      }
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
    p *= R;
  }
  return src;
}

// Lines addressed as in k_fft_lines; LDS: two buffers of lpb n points, the n twiddles, and the
// offset of each of the block's lines (formed once per line, not per point).
template <int MAXR>
__global__ __launch_bounds__(kFftThreads) void k_fft_lines_mr(double2* __restrict__ data, int n, MrPlan pl,
                                                              long long pstride, long long la, long long lb,
                                                              long long lc, long long nlines, int lpb,
                                                              const double2* __restrict__ tw, int inverse,
                                                              int contiguous, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  data = bat_at(data, bo);
  extern __shared__ double2 sm[];
  double2* b0 = sm;
  double2* b1 = sm + lpb * n;
  double2* tws = sm + 2 * lpb * n;
  long long* loff = reinterpret_cast<long long*>(tws + n);  // -1: past the last line
  for (int e = threadIdx.x; e < n; e += kFftThreads) tws[e] = tw[e];
  const long long line0 = (long long)blockIdx.x * lpb;
  for (int l = threadIdx.x; l < lpb; l += kFftThreads) {
    const long long line = line0 + l;
    loff[l] = (line < nlines) ? (line % la) * lb + (line / la) * lc : -1;
  }
  __syncthreads();
  const int total = lpb * n;
  for (int e = threadIdx.x; e < total; e += kFftThreads) {
    int l, q;
    if (contiguous) {
      l = e / n;
      q = e - l * n;
    } else {
      l = e % lpb;
      q = e / lpb;
    }
    const long long off = loff[l];
    b0[l * n + q] = (off >= 0) ? data[off + q * pstride] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double2* src = mr_lines<MAXR>(b0, b1, tws, n, lpb, pl, inverse);
  for (int e = threadIdx.x; e < total; e += kFftThreads) {
    int l, q;
    if (contiguous) {
      l = e / n;
      q = e - l * n;
    } else {
      l = e % lpb;
      q = e / lpb;
    }
    const long long off = loff[l];
    if (off >= 0) data[off + q * pstride] = src[l * n + q];
  }
}

// ---- fused 2D solve for sides that are not powers of two ---------------------------------
// The three passes of the power-of-two 2D path (rows forward with q = r_u + a Dhat z_c formed
// on the fly; column pairs (kx, nx - kx) forward, 2 x 2 symbol solve, inverse; rows inverse
// with the unpack), each line transformed in LDS by the mixed-radix stages above.  LDS per
// workgroup: two buffers of the block's lines and the line length's twiddles.

// pass 1: rows j0 .. j0 + nl - 1
template <typename T, int MAXR>
__global__ __launch_bounds__(kFftThreads) void k_fft2mr_rows_fwd(Consts K, const T* __restrict__ r, double a,
                                                                 const T* __restrict__ zc, int nl, MrPlan pl,
                                                                 const double2* __restrict__ tw,
                                                                 double2* __restrict__ out, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  r = bat_at(r, bo);
  zc = bat_at(zc, bo);
  out = bat_at(out, bo);
  extern __shared__ double2 sm[];
  const int n = K.nx;
  double2* b0 = sm;
  double2* b1 = sm + nl * n;
  double2* tws = sm + 2 * nl * n;
  for (int e = threadIdx.x; e < n; e += kFftThreads) tws[e] = tw[e];
  const int j0 = xcd_band(blockIdx.x, gridDim.x) * nl;
  for (int e = threadIdx.x; e < nl * n; e += kFftThreads) {
    const int l = e / n, i = e - l * n, j = j0 + l;
    const long long m = (long long)i + (long long)n * j;
    double qx = r ? (double)r[m] : 0.0, qy = r ? (double)r[K.N + m] : 0.0;
    if (zc && a != 0.0) {
      const int ip = (i + 1 == n) ? 0 : i + 1, im = (i == 0) ? n - 1 : i - 1;
      const int jp = (j + 1 == K.ny) ? 0 : j + 1, jm = (j == 0) ? K.ny - 1 : j - 1;
      qx += a * ((double)zc[ip + (long long)n * j] - (double)zc[im + (long long)n * j]) * K.i2h;
      qy += a * ((double)zc[i + (long long)n * jp] - (double)zc[i + (long long)n * jm]) * K.i2h;
    }
    b0[e] = make_double2(qx, qy);
  }
  __syncthreads();
  const double2* res = mr_lines<MAXR>(b0, b1, tws, n, nl, pl, 0);
  for (int e = threadIdx.x; e < nl * n; e += kFftThreads) {
    const int l = e / n, i = e - l * n;
    out[(long long)i + (long long)n * (j0 + l)] = res[e];
  }
}

// pass 2: block kx (0 .. nx/2 - 1) takes columns kx and nx - kx (block 0: 0 and nx/2)
template <int MAXR>
__global__ __launch_bounds__(kFftThreads) void k_fft2mr_cols_solve(Consts K, MrPlan pl,
                                                                   const double2* __restrict__ tw,
                                                                   const double* __restrict__ sx,
                                                                   const double* __restrict__ syt,
                                                                   double2* __restrict__ data, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  data = bat_at(data, binst * bt.stride);
  extern __shared__ double2 sm[];
  const int n = K.ny, nx = K.nx;
  double2* b0 = sm;
  double2* b1 = sm + 2 * n;
  double2* tws = sm + 4 * n;
  for (int e = threadIdx.x; e < n; e += kFftThreads) tws[e] = tw[e];
  const int kx = xcd_band(blockIdx.x, gridDim.x);
  const bool self = (kx == 0);
  const int kxm = self ? nx / 2 : nx - kx;
  for (int e = threadIdx.x; e < 2 * n; e += kFftThreads) {
    const int l = e / n, j = e - l * n;
    b0[e] = data[(long long)(l ? kxm : kx) + (long long)nx * j];
  }
  __syncthreads();
  double2* spec = mr_lines<MAXR>(b0, b1, tws, n, 2, pl, 0);
  double2* other = (spec == b0) ? b1 : b0;
  for (int e = threadIdx.x; e < 2 * n; e += kFftThreads) {
    const int l = e / n, j = e - l * n;
    const int col = l ? kxm : kx;
    const int lm = self ? l : 1 - l;   // the mirror column's line
    const int jm = (j == 0) ? 0 : n - j;
    other[e] = symbol_solve2(K, spec[e], spec[lm * n + jm], sx[col], syt[j]);
  }
  __syncthreads();
  const double2* res = mr_lines<MAXR>(other, spec, tws, n, 2, pl, 1);
  for (int e = threadIdx.x; e < 2 * n; e += kFftThreads) {
    const int l = e / n, j = e - l * n;
    data[(long long)(l ? kxm : kx) + (long long)nx * j] = res[e];
  }
}

// pass 3: inverse along x, u_x = Re / N, u_y = Im / N
template <typename T, int MAXR>
__global__ __launch_bounds__(kFftThreads) void k_fft2mr_rows_inv(Consts K, int nl, MrPlan pl,
                                                                 const double2* __restrict__ tw,
                                                                 const double2* __restrict__ in, T* __restrict__ u,
                                                                 Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  in = bat_at(in, bo);
  u = bat_at(u, bo);
  extern __shared__ double2 sm[];
  const int n = K.nx;
  double2* b0 = sm;
  double2* b1 = sm + nl * n;
  double2* tws = sm + 2 * nl * n;
  for (int e = threadIdx.x; e < n; e += kFftThreads) tws[e] = tw[e];
  const int j0 = xcd_band(blockIdx.x, gridDim.x) * nl;
  for (int e = threadIdx.x; e < nl * n; e += kFftThreads) {
    const int l = e / n, i = e - l * n;
    b0[e] = in[(long long)i + (long long)n * (j0 + l)];
  }
  __syncthreads();
  const double2* res = mr_lines<MAXR>(b0, b1, tws, n, nl, pl, 1);
  const double inv = 1.0 / (double)K.N;
  for (int e = threadIdx.x; e < nl * n; e += kFftThreads) {
    const int l = e / n, i = e - l * n;
    const long long m = (long long)i + (long long)n * (j0 + l);
    u[m] = (T)(res[e].x * inv);
    u[K.N + m] = (T)(res[e].y * inv);
  }
}

// q_I = r_I + a Dhat_I zc; z0 = q_1 + i q_2, z1 = q_3 (3D)
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_pack(Consts K, const T* __restrict__ r, double a,
                                              const T* __restrict__ zc, double2* __restrict__ z0,
                                              double2* __restrict__ z1, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  r = bat_at(r, bo);
  zc = bat_at(zc, bo);
  z0 = bat_at(z0, bo);
  z1 = bat_at(z1, bo);
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= K.N) return;
  {
    const int i = (int)(n % K.nx), j = (int)((n / K.nx) % K.ny), k = (int)(n / ((long long)K.nx * K.ny));
    double q[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int I = 0; I < DIM; ++I) {
      double v = r ? (double)r[I * K.N + n] : 0.0;
      if (zc && a != 0.0) {
        long long np, nm;
        if (I == 0) {
          np = wrapi(i + 1, K.nx) + (long long)K.nx * (j + (long long)K.ny * k);
          nm = wrapi(i - 1, K.nx) + (long long)K.nx * (j + (long long)K.ny * k);
        } else if (I == 1) {
          np = i + (long long)K.nx * (wrapi(j + 1, K.ny) + (long long)K.ny * k);
          nm = i + (long long)K.nx * (wrapi(j - 1, K.ny) + (long long)K.ny * k);
        } else {
          np = i + (long long)K.nx * (j + (long long)K.ny * wrapi(k + 1, K.nz));
          nm = i + (long long)K.nx * (j + (long long)K.ny * wrapi(k - 1, K.nz));
        }
        v += a * ((double)zc[np] - (double)zc[nm]) * K.i2h;
      }
      q[I] = v;
    }
    z0[n] = make_double2(q[0], q[1]);
    if (DIM == 3) z1[n] = make_double2(q[2], 0.0);
  }
}

// pointwise solve Khat uhat = qhat; w0 = uhat_1 + i uhat_2, w1 = uhat_3
template <int DIM>
__global__ __launch_bounds__(256) void k_symbol_solve(Consts K, const double2* __restrict__ z0,
                                                      const double2* __restrict__ z1,
                                                      double2* __restrict__ w0,
                                                      double2* __restrict__ w1,
                                                      const double* __restrict__ sx,
                                                      const double* __restrict__ sy,
                                                      const double* __restrict__ szt, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  z0 = bat_at(z0, bo);
  z1 = bat_at(z1, bo);
  w0 = bat_at(w0, bo);
  w1 = bat_at(w1, bo);
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= K.N) return;
  {
    const int i = (int)(n % K.nx), j = (int)((n / K.nx) % K.ny), k = (int)(n / ((long long)K.nx * K.ny));
    const long long nm = (long long)wrapi(-i, K.nx) +
                         (long long)K.nx * ((long long)wrapi(-j, K.ny) + (long long)K.ny * wrapi(-k, K.nz));
    double S[3];
    S[0] = sx[i];
    S[1] = sy[j];
    S[2] = (DIM == 3) ? szt[k] : 0.0;
    const double2 a = z0[n], b = z0[nm];
    // spectra of the two real fields packed in z0
    double2 Q[3];
    Q[0] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    Q[1] = make_double2(0.5 * (a.y + b.y), -0.5 * (a.x - b.x));
    Q[2] = (DIM == 3) ? z1[n] : make_double2(0.0, 0.0);
    double2 U[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    double s2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
    if (!K.elastic) {
#pragma unroll
      for (int I = 0; I < DIM; ++I) U[I] = Q[I];  // identity rows when there is no elasticity
    } else if (s2 != 0.0) {
      double A[3][3];
#pragma unroll
      for (int I = 0; I < DIM; ++I)
#pragma unroll
        for (int L = 0; L < DIM; ++L) {
          if (I == L) {
            A[I][I] = -(K.C11 * S[I] * S[I] + K.C44 * (s2 - S[I] * S[I]));
          } else {
            A[I][L] = -(K.C12 + K.C44) * S[I] * S[L];
          }
        }
      if (DIM == 2) {
        const double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        const double id = 1.0 / det;
        for (int c = 0; c < 2; ++c) {
          const double q0 = c ? Q[0].y : Q[0].x, q1 = c ? Q[1].y : Q[1].x;
          const double u0 = (A[1][1] * q0 - A[0][1] * q1) * id;
          const double u1 = (A[0][0] * q1 - A[1][0] * q0) * id;
          if (c) {
            U[0].y = u0;
            U[1].y = u1;
          } else {
            U[0].x = u0;
            U[1].x = u1;
          }
        }
      } else {
        // symmetric 3 x 3 by the adjugate
        const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        const double c01 = A[0][2] * A[2][1] - A[0][1] * A[2][2];
        const double c02 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
        const double c11 = A[0][0] * A[2][2] - A[0][2] * A[2][0];
        const double c12 = A[0][2] * A[1][0] - A[0][0] * A[1][2];
        const double c22 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        const double det = A[0][0] * c00 + A[0][1] * (A[1][2] * A[2][0] - A[1][0] * A[2][2]) +
                           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        const double id = 1.0 / det;
        const double Ai[3][3] = {{c00 * id, c01 * id, c02 * id},
                                 {c01 * id, c11 * id, c12 * id},
                                 {c02 * id, c12 * id, c22 * id}};
        for (int I = 0; I < 3; ++I) {
          double re = 0.0, im = 0.0;
          for (int L = 0; L < 3; ++L) {
            re += Ai[I][L] * Q[L].x;
            im += Ai[I][L] * Q[L].y;
          }
          U[I] = make_double2(re, im);
        }
      }
    }
    // u_1 + i u_2 has spectrum U_1 + i U_2
    w0[n] = make_double2(U[0].x - U[1].y, U[0].y + U[1].x);
    if (DIM == 3) w1[n] = U[2];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(Consts K, const double2* __restrict__ w0,
                                                const double2* __restrict__ w1,
                                                T* __restrict__ u, Bat bt) {
  const int binst = bat_inst(bt);
  if (bat_skip(bt, binst)) return;
  const long long bo = binst * bt.stride;
  w0 = bat_at(w0, bo);
  w1 = bat_at(w1, bo);
  u = bat_at(u, bo);
  const double inv = 1.0 / (double)K.N;
  for (long long n = (long long)blockIdx.x * 256 + threadIdx.x; n < K.N; n += (long long)gridDim.x * 256) {
    const double2 a = w0[n];
    u[n] = (T)(a.x * inv);
    u[K.N + n] = (T)(a.y * inv);
    if (K.dim == 3) u[2 * K.N + n] = (T)(w1[n].x * inv);
  }
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// k_fft_lines with its LDS: lpb lines and the n/2 twiddles (beyond 64 KiB for the longest lines)
void launch_lines(double2* data, int n, int logn, long long pstride, long long la, long long lb, long long lc,
                  long long nlines, int lpb, const double2* tw, int inverse, int contiguous, hipStream_t s,
                  const Bat& bt) {
  const size_t lds = sizeof(double2) * ((size_t)lp_size(lpb * n) + n / 2);
  if (lds > 64 * 1024) {
    allow_max_lds((const void*)k_fft_lines);
  }
  const long long blocks = (nlines + lpb - 1) / lpb;
  hipLaunchKernelGGL(k_fft_lines, bat_grid(dim3((unsigned)blocks), bt), dim3(kFftThreads), lds, s, data, n, logn,
                     pstride, la, lb, lc, nlines, lpb, tw, inverse, contiguous, bt);
}

bool pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }

// radices of a mixed-radix line: 4s, then a 2, then the odd primes ascending
MrPlan mr_plan(int n) {
  MrPlan pl{};
  auto add = [&](int r) { pl.r[pl.nst++] = r; };
  while (n % 4 == 0) { add(4); n /= 4; }
  while (n % 2 == 0) { add(2); n /= 2; }
  for (int f = 3; f <= 13 && n > 1; f += 2)
    while (n % f == 0) { add(f); n /= f; }
  return pl;
}

// the build of the mixed-radix kernels a plan needs: its largest radix, rounded up to 5, 7 or 13
int mr_bucket(const MrPlan& pl) {
  int m = 2;
  for (int st = 0; st < pl.nst; ++st) m = pl.r[st] > m ? pl.r[st] : m;
  return m <= 5 ? 5 : (m <= 7 ? 7 : 13);
}

void fft_dir_mr(const Consts& K, const FftPlan& P, double2* data, int dir, int inverse, hipStream_t s,
                const Bat& bt) {
  const int n = P.n[dir];
  const MrPlan pl = mr_plan(n);
  // two buffers of lpb lines plus n twiddles within 64 KiB; strided lines at most 16 adjacent
  int lpb = (4096 - n) / (2 * n);
  if (lpb < 1) lpb = 1;
  if (dir != 0 && lpb > 16) lpb = 16;
  long long nlines, la, lb, lc, pstride;
  const long long nx = K.nx, ny = K.ny;
  if (dir == 0) {
    nlines = ny * K.nz; la = 1; lb = 0; lc = nx; pstride = 1;
  } else if (dir == 1) {
    nlines = nx * K.nz; la = nx; lb = 1; lc = nx * ny; pstride = nx;
  } else {
    nlines = nx * ny; la = nx * ny; lb = 1; lc = 0; pstride = nx * ny;
  }
  if (dir != 0 && lpb > la) lpb = (int)la;
  // small grids: fewer lines per workgroup, so that the lines spread over more compute units
  // (at least 512 workgroups where the line count allows)
  while (lpb > 1 && (nlines + lpb - 1) / lpb < 512) lpb = (lpb + 1) / 2;
  const size_t lds = sizeof(double2) * ((size_t)2 * lpb * n + n) + sizeof(long long) * (size_t)lpb;
  const long long blocks = (nlines + lpb - 1) / lpb;
  auto go = [&](auto kern) {
    if (lds > 64 * 1024) allow_max_lds((const void*)kern);
    hipLaunchKernelGGL(kern, bat_grid(dim3((unsigned)blocks), bt), dim3(kFftThreads), lds, s, data, n, pl, pstride,
                       la, lb, lc, nlines, lpb, P.tw[dir], inverse, dir == 0 ? 1 : 0, bt);
  };
  const int mr = mr_bucket(pl);
  if (mr == 5) go(k_fft_lines_mr<5>);
  else if (mr == 7) go(k_fft_lines_mr<7>);
  else go(k_fft_lines_mr<13>);
}

void fft_dir(const Consts& K, const FftPlan& P, double2* data, int dir, int inverse, hipStream_t s,
             const Bat& bt) {
  const int n = P.n[dir];
  if (!pow2(n)) {
    fft_dir_mr(K, P, data, dir, inverse, s, bt);
    return;
  }
  const int logn = ilog2(n);
  // enough workgroups to fill the chip: one 256-butterfly stage per workgroup (n <= 512),
  // at least two adjacent lines for the strided passes (32-byte segments)
  // contiguous lines: enough per workgroup for one 256-butterfly stage (n <= 512); strided
  // lines: 16 adjacent ones, so that every row of the block reads 256 contiguous bytes
  int lpb = (dir == 0) ? 512 / n : 16;
  if (lpb < 1) lpb = 1;
  if (lpb * n > kFftLds) lpb = kFftLds / n;
  long long nlines, la, lb, lc, pstride;
  const long long nx = K.nx, ny = K.ny;
  if (dir == 0) {
    nlines = ny * K.nz;
    la = 1;
    lb = 0;
    lc = nx;
    pstride = 1;
  } else if (dir == 1) {
    nlines = nx * K.nz;
    la = nx;
    lb = 1;
    lc = nx * ny;
    pstride = nx;
  } else {
    nlines = nx * ny;
    la = nx * ny;
    lb = 1;
    lc = 0;
    pstride = nx * ny;
  }
  if (dir != 0 && lpb > la) lpb = (int)la;  // consecutive lines of a block stay adjacent
  launch_lines(data, n, logn, pstride, la, lb, lc, nlines, lpb, P.tw[dir], inverse, dir == 0 ? 1 : 0, s, bt);
}

void fft_all(const Consts& K, const FftPlan& P, double2* data, int inverse, hipStream_t s, const Bat& bt) {
  for (int dir = 0; dir < K.dim; ++dir) fft_dir(K, P, data, dir, inverse, s, bt);
}

int grid_n(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 4096 ? b : 4096);
}

}  // namespace

// u = K^{-1} (r + a Dhat zc) on the displacement block.  work0, work1: 2 N complex each in 3D
// (N each in 2D).  T: element type of r, zc and u (the transforms run in double).
template <typename T>
void launch_spectral_solve(const Consts& K, const FftPlan& P, const T* r, double a,
                           const T* zc, double2* work0, double2* work1, T* u,
                           hipStream_t s, const Bat& bt) {
  auto G = [&](unsigned blocks) { return bat_grid(dim3(blocks), bt); };
  const bool all_pow2 = pow2(K.nx) && pow2(K.ny) && pow2(K.nz);
  if (all_pow2 && K.dim == 2 && K.ny <= 1024 && K.nx <= 1024) {
    const int lx = ilog2(K.nx), ly = ilog2(K.ny);
    int nl = 512 / K.nx;  // rows per x block (one 512-point row: 512 blocks measured faster than 256)
    if (nl < 1) nl = 1;
    while (K.ny % nl) nl >>= 1;
    const size_t lrow = sizeof(double2) * (lp_size(nl * K.nx) + K.nx / 2);
    const size_t lcol = sizeof(double2) * (lp_size(4 * K.ny) + K.ny / 2);
    if (lcol > 64 * 1024) {  // ny = 1024: 80 KiB
      allow_max_lds((const void*)k_fft2_cols_solve);
    }
    hipLaunchKernelGGL(k_fft2_rows_fwd<T>, G(K.ny / nl), dim3(256), lrow, s, K, r, a, zc, lx, nl, P.tw[0], work0, bt);
    hipLaunchKernelGGL(k_fft2_cols_solve, G(K.nx / 2), dim3(256), lcol, s, K, ly, P.tw[1], P.sn[0],
                       P.sn[1], work0, bt);
    hipLaunchKernelGGL(k_fft2_rows_inv<T>, G(K.ny / nl), dim3(256), lrow, s, K, lx, nl, P.tw[0], work0, u, bt);
    return;
  }
  if (!all_pow2 && K.dim == 2 && K.ny <= 1024 && K.nx <= 1024) {
    const MrPlan px = mr_plan(K.nx), py = mr_plan(K.ny);
    // rows per x block: about 512 points (as the power-of-two rows), dividing ny
    int nl = 512 / K.nx;
    if (nl < 1) nl = 1;
    while (K.ny % nl) --nl;
    const size_t lrow = sizeof(double2) * ((size_t)2 * nl * K.nx + K.nx);
    const size_t lcol = sizeof(double2) * ((size_t)4 * K.ny + K.ny);
    auto rows = [&](auto kf, auto ki) {
      if (lrow > 64 * 1024) {
        allow_max_lds((const void*)kf);
        allow_max_lds((const void*)ki);
      }
      hipLaunchKernelGGL(kf, G(K.ny / nl), dim3(kFftThreads), lrow, s, K, r, a, zc, nl, px, P.tw[0], work0, bt);
      return ki;
    };
    auto cols = [&](auto kc) {
      if (lcol > 64 * 1024) allow_max_lds((const void*)kc);
      hipLaunchKernelGGL(kc, G(K.nx / 2), dim3(kFftThreads), lcol, s, K, py, P.tw[1], P.sn[0], P.sn[1], work0, bt);
    };
    const int bx = mr_bucket(px), by = mr_bucket(py);
    auto ki = (bx == 5) ? rows(k_fft2mr_rows_fwd<T, 5>, k_fft2mr_rows_inv<T, 5>)
              : (bx == 7) ? rows(k_fft2mr_rows_fwd<T, 7>, k_fft2mr_rows_inv<T, 7>)
                          : rows(k_fft2mr_rows_fwd<T, 13>, k_fft2mr_rows_inv<T, 13>);
    if (by == 5) cols(k_fft2mr_cols_solve<5>);
    else if (by == 7) cols(k_fft2mr_cols_solve<7>);
    else cols(k_fft2mr_cols_solve<13>);
    hipLaunchKernelGGL(ki, G(K.ny / nl), dim3(kFftThreads), lrow, s, K, nl, px, P.tw[0], work0, u, bt);
    return;
  }
  if (all_pow2 && K.dim == 3 && K.nx >= 8 && K.nx <= 1024 && K.nz <= 1024 && K.ny <= 4096) {
    const int lx = ilog2(K.nx), ly = ilog2(K.ny), lz = ilog2(K.nz);
    const int nxh = K.nx / 2 + 1;
    double2* Qh = work0;  // 3 nxh ny nz <= 2 N complex for nx >= 8
    int rp = 256 / K.nx;  // row pairs per x block: about 768 points per block
    if (rp < 1) rp = 1;
    while (rp > 1 && (K.ny / 2) % rp) rp >>= 1;
    const size_t lx_bytes = sizeof(double2) * (lp_size(3 * rp * K.nx) + K.nx / 2);
    const unsigned xblocks = (unsigned)((K.ny / (2 * rp)) * K.nz);
    int lpz = 1024 / K.nz;  // kx columns per z block: at most 53 KiB of LDS (three blocks per CU)
    if (lpz > 8) lpz = 8;
    if (lpz < 1) lpz = 1;
    while (lpz > 1 && sizeof(double2) * (lp_size(3 * lpz * K.nz) + K.nz / 2) > 53 * 1024) --lpz;
    const size_t lz_bytes = sizeof(double2) * (lp_size(3 * lpz * K.nz) + K.nz / 2);
    const unsigned zblocks = (unsigned)(((nxh + lpz - 1) / lpz) * K.ny);
    int lpy = kFftLds / K.ny;  // adjacent kx lines per y block
    if (lpy > 16) lpy = 16;
    const long long ylines = 3LL * nxh * K.nz;
    hipLaunchKernelGGL(k_r2c_x<T>, G(xblocks), dim3(256), lx_bytes, s, K, r, a, zc, lx, rp, P.tw[0], Qh, bt);
    launch_lines(Qh, K.ny, ly, nxh, nxh, 1, (long long)nxh * K.ny, ylines, lpy, P.tw[1], 0, 0, s, bt);
    hipLaunchKernelGGL(k_z_solve, G(zblocks), dim3(256), lz_bytes, s, K, lz, lpz, P.tw[2], P.sn[0], P.sn[1],
                       P.sn[2], Qh, bt);
    launch_lines(Qh, K.ny, ly, nxh, nxh, 1, (long long)nxh * K.ny, ylines, lpy, P.tw[1], 1, 0, s, bt);
    hipLaunchKernelGGL(k_c2r_x<T>, G(xblocks), dim3(256), lx_bytes, s, K, lx, rp, P.tw[0], Qh, u, bt);
    return;
  }
  double2* z0 = work0;
  double2* z1 = work0 + K.N;
  double2* w0 = work1;
  double2* w1 = work1 + K.N;
  const dim3 g3 = G((unsigned)((K.N + 255) / 256));
  if (K.dim == 2) hipLaunchKernelGGL((k_pack<2, T>), g3, dim3(256), 0, s, K, r, a, zc, z0, z1, bt);
  else hipLaunchKernelGGL((k_pack<3, T>), g3, dim3(256), 0, s, K, r, a, zc, z0, z1, bt);
  fft_all(K, P, z0, 0, s, bt);
  if (K.dim == 3) fft_all(K, P, z1, 0, s, bt);
  if (K.dim == 2)
    hipLaunchKernelGGL(k_symbol_solve<2>, g3, dim3(256), 0, s, K, z0, z1, w0, w1, P.sn[0], P.sn[1], P.sn[2], bt);
  else
    hipLaunchKernelGGL(k_symbol_solve<3>, g3, dim3(256), 0, s, K, z0, z1, w0, w1, P.sn[0], P.sn[1], P.sn[2], bt);
  fft_all(K, P, w0, 1, s, bt);
  if (K.dim == 3) fft_all(K, P, w1, 1, s, bt);
  hipLaunchKernelGGL(k_unpack<T>, G(grid_n(K.N)), dim3(256), 0, s, K, w0, w1, u, bt);
}

template void launch_spectral_solve<double>(const Consts&, const FftPlan&, const double*, double, const double*,
                                            double2*, double2*, double*, hipStream_t, const Bat&);
template void launch_spectral_solve<float>(const Consts&, const FftPlan&, const float*, double, const float*,
                                           double2*, double2*, float*, hipStream_t, const Bat&);

}  // namespace pf
