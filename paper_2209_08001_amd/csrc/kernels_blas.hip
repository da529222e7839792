// Vector kernels of the Krylov solver and the grid reductions of the Newton step.
//
// Every reduction is two-stage and deterministic: each of kRedBlocks workgroups writes one
// partial per value (partial[v * kRedBlocks + block]), then launch_finalize sums the partials
// in a fixed tree order.  No atomics, so results are bitwise reproducible run to run.
#include "pf_internal.h"

namespace pf {

namespace {

constexpr int kThreads = 256;

// two-element vector of the basis type (16-byte loads for double, 8-byte for float)
template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

// Sum of one value over the workgroup (wave64 shuffles, then the four waves via LDS).
__device__ inline double block_sum(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < kThreads / 64; ++w) r += lds[w];
  }
  return r;  // valid in thread 0
}

// Maximum of one non-negative value over the workgroup (valid in thread 0).
__device__ inline double block_max(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < kThreads / 64; ++w) r = fmax(r, lds[w]);
  }
  return r;
}

template <int MAXV, typename T>
__global__ __launch_bounds__(kThreads) void k_multidot(long long n, int nv, const T* __restrict__ V,
                                                       long long ldv, const double* __restrict__ w,
                                                       double* __restrict__ partial, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  V = bat_at(V, bi * bt.stride);
  w = bat_at(w, bi * bt.stride);
  partial = bat_at(partial, bi * bt.stride);
  __shared__ double lds[kThreads / 64];
  double acc[MAXV + 1];
#pragma unroll
  for (int v = 0; v <= MAXV; ++v) acc[v] = 0.0;
  // n and ldv are even and every vector is 16-byte aligned: two elements per load
  const long long n2 = n >> 1, ld2 = ldv >> 1;
  using T2 = typename Vec2<T>::type;
  const T2* __restrict__ V2 = reinterpret_cast<const T2*>(V);
  const double2* __restrict__ w2 = reinterpret_cast<const double2*>(w);
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n2;
       e += (long long)gridDim.x * kThreads) {
    const double2 we = w2[e];
#pragma unroll
    for (int v = 0; v < MAXV; ++v)
      if (MAXV <= 32 || v < nv) {
        const T2 y = V2[v * ld2 + e];
        acc[v] += we.x * (double)y.x + we.y * (double)y.y;
      }
    acc[MAXV] += we.x * we.x + we.y * we.y;
  }
  // every wave reduces all its values with shuffles; one barrier; then one thread per value
  __shared__ double wl[kThreads / 64][MAXV + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v <= MAXV; ++v) {
    if (MAXV <= 32 || v < nv || v == MAXV) {
      double x = acc[v];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) wl[wave][v] = x;
    }
  }
  (void)lds;
  __syncthreads();
  if ((int)threadIdx.x <= nv) {
    const int v = (threadIdx.x == (unsigned)nv) ? MAXV : threadIdx.x;
    double x = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) x += wl[w][v];
    partial[threadIdx.x * kRedBlocks + blockIdx.x] = x;
  }
}

struct Coefs {
  double c[kMaxRed];
};

// v_{j+1} = (w - sum_v h_v V_v) / h_{j+1,j} with the coefficients read from device memory
// (hc = [h_0 .. h_{nv-1}, <w, w>], written by the finalize of the multi-dot) and
// h_{j+1,j} = sqrt(<w,w> - sum h_v^2).
template <int MAXV, typename T>
__global__ __launch_bounds__(kThreads) void k_update_dev(long long n, int nv, const T* __restrict__ V,
                                                         long long ldv, const double* __restrict__ hc,
                                                         const double* __restrict__ w, T* __restrict__ out, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  V = bat_at(V, bi * bt.stride);
  hc = bat_at(hc, bi * bt.stride);
  w = bat_at(w, bi * bt.stride);
  out = bat_at(out, bi * bt.stride);
  double c[MAXV];
  double hh = 0.0;
#pragma unroll
  for (int v = 0; v < MAXV; ++v) {
    c[v] = (MAXV <= 32 || v < nv) ? hc[v] : 0.0;
    hh += c[v] * c[v];
  }
  const double scale = 1.0 / sqrt(hc[nv] - hh);
  const long long n2 = n >> 1, ld2 = ldv >> 1;
  using T2 = typename Vec2<T>::type;
  const T2* __restrict__ V2 = reinterpret_cast<const T2*>(V);
  const double2* __restrict__ w2 = reinterpret_cast<const double2*>(w);
  T2* __restrict__ o2 = reinterpret_cast<T2*>(out);
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n2;
       e += (long long)gridDim.x * kThreads) {
    double2 x = w2[e];
#pragma unroll
    for (int v = 0; v < MAXV; ++v)
      if (MAXV <= 32 || v < nv) {
        const T2 y = V2[v * ld2 + e];
        x.x -= c[v] * (double)y.x;
        x.y -= c[v] * (double)y.y;
      }
    T2 o;
    o.x = (T)(scale * x.x);
    o.y = (T)(scale * x.y);
    o2[e] = o;
  }
}

template <int MAXV, typename T, typename To>
__global__ __launch_bounds__(kThreads) void k_lincomb(long long n, int nv, const T* __restrict__ V,
                                                      long long ldv, Coefs cf, double beta,
                                                      To* __restrict__ out, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  V = bat_at(V, bi * bt.stride);
  out = bat_at(out, bi * bt.stride);
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (long long)gridDim.x * kThreads) {
    double x = (beta == 0.0) ? 0.0 : beta * (double)out[e];
#pragma unroll
    for (int v = 0; v < MAXV; ++v)
      if (MAXV <= 32 || v < nv) x += cf.c[v] * (double)V[v * ldv + e];
    out[e] = (To)x;
  }
}

template <typename Tx, typename Ty, typename To>
__global__ __launch_bounds__(kThreads) void k_axpby(long long n, double a, const Tx* __restrict__ x,
                                                    double b, const Ty* __restrict__ y,
                                                    To* __restrict__ out, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  x = bat_at(x, bi * bt.stride);
  y = bat_at(y, bi * bt.stride);
  out = bat_at(out, bi * bt.stride);
  a = bat_s(bt, bi, a);
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (long long)gridDim.x * kThreads) {
    double v = a * (double)x[e];
    if (b != 0.0) v += b * (double)y[e];
    out[e] = (To)v;
  }
}

// Second stage: one thread per partial (kRedBlocks threads), every value loaded at once
// (independent loads in flight), wave shuffle trees, then one thread per value sums the
// waves.  Fixed order, so the result is deterministic.
template <int MAXV>
__global__ __launch_bounds__(kRedBlocks) void k_finalize(const double* __restrict__ partial, int nvals,
                                                         double* __restrict__ out, double* __restrict__ out2,
                                                         Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  partial = bat_at(partial, bi * bt.stride);
  out = bat_at(out, bi * bt.stride);
  out2 = bat_at(out2, bi * bt.hstride);
  __shared__ double wl[kRedBlocks / 64][MAXV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[MAXV];
#pragma unroll
  for (int v = 0; v < MAXV; ++v) acc[v] = (MAXV <= 32 || v < nvals) ? partial[v * kRedBlocks + threadIdx.x] : 0.0;
#pragma unroll
  for (int v = 0; v < MAXV; ++v) {
    if (MAXV <= 32 || v < nvals) {
      double x = acc[v];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) wl[wave][v] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nvals) {
    double x = 0.0;
    for (int w = 0; w < kRedBlocks / 64; ++w) x += wl[w][threadIdx.x];
    out[threadIdx.x] = x;
    if (out2) out2[threadIdx.x] = x;
  }
}

// The same second stage for per-block maxima of non-negative values.
constexpr int kMaxVals = 16;
__global__ __launch_bounds__(kRedBlocks) void k_finalize_max(const double* __restrict__ partial, int nvals,
                                                             double* __restrict__ out, double* __restrict__ out2,
                                                             Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  partial = bat_at(partial, bi * bt.stride);
  out = bat_at(out, bi * bt.stride);
  out2 = bat_at(out2, bi * bt.hstride);
  __shared__ double wl[kRedBlocks / 64][kMaxVals];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = 0; v < nvals; ++v) {
    double x = partial[v * kRedBlocks + threadIdx.x];
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
    if (lane == 0) wl[wave][v] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < nvals) {
    double x = 0.0;
    for (int w = 0; w < kRedBlocks / 64; ++w) x = fmax(x, wl[w][threadIdx.x]);
    out[threadIdx.x] = x;
    if (out2) out2[threadIdx.x] = x;
  }
}

// sum of x, and sum of (y - yn): the two means of the mass projection of a Newton update
__global__ __launch_bounds__(kThreads) void k_sum2(long long n, const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ yn,
                                                   double* __restrict__ partial, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  x = bat_at(x, bi * bt.stride);
  y = bat_at(y, bi * bt.stride);
  yn = bat_at(yn, bi * bt.stride);
  partial = bat_at(partial, bi * bt.stride);
  __shared__ double lds[kThreads / 64];
  double a = 0.0, b = 0.0;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (long long)gridDim.x * kThreads) {
    a += x[e];
    b += y[e] - yn[e];
  }
  double sa = block_sum(a, lds);
  double sb = block_sum(b, lds);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = sa;
    partial[kRedBlocks + blockIdx.x] = sb;
  }
}

// Trial point of the line search, X_t = X + lam (S + shift e_c), with the log-domain check
// 0 < c < 1, 0 < c eta_i < 1 (i = 1..4, eta_4 = 4 - eta_1 - eta_2 - eta_3).
// pmax (may be null): per-block maxima of |S_f + shift_f| and |X_f| of every field f, for the
// update test of the Newton stop (values 2 f and 2 f + 1, kRedBlocks apart).
__global__ __launch_bounds__(kThreads) void k_trial(long long N, int nf, const double* __restrict__ X,
                                                    const double* __restrict__ S, double lam,
                                                    const double* __restrict__ msums, double* __restrict__ Xt,
                                                    double* __restrict__ partial, double* __restrict__ pmax,
                                                    Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  const long long bo = bi * bt.stride;
  X = bat_at(X, bo);
  S = bat_at(S, bo);
  msums = bat_at(msums, bo);
  Xt = bat_at(Xt, bo);
  partial = bat_at(partial, bo);
  pmax = bat_at(pmax, bo);
  lam = bat_s(bt, bi, lam);
  __shared__ double lds[kThreads / 64];
  // mass projection of the update: shift = -(sum S_c + sum (c - c^n)) / N, from the device sums
  const double shift = -(msums[0] + msums[1]) / (double)N;
  double bad = 0.0;
  double ms[7] = {0, 0, 0, 0, 0, 0, 0}, mx[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < N;
       e += (long long)gridDim.x * kThreads) {
    const double sc = S[e] + shift, xc = X[e];
    const double c = xc + lam * sc;
    Xt[e] = c;
    ms[0] = fmax(ms[0], fabs(sc));
    mx[0] = fmax(mx[0], fabs(xc));
    double esum = 0.0;
    double prod_ok = (c > 0.0 && c < 1.0) ? 1.0 : 0.0;
#pragma unroll
    for (int p = 1; p <= 3; ++p) {
      const double sp = S[p * N + e], xp = X[p * N + e];
      const double ep = xp + lam * sp;
      Xt[p * N + e] = ep;
      ms[p] = fmax(ms[p], fabs(sp));
      mx[p] = fmax(mx[p], fabs(xp));
      esum += ep;
      const double y = c * ep;
      if (!(y > 0.0 && y < 1.0)) prod_ok = 0.0;
    }
    const double y4 = c * (4.0 - esum);
    if (!(y4 > 0.0 && y4 < 1.0)) prod_ok = 0.0;
#pragma unroll
    for (int f = 4; f < 7; ++f) {
      if (f < nf) {
        const double sf = S[f * N + e], xf = X[f * N + e];
        Xt[f * N + e] = xf + lam * sf;
        ms[f] = fmax(ms[f], fabs(sf));
        mx[f] = fmax(mx[f], fabs(xf));
      }
    }
    bad += 1.0 - prod_ok;
  }
  double s = block_sum(bad, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
  if (pmax) {
#pragma unroll
    for (int f = 0; f < 7; ++f) {
      if (f < nf) {
        const double a = block_max(ms[f], lds);
        if (threadIdx.x == 0) pmax[(2 * f) * kRedBlocks + blockIdx.x] = a;
        const double b = block_max(mx[f], lds);
        if (threadIdx.x == 0) pmax[(2 * f + 1) * kRedBlocks + blockIdx.x] = b;
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_dx2(long long n, const double* __restrict__ X,
                                                  const double* __restrict__ Xn,
                                                  double* __restrict__ partial, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  X = bat_at(X, bi * bt.stride);
  Xn = bat_at(Xn, bi * bt.stride);
  partial = bat_at(partial, bi * bt.stride);
  __shared__ double lds[kThreads / 64];
  double a = 0.0;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (long long)gridDim.x * kThreads) {
    const double d = X[e] - Xn[e];
    a += d * d;
  }
  double s = block_sum(a, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sums of each displacement component over each parity class (i mod 2, j mod 2, k mod 2).
__global__ __launch_bounds__(kThreads) void k_class_sums(Consts K, const double* __restrict__ u,
                                                         double* __restrict__ partial, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  u = bat_at(u, bi * bt.stride);
  partial = bat_at(partial, bi * bt.stride);
  __shared__ double lds[kThreads / 64];
  const int ncls = 1 << K.dim;
  double acc[3][8];
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[I][c] = 0.0;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < K.N;
       e += (long long)gridDim.x * kThreads) {
    const long long i = e % K.nx, t = e / K.nx, j = t % K.ny, k = t / K.ny;
    const int cls = (int)((i & 1) | ((j & 1) << 1) | ((k & 1) << 2));
#pragma unroll
    for (int I = 0; I < 3; ++I) {
      const double v = (I < K.dim) ? u[I * K.N + e] : 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c == cls) acc[I][c] += v;
    }
  }
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (I < K.dim && c < ncls) {
        double s = block_sum(acc[I][c], lds);
        if (threadIdx.x == 0) partial[(I * ncls + c) * kRedBlocks + blockIdx.x] = s;
      }
    }
}

__global__ __launch_bounds__(kThreads) void k_class_shift(Consts K, double* __restrict__ u,
                                                          const double* __restrict__ sums, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  u = bat_at(u, bi * bt.stride);
  sums = bat_at(sums, bi * bt.stride);
  const int ncls = 1 << K.dim;
  const double inv = (double)ncls / (double)K.N;  // every class holds N / 2^d nodes
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < K.N;
       e += (long long)gridDim.x * kThreads) {
    const long long i = e % K.nx, t = e / K.nx, j = t % K.ny, k = t / K.ny;
    const int cls = (int)((i & 1) | ((j & 1) << 1) | ((k & 1) << 2));
    for (int I = 0; I < K.dim; ++I) u[I * K.N + e] -= sums[I * ncls + cls] * inv;
  }
}

// ---- device-side GMRES cycle of a lockstep batch (pfnks_group) -----------------------
// Arnoldi column j, one workgroup per instance: the second stage of the multi-dot (as
// k_finalize) into hcol = [h_0 .. h_j, <w, w>], then, in thread 0, h_{j+1,j} =
// sqrt(<w,w> - sum h_i^2), the earlier Givens rotations and a new one applied to column j of
// H and to the rotated right-hand side g, and the end test of the cycle: |g_{j+1}| <= tol,
// the loss of more than two digits in <w,w> - sum h_i^2, a zero h_{j+1,j}, the column limit
// of the cycle, or an estimate that is not finite.  The status goes to the instance's state
// and to its pinned host slots (ended, |g_{j+1}|, columns, not finite).  An instance whose
// cycle has already ended (a step launched ahead of the host's test) is left untouched.
template <int MAXV>
__global__ __launch_bounds__(kRedBlocks) void k_arnoldi(const double* __restrict__ partial, int j, int m,
                                                        double* __restrict__ hcol, double* __restrict__ giv,
                                                        double* __restrict__ host, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  partial = bat_at(partial, bi * bt.stride);
  hcol = bat_at(hcol, bi * bt.stride);
  giv = bat_at(giv, bi * bt.stride);
  host = bat_at(host, bi * bt.hstride);
  const GivLayout L = giv_layout(m);
  double* st = giv + L.st;
  if (st[kGivEnded] != 0.0) return;
  // what thread 0's rotation step reads from the state, loaded before anything is stored to
  // it (the loads then overlap the reduction instead of waiting behind the stores)
  double gj = 0.0, tol = 0.0, lim = 0.0;
  if (threadIdx.x == 0) {
    gj = giv[L.g + j];
    tol = st[kGivTol];
    lim = st[kGivLim];
  }
  const int nvals = j + 2;
  __shared__ double wl[kRedBlocks / 64][MAXV];
  __shared__ double col[MAXV];
  // the earlier rotations, staged in LDS by all threads (thread 0's rotation loop then waits on
  // LDS, not on a global load behind each of its own stores)
  __shared__ double rc[kMaxRed], rs[kMaxRed];
  for (int i = threadIdx.x; i < j; i += kRedBlocks) {
    rc[i] = giv[L.cs + i];
    rs[i] = giv[L.sn + i];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[MAXV];
#pragma unroll
  for (int v = 0; v < MAXV; ++v) acc[v] = (MAXV <= 32 || v < nvals) ? partial[v * kRedBlocks + threadIdx.x] : 0.0;
#pragma unroll
  for (int v = 0; v < MAXV; ++v) {
    if (MAXV <= 32 || v < nvals) {
      double x = acc[v];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) wl[wave][v] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nvals) {
    double x = 0.0;
    for (int w = 0; w < kRedBlocks / 64; ++w) x += wl[w][threadIdx.x];
    hcol[threadIdx.x] = x;
    col[threadIdx.x] = x;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double* g = giv + L.g;
  double* h = giv + L.H + (long long)j * (m + 1);
  double hh = 0.0;
  for (int i = 0; i <= j; ++i) hh += col[i] * col[i];
  const double ww = col[j + 1];
  const double nrm2 = ww - hh;
  const bool cancel = !(nrm2 > 1e-2 * ww);
  const double hnext = sqrt(fmax(nrm2, 0.0));
  // the earlier rotations applied to column j, the rotated entry carried in a register
  double a = col[0];
  for (int i = 0; i < j; ++i) {
    const double b = col[i + 1];
    h[i] = rc[i] * a + rs[i] * b;
    a = -rs[i] * a + rc[i] * b;
  }
  const double b = hnext;
  const double r = hypot(a, b);
  const double c_ = (r == 0.0) ? 1.0 : a / r;
  const double s_ = (r == 0.0) ? 0.0 : b / r;
  giv[L.cs + j] = c_;
  giv[L.sn + j] = s_;
  h[j] = r;
  h[j + 1] = 0.0;
  g[j + 1] = -s_ * gj;
  g[j] = c_ * gj;
  const double resid = fabs(-s_ * gj);
  const bool nonfinite = !isfinite(resid);
  const bool ended = nonfinite || resid <= tol || cancel || hnext == 0.0 || (double)(j + 1) >= lim;
  st[kGivEnded] = ended ? 1.0 : 0.0;
  st[kGivCols] = (double)(j + 1);
  st[kGivResid] = resid;
  st[kGivNonfinite] = nonfinite ? 1.0 : 0.0;
  host[0] = ended ? 1.0 : 0.0;
  host[1] = resid;
  host[2] = (double)(j + 1);
  host[3] = nonfinite ? 1.0 : 0.0;
}

// start of a cycle, per instance: g = beta e_1 (beta = bt.s), tolerance bt.s2, column limit
// bt.s3, nothing ended yet
__global__ __launch_bounds__(64) void k_giv_init(double* __restrict__ giv, int m, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  giv = bat_at(giv, bi * bt.stride);
  const GivLayout L = giv_layout(m);
  for (int i = threadIdx.x; i <= m; i += 64) giv[L.g + i] = (i == 0) ? bt.s[bi] : 0.0;
  if (threadIdx.x == 0) {
    double* st = giv + L.st;
    st[kGivEnded] = 0.0;
    st[kGivCols] = 0.0;
    st[kGivTol] = bt.s2[bi];
    st[kGivLim] = bt.s3[bi];
    st[kGivResid] = bt.s[bi];
    st[kGivNonfinite] = 0.0;
  }
}

// end of a cycle, per instance: y = H^{-1} g over the cycle's k columns (upper triangular),
// zero beyond, and y[m] = k for the combination S += Z y
// (H, g and y staged in LDS by the workgroup; thread 0 runs the back substitution there)
constexpr int kMaxRestart = 64;
__global__ __launch_bounds__(256) void k_ysolve(double* __restrict__ giv, int m, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  giv = bat_at(giv, bi * bt.stride);
  const GivLayout L = giv_layout(m);
  __shared__ double Hs[kMaxRestart * kMaxRestart], gs[kMaxRestart], ys[kMaxRestart];
  const int k = (int)giv[L.st + kGivCols];
  // the leading k x k block of H (column c at c (m + 1)), row-major in LDS, and g
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int c = e / k, i = e - c * k;
    Hs[i * kMaxRestart + c] = giv[L.H + (long long)c * (m + 1) + i];
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = giv[L.g + i];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double s_ = gs[i];
      for (int c = i + 1; c < k; ++c) s_ -= Hs[i * kMaxRestart + c] * ys[c];
      ys[i] = s_ / Hs[i * kMaxRestart + i];
    }
  }
  __syncthreads();
  double* y = giv + L.y;
  for (int i = threadIdx.x; i < m; i += blockDim.x) y[i] = (i < k) ? ys[i] : 0.0;
  if (threadIdx.x == 0) y[m] = (double)k;
}

// out += sum_{v < k} y_v V_v with each instance's own y and column count k (from k_ysolve);
// nv: the largest k of the launch
template <int MAXV, typename T, typename To>
__global__ __launch_bounds__(kThreads) void k_lincomb_dev(long long n, int nv, const T* __restrict__ V,
                                                          long long ldv, const double* __restrict__ giv, int m,
                                                          To* __restrict__ out, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  V = bat_at(V, bi * bt.stride);
  giv = bat_at(giv, bi * bt.stride);
  out = bat_at(out, bi * bt.stride);
  const double* y = giv + giv_layout(m).y;
  const int k = (int)y[m];
  const int nvb = k < nv ? k : nv;
  double c[MAXV];
#pragma unroll
  for (int v = 0; v < MAXV; ++v) c[v] = (v < nvb) ? y[v] : 0.0;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (long long)gridDim.x * kThreads) {
    double x = (double)out[e];
#pragma unroll
    for (int v = 0; v < MAXV; ++v)
      if (v < nvb) x += c[v] * (double)V[v * ldv + e];
    out[e] = (To)x;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_zero(long long n, T* __restrict__ out, Bat bt) {
  const int bi = bat_inst(bt);
  if (bat_skip(bt, bi)) return;
  out = bat_at(out, bi * bt.stride);
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < n;
       e += (long long)gridDim.x * kThreads)
    out[e] = T(0);
}

int grid_for(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  return (int)(b < kRedBlocks ? b : kRedBlocks);
}

dim3 bg(int x, const Bat& bt) { return bat_grid(dim3((unsigned)x), bt); }

}  // namespace

// Exact-count instantiations (every guarded load is then unconditional and all of them can be
// in flight at once); counts above 32 use the 64-wide guarded form.
#define PF_NV_CASES(F)                                                                        \
  case 1: F(1); break; case 2: F(2); break; case 3: F(3); break; case 4: F(4); break;         \
  case 5: F(5); break; case 6: F(6); break; case 7: F(7); break; case 8: F(8); break;         \
  case 9: F(9); break; case 10: F(10); break; case 11: F(11); break; case 12: F(12); break;   \
  case 13: F(13); break; case 14: F(14); break; case 15: F(15); break; case 16: F(16); break; \
  case 17: F(17); break; case 18: F(18); break; case 19: F(19); break; case 20: F(20); break; \
  case 21: F(21); break; case 22: F(22); break; case 23: F(23); break; case 24: F(24); break; \
  case 25: F(25); break; case 26: F(26); break; case 27: F(27); break; case 28: F(28); break; \
  case 29: F(29); break; case 30: F(30); break; case 31: F(31); break; case 32: F(32); break; \
  default: F(64);

// partial receives nv + 1 values: <w, V_v> for v < nv and <w, w>.  Always kRedBlocks blocks.
template <typename T>
void launch_multidot(long long n, int nv, const T* V, long long ldv, const double* w, double* partial,
                     hipStream_t s, const Bat& bt) {
  if (nv == 0) {
    hipLaunchKernelGGL((k_multidot<0, T>), bg(kRedBlocks, bt), dim3(kThreads), 0, s, n, nv, V, ldv, w, partial, bt);
    return;
  }
#define F(N) hipLaunchKernelGGL((k_multidot<N, T>), bg(kRedBlocks, bt), dim3(kThreads), 0, s, n, nv, V, ldv, w, partial, bt)
  switch (nv) { PF_NV_CASES(F) }
#undef F
}
template void launch_multidot<double>(long long, int, const double*, long long, const double*, double*, hipStream_t,
                                      const Bat&);
template void launch_multidot<float>(long long, int, const float*, long long, const double*, double*, hipStream_t,
                                     const Bat&);

template <typename T>
void launch_update_dev(long long n, int nv, const T* V, long long ldv, const double* hc, const double* w,
                       T* out, hipStream_t s, const Bat& bt) {
#define F(N) hipLaunchKernelGGL((k_update_dev<N, T>), bg(kRedBlocks, bt), dim3(kThreads), 0, s, n, nv, V, ldv, hc, w, out, bt)
  switch (nv) { PF_NV_CASES(F) }
#undef F
}
template void launch_update_dev<double>(long long, int, const double*, long long, const double*, const double*,
                                        double*, hipStream_t, const Bat&);
template void launch_update_dev<float>(long long, int, const float*, long long, const double*, const double*,
                                       float*, hipStream_t, const Bat&);

// out = beta * out + sum_v coef[v] V_v
template <typename T, typename To>
void launch_lincomb(long long n, int nv, const T* V, long long ldv, const double* coef, double beta, To* out,
                    hipStream_t s, const Bat& bt) {
  Coefs cf{};
  for (int v = 0; v < nv; ++v) cf.c[v] = coef[v];
#define F(N) hipLaunchKernelGGL((k_lincomb<N, T, To>), bg(grid_for(n), bt), dim3(kThreads), 0, s, n, nv, V, ldv, cf, beta, out, bt)
  switch (nv) { PF_NV_CASES(F) }
#undef F
}
template void launch_lincomb<double, double>(long long, int, const double*, long long, const double*, double,
                                             double*, hipStream_t, const Bat&);
template void launch_lincomb<float, double>(long long, int, const float*, long long, const double*, double,
                                            double*, hipStream_t, const Bat&);

template <typename Tx, typename Ty, typename To>
void launch_axpby(long long n, double a, const Tx* x, double b, const Ty* y, To* out, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL((k_axpby<Tx, Ty, To>), bg(grid_for(n), bt), dim3(kThreads), 0, s, n, a, x, b, y, out, bt);
}
template void launch_axpby<double, double, double>(long long, double, const double*, double, const double*,
                                                   double*, hipStream_t, const Bat&);
template void launch_axpby<double, double, float>(long long, double, const double*, double, const double*, float*,
                                                  hipStream_t, const Bat&);
template void launch_axpby<float, float, float>(long long, double, const float*, double, const float*, float*,
                                                hipStream_t, const Bat&);
template void launch_axpby<float, float, double>(long long, double, const float*, double, const float*, double*,
                                                 hipStream_t, const Bat&);

void launch_finalize(const double* partial, int nvals, double* out, hipStream_t s, double* out2, const Bat& bt) {
#define F(N) hipLaunchKernelGGL(k_finalize<N>, bg(1, bt), dim3(kRedBlocks), 0, s, partial, nvals, out, out2, bt)
  if (nvals > 32) {
    F(80);
    return;
  }
  switch (nvals) { PF_NV_CASES(F) }
#undef F
}

void launch_finalize_max(const double* partial, int nvals, double* out, hipStream_t s, double* out2,
                         const Bat& bt) {
  hipLaunchKernelGGL(k_finalize_max, bg(1, bt), dim3(kRedBlocks), 0, s, partial, nvals, out, out2, bt);
}

void launch_sum2(long long n, const double* x, const double* y, const double* yn, double* partial,
                 hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_sum2, bg(kRedBlocks, bt), dim3(kThreads), 0, s, n, x, y, yn, partial, bt);
}

void launch_trial(const Consts& K, int nf, const double* X, const double* S, double lam,
                  const double* msums, double* Xt, double* partial, double* pmax, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_trial, bg(kRedBlocks, bt), dim3(kThreads), 0, s, K.N, nf, X, S, lam, msums,
                     Xt, partial, pmax, bt);
}

void launch_dx2(long long n4, const double* X, const double* Xn, double* partial, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_dx2, bg(kRedBlocks, bt), dim3(kThreads), 0, s, n4, X, Xn, partial, bt);
}

void launch_class_sums(const Consts& K, const double* u, double* partial, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_class_sums, bg(kRedBlocks, bt), dim3(kThreads), 0, s, K, u, partial, bt);
}

void launch_class_shift(const Consts& K, double* u, const double* sums, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_class_shift, bg(grid_for(K.N), bt), dim3(kThreads), 0, s, K, u, sums, bt);
}

void launch_arnoldi(const double* partial, int j, int m, double* hcol, double* giv, double* host, hipStream_t s,
                    const Bat& bt) {
  const int nvals = j + 2;
#define F(N) hipLaunchKernelGGL(k_arnoldi<N>, bg(1, bt), dim3(kRedBlocks), 0, s, partial, j, m, hcol, giv, host, bt)
  if (nvals > 32) {
    F(80);
    return;
  }
  switch (nvals) { PF_NV_CASES(F) }
#undef F
}

void launch_giv_init(double* giv, int m, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_giv_init, bg(1, bt), dim3(64), 0, s, giv, m, bt);
}

void launch_ysolve(double* giv, int m, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_ysolve, bg(1, bt), dim3(256), 0, s, giv, m, bt);
}

template <typename T, typename To>
void launch_lincomb_dev(long long n, int nv, const T* V, long long ldv, const double* giv, int m, To* out,
                        hipStream_t s, const Bat& bt) {
#define F(N) hipLaunchKernelGGL((k_lincomb_dev<N, T, To>), bg(grid_for(n), bt), dim3(kThreads), 0, s, n, nv, V, ldv, giv, m, out, bt)
  switch (nv) { PF_NV_CASES(F) }
#undef F
}
template void launch_lincomb_dev<double, double>(long long, int, const double*, long long, const double*, int,
                                                 double*, hipStream_t, const Bat&);
template void launch_lincomb_dev<float, double>(long long, int, const float*, long long, const double*, int,
                                                double*, hipStream_t, const Bat&);

template <typename T>
void launch_fill_zero(long long n, T* out, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL((k_fill_zero<T>), bg(grid_for(n), bt), dim3(kThreads), 0, s, n, out, bt);
}
template void launch_fill_zero<double>(long long, double*, hipStream_t, const Bat&);
template void launch_fill_zero<float>(long long, float*, hipStream_t, const Bat&);

}  // namespace pf
