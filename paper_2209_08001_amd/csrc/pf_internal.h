// Internal declarations of the pfnks library: the per-problem constant block the kernels
// read and the host-side launch wrappers.  Not part of the public ABI (include/pfnks.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <mutex>
#include <unordered_set>

namespace pf {

constexpr int kMaxS = 30;         // largest order of the Psi_S quotient
constexpr int kRedBlocks = 1024;  // partial sums of the two-stage grid reductions
constexpr int kMaxRed = 80;       // values reduced in one pass (GMRES multi-dot: j + 2 <= 66)

// Everything a kernel needs to know about the grid and the model.  Passed by value.
struct Consts {
  int dim;
  int nx, ny, nz;        // nodes per direction (nz = 1 in 2D)
  long long N;           // nodes
  double h, ih, ih2;     // h, 1/h, 1/h^2
  double i2h;            // 1/(2h)
  // chemical energy, dimensionless (Appendix A)
  double pc[6];          // p(c) = sum pc[m] c^m   (e0 c + c(1-c) sum L_k (2c-1)^k)
  double A2, A3;         // A(c) = A2 c^2 + A3 c^3  (sum phi^2 coefficient)
  double B3;             // B(c) = B3 c^3           (phi1 phi2 phi3 coefficient)
  double theta, w_c;
  double gamma_c, gamma_eta, kappa, L_eta;
  double eps0, cbar0;
  double C11, C12, C44;  // already multiplied by Lscale
  double Ctr;            // C11 + (d-1) C12: sum_I sigma_II = Ctr * trace(eps)
  double kel;            // (d/2) eps0^2 Ctr: d/dc^{n+1} of -eps0 * trace(sigma_bar)
  int elastic;           // 0: Lscale = 0, the displacement rows become u = 0
  int S;
  double qs[kMaxS];      // qs[j-1] = 1/(2j(2j+1)), j = 1..S-1  (coefficients of P)
  double qd[kMaxS];      // qd[j-1] = 1/(2(2j+1))               (coefficients of P')
};

// ---- lockstep batches of one grid shape (pfnks_group) --------------------------------
// A launch may cover several problems of one shape at once.  Instance b's workspace starts
// b * stride bytes after instance 0's, so every pointer argument points into instance 0's
// workspace and a workgroup of instance b adds b * stride; pinned host slots (the second
// output of the finalize kernels) are hstride bytes apart.  The slowest grid axis (z) is
// split into count equal parts, one per launched instance: part k works on instance map[k]
// (only the instances a phase still works on are launched); a workgroup whose instance has its
// bit of mask clear returns at once.  Tables that every instance shares (twiddles, Fourier
// symbols, colour order) are read from instance 0.  A single problem is the batch of one.
// With per = 1 the per-instance scalars replace a launch's scalar argument: s is the time
// step of the stencil, tile and residual launches, the coefficient a of axpby and the step
// length of the line-search trial; cb is the mean composition cbar0 of each instance (the
// eigenstrain reference of the residual and the energy).
constexpr int kMaxBatch = 32;
struct Bat {
  long long stride = 0;
  long long hstride = 0;
  int count = 1;
  int per = 0;
  unsigned mask = 0xffffffffu;
  unsigned char map[kMaxBatch] = {0,  1,  2,  3,  4,  5,  6,  7,  8,  9,  10, 11, 12, 13, 14, 15,
                                  16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31};
  double s[kMaxBatch] = {};
  double s2[kMaxBatch] = {};
  double s3[kMaxBatch] = {};
  double cb[kMaxBatch] = {};
};

// the grid of a launch over every instance of bt (z multiplied by the instance count)
inline dim3 bat_grid(dim3 g, const Bat& bt) {
  g.z *= (unsigned)bt.count;
  return g;
}
// p moved by off bytes; null stays null (optional arguments)
template <typename T>
__host__ __device__ inline T* bat_at(T* p, long long off) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<char*>(p) + off) : p;
}
template <typename T>
__host__ __device__ inline const T* bat_at(const T* p, long long off) {
  return p ? reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off) : p;
}
// Per-instance state of the device-side GMRES cycle of a lockstep batch: the Hessenberg
// matrix H ((m + 1) x m, column j at j (m + 1)), the Givens rotations cs, sn, the rotated
// right-hand side g (m + 1), the cycle's solution y (m + 1; y[m] = its column count) and a
// status block (kGiv*).
struct GivLayout {
  long long H, cs, sn, g, y, st, total;
};
__host__ __device__ inline GivLayout giv_layout(int m) {
  GivLayout L;
  L.H = 0;
  L.cs = L.H + (long long)(m + 1) * m;
  L.sn = L.cs + m;
  L.g = L.sn + m;
  L.y = L.g + m + 1;
  L.st = L.y + m + 1;
  L.total = L.st + 8;
  return L;
}
constexpr int kGivEnded = 0, kGivCols = 1, kGivTol = 2, kGivLim = 3, kGivResid = 4, kGivNonfinite = 5;

// instance of this workgroup
__device__ inline int bat_inst(const Bat& bt) { return bt.map[blockIdx.z / (gridDim.z / (unsigned)bt.count)]; }
__device__ inline bool bat_skip(const Bat& bt, int b) { return ((bt.mask >> b) & 1u) == 0u; }
__device__ inline double bat_s(const Bat& bt, int b, double v) { return bt.per ? bt.s[b] : v; }

// Allow a kernel the largest dynamic LDS of one workgroup (160 KiB); its launches then ask for
// what they need.  The attribute is set once per kernel (a set of the kernels already done,
// behind a mutex: launch sites run on several host threads), not on every launch.
inline void allow_max_lds(const void* kernel) {
  static std::mutex mu;
  static std::unordered_set<const void*> done;
  std::lock_guard<std::mutex> lock(mu);
  if (done.insert(kernel).second)
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// ---- phase-field kernels (kernels_phase.hip) ---------------------------------------
// X, Xn: nf planes (c, eta1..3, u1..ud); all plane strides are N.
// sig (may be null): in 3D, six planes of N doubles through which the first stage runs as two
// passes (the stress); null keeps the single-pass stencil
void launch_residual(const Consts& K, double dt, const double* X, const double* Xn, double* G4,
                     double* F, double* partial, hipStream_t s, const Bat& bt = Bat(),
                     double* sig = nullptr);
// B: 16 block planes; Bf (may be null): the same rounded to float
void launch_linearise(const Consts& K, const double* X, const double* Xn, double* B, float* Bf,
                      hipStream_t s, const Bat& bt = Bat());
// w = J v; v has element type Tv (double or float), w is double.  scr: in 3D, seven planes of
// N doubles that the two passes of the 3D product pass between them (unused in 2D)
template <typename Tv>
void launch_jv(const Consts& K, double dt, const double* B, const double* cn, const Tv* v, double* w,
               double* scr, hipStream_t s, const Bat& bt = Bat());
void launch_energy(const Consts& K, const double* X, double* partial, hipStream_t s, const Bat& bt = Bat());

// ---- Schwarz tile solve (kernels_ras.hip) -------------------------------------------
struct TileCfg {
  int tx, ty, tz;   // owned tile
  int ov;           // overlap delta
  int sweeps;       // symmetric GS sweeps
  double omega;     // over-relaxation factor of the sweeps (1: Gauss-Seidel)
  int with_u;       // 1: all fields (plain RAS); 0: (c, eta) block only
  const int* perm;  // device: nodes of the extended tile sorted by colour (ras_colour_order),
                    // followed by the inverse order (colour position of each node)
  int mode;         // 0 left-RAS, 1 classical AS, 2 right-RAS
  void* scratch;    // modes 1, 2: one extended solution per tile (Krylov type)
  void* pack;       // per tile and extended node, colour order: E^{-1}, E^{-1} v, Schur
                    // denominator of the node block (13 values, Krylov type; launch_ras_pack)
};
// R (double or float): element type of the blocks B, of r and z, and of the tile arithmetic
template <typename R>
void launch_ras(const Consts& K, const TileCfg& T, double dt, const R* B, const double* cn,
                const R* r, R* z, hipStream_t s, const Bat& bt = Bat());
size_t ras_lds_bytes(const Consts& K, const TileCfg& T, size_t real_bytes);
// once per time step, after the preconditioner blocks B: the node-block pieces of every
// extended tile into T.pack (ras_pack_values(K, T) elements of type R)
template <typename R>
void launch_ras_pack(const Consts& K, const TileCfg& T, double dt, const R* B, const double* cn, hipStream_t s,
                     const Bat& bt = Bat());
size_t ras_pack_values(const Consts& K, const TileCfg& T);
// workgroup size of the tile kernel for this tile shape and element size (0: shape not
// supported); *npt (may be null): nodes of the extended tile per thread
int ras_threads(const Consts& K, const TileCfg& T, size_t real_bytes, int* npt);
// nodes of one extended tile, and their colour-sorted order (host; the same for every tile)
int ras_ext_nodes(const Consts& K, const TileCfg& T);
void ras_colour_order(const Consts& K, const TileCfg& T, int* perm);

// ---- spectral displacement solve (kernels_fft.hip) -----------------------------------
struct FftPlan {
  int n[3];
  const double2* tw[3];  // twiddles exp(-2 pi i k / n), k <= n, one table per direction
  const double* sn[3];   // symbols S_m = sin(2 pi m / n) / h, m < n (exact 0 at m = 0, n/2)
};
// q_I = r_I + a D-hat_I zc (r may be null), solve K u = q by FFT, write u (d planes).
// T (double or float) is the element type of r, zc and u; the transforms run in double.
template <typename T>
void launch_spectral_solve(const Consts& K, const FftPlan& P, const T* r, double a,
                           const T* zc, double2* work0, double2* work1, T* u,
                           hipStream_t s, const Bat& bt = Bat());

// ---- vector kernels and reductions (kernels_blas.hip) --------------------------------
// V: nv vectors of length n stored ldv apart.  The basis element type T is double or float
// (instantiated for both); every sum is accumulated in double.
template <typename T>
void launch_multidot(long long n, int nv, const T* V, long long ldv, const double* w,
                     double* partial, hipStream_t s, const Bat& bt = Bat());
template <typename T, typename To>
void launch_lincomb(long long n, int nv, const T* V, long long ldv, const double* coef,
                    double beta, To* out, hipStream_t s, const Bat& bt = Bat());
// out = a x + b y (y unread when b == 0); instantiated for (d,d,d), (d,d,f), (f,f,f), (f,f,d)
template <typename Tx, typename Ty, typename To>
void launch_axpby(long long n, double a, const Tx* x, double b, const Ty* y, To* out, hipStream_t s,
                  const Bat& bt = Bat());
void launch_finalize(const double* partial, int nvals, double* out, hipStream_t s, double* out2 = nullptr,
                     const Bat& bt = Bat());
// v_{j+1} from device-resident Gram-Schmidt coefficients hc = [h_0..h_{nv-1}, <w,w>]
template <typename T>
void launch_update_dev(long long n, int nv, const T* V, long long ldv, const double* hc,
                       const double* w, T* out, hipStream_t s, const Bat& bt = Bat());
void launch_sum2(long long n, const double* x, const double* y, const double* yn, double* partial,
                 hipStream_t s, const Bat& bt = Bat());
// Xt = X + lam (S + shift e_c), shift = -(msums[0] + msums[1]) / N (device sums of launch_sum2,
// finalized); partial: count of nodes outside the log domain; pmax (may be null): per-block
// maxima of |S_f + shift_f| and |X_f| for every field f (2 nf values, for launch_finalize_max)
void launch_trial(const Consts& K, int nf, const double* X, const double* S, double lam,
                  const double* msums, double* Xt, double* partial, double* pmax, hipStream_t s,
                  const Bat& bt = Bat());
// second stage of per-block maxima of non-negative values (nvals <= 16)
void launch_finalize_max(const double* partial, int nvals, double* out, hipStream_t s, double* out2 = nullptr,
                         const Bat& bt = Bat());
void launch_dx2(long long n4, const double* X, const double* Xn, double* partial, hipStream_t s,
                const Bat& bt = Bat());
void launch_class_sums(const Consts& K, const double* u, double* partial, hipStream_t s, const Bat& bt = Bat());
void launch_class_shift(const Consts& K, double* u, const double* sums, hipStream_t s, const Bat& bt = Bat());

// ---- device-side GMRES cycle of a lockstep batch (kernels_blas.hip) -------------------
// giv: each instance's GivLayout(m) block.  launch_giv_init starts a cycle (bt.s: beta,
// bt.s2: tolerance, bt.s3: column limit); launch_arnoldi finalizes the multi-dot partials of
// Arnoldi step j into hcol (as launch_finalize), applies the Givens rotations and the end
// test, and writes (ended, |g_{j+1}|, columns, not finite) to host (pinned, hstride apart);
// launch_ysolve solves the cycle's triangular system; launch_lincomb_dev adds Z y to out.
void launch_giv_init(double* giv, int m, hipStream_t s, const Bat& bt);
void launch_arnoldi(const double* partial, int j, int m, double* hcol, double* giv, double* host, hipStream_t s,
                    const Bat& bt);
void launch_ysolve(double* giv, int m, hipStream_t s, const Bat& bt);
template <typename T, typename To>
void launch_lincomb_dev(long long n, int nv, const T* V, long long ldv, const double* giv, int m, To* out,
                        hipStream_t s, const Bat& bt);
template <typename T>
void launch_fill_zero(long long n, T* out, hipStream_t s, const Bat& bt = Bat());

}  // namespace pf
