// C ABI of the pfnks library (include/pfnks.h): problem set-up, the Newton-Krylov-Schwarz
// step of Section 4 of Huang & Yang, and the energy / mass queries.
//
// Host code drives the kernels on one HIP stream.  Scalars cross to the host once per GMRES
// iteration (the Hessenberg column), once per residual evaluation and once per reduction of
// the step close; all vectors stay in the caller's device workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pfnks.h"
#include "pf_internal.h"

using pf::Consts;

namespace {

thread_local std::string g_last_error;

int device_error(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return PFNKS_EDEVICE;
}

#define HIPCHK(call)                                       \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return device_error(e_, #call);  \
  } while (0)

// grid sides: even (the parity classes of the central difference), and products of the
// radices of the Fourier transforms (2, 3, 5, 7, 11, 13)
bool fft_side(int n) {
  if (n < 4 || (n & 1)) return false;
  for (int f = 2; f <= 13; ++f)
    while (n % f == 0) n /= f;
  return n == 1;
}

// preconditioners built on the Schwarz tile solve, and those that solve all fields there
bool uses_tiles(int pc) { return pc == PFNKS_PC_RAS || pc == PFNKS_PC_RAS_SPECTRAL || pc == PFNKS_PC_AS || pc == PFNKS_PC_RRAS; }
bool tiles_all_fields(int pc) { return pc == PFNKS_PC_RAS || pc == PFNKS_PC_AS || pc == PFNKS_PC_RRAS; }
bool sums_overlap(int pc) { return pc == PFNKS_PC_AS || pc == PFNKS_PC_RRAS; }

// ---------------------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------------------
struct Layout {
  size_t off[32];
  size_t total;
};

enum Buf {
  B_X, B_XN, B_XT, B_F, B_FT, B_S, B_B, B_BPC, B_G4, B_V, B_ZB, B_W, B_Z, B_TMP, B_TMPV, B_PART, B_RED,
  B_FFT0, B_FFT1, B_TW0, B_TW1, B_TW2, B_SN0, B_SN1, B_SN2, B_HDEV, B_PERM, B_ASX, B_PACK, B_GIV, B_COUNT
};

// bytes of one element of the Krylov basis, the preconditioner blocks and the tile solve
size_t krylov_bytes(int precision) { return precision == PFNKS_MIXED ? sizeof(float) : sizeof(double); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Krylov basis V, the preconditioned basis Z, the single vectors z and tmpv and the lagged
// preconditioner blocks Bpc are stored in the Krylov element type (float when mixed); the
// state, residuals, Newton update S, J v output w and the Jacobian blocks B are double.
Layout make_layout(int dim, long long N, int restart, const int* n, int precision, long long ext_nodes,
                   long long tiles_summed, long long tiles_packed) {
  const int nf = 4 + dim;
  const size_t kb = krylov_bytes(precision);
  const size_t vec = sizeof(double) * (size_t)nf * N;
  const size_t kvec = kb * (size_t)nf * N;
  size_t sz[B_COUNT];
  sz[B_X] = sz[B_XN] = sz[B_XT] = sz[B_F] = sz[B_FT] = sz[B_S] = vec;
  sz[B_B] = sizeof(double) * 16 * (size_t)N;
  sz[B_BPC] = kb * 16 * (size_t)N;
  sz[B_G4] = sizeof(double) * 4 * (size_t)N;
  sz[B_V] = kvec * (size_t)(restart + 1);
  sz[B_ZB] = kvec * (size_t)restart;
  sz[B_W] = sz[B_TMP] = vec;
  sz[B_Z] = kvec;
  sz[B_TMPV] = (precision == PFNKS_MIXED) ? kvec : 0;  // aliases tmp in FP64
  sz[B_PART] = sizeof(double) * (size_t)pf::kRedBlocks * pf::kMaxRed;
  sz[B_RED] = sizeof(double) * pf::kMaxRed;
  const size_t cplx = sizeof(double2) * (size_t)N * (dim == 3 ? 2 : 1);
  sz[B_FFT0] = sz[B_FFT1] = cplx;
  sz[B_TW0] = sizeof(double2) * (size_t)(n[0] + 1);
  sz[B_TW1] = sizeof(double2) * (size_t)(n[1] + 1);
  sz[B_TW2] = sizeof(double2) * (size_t)((dim == 3 ? n[2] : 2) + 1);
  sz[B_SN0] = sizeof(double) * (size_t)n[0];
  sz[B_SN1] = sizeof(double) * (size_t)n[1];
  sz[B_SN2] = sizeof(double) * (size_t)(dim == 3 ? n[2] : 2);
  sz[B_HDEV] = sizeof(double) * (size_t)(restart + 1) * (restart + 2);
  sz[B_PERM] = sizeof(int) * 2 * (size_t)ext_nodes;  // colour order of one extended tile, and its inverse
  // classical AS / right-RAS: every tile's extended solution (all fields), summed afterwards
  sz[B_ASX] = kb * (size_t)nf * (size_t)ext_nodes * (size_t)tiles_summed;
  // every tile's node-block pieces (13 per extended node), formed once per time step
  sz[B_PACK] = kb * 13 * (size_t)ext_nodes * (size_t)tiles_packed;
  // Hessenberg matrix, rotations and status of the device-side GMRES cycle (problem groups)
  sz[B_GIV] = sizeof(double) * (size_t)pf::giv_layout(restart).total;
  Layout L{};
  size_t o = 0;
  for (int b = 0; b < B_COUNT; ++b) {
    L.off[b] = o;
    o += align256(sz[b]);
  }
  L.total = o;
  return L;
}

// nodes of one extended Schwarz tile
long long ext_nodes(const pfnks_grid* g, const pfnks_solver* s) {
  long long e = 1;
  for (int k = 0; k < g->dim; ++k) e *= s->tile[k] + 2 * s->overlap;
  return e;
}

// tiles whose extended solutions need storing (classical AS / right-RAS), else 0
long long tiles_summed(const pfnks_grid* g, const pfnks_solver* s) {
  if (!sums_overlap(s->pc)) return 0;
  long long t = 1;
  for (int k = 0; k < g->dim; ++k) t *= g->n[k] / s->tile[k];
  return t;
}

// tiles of the Schwarz preconditioners (their node blocks are set up per time step), else 0
long long tiles_packed(const pfnks_grid* g, const pfnks_solver* s) {
  if (!uses_tiles(s->pc)) return 0;
  long long t = 1;
  for (int k = 0; k < g->dim; ++k) t *= g->n[k] / s->tile[k];
  return t;
}

int validate(const pfnks_grid* g, const pfnks_model* m, const pfnks_solver* s) {
  if (!g || !m || !s) return PFNKS_EINVAL;
  if (g->dim != 2 && g->dim != 3) return PFNKS_EINVAL;
  if (!(g->h > 0.0)) return PFNKS_EINVAL;
  for (int k = 0; k < g->dim; ++k) {
    if (!fft_side(g->n[k])) return PFNKS_EINVAL;
    const int t = s->tile[k];
    if (t <= 0 || g->n[k] % t != 0) return PFNKS_EINVAL;
    if (t + 2 * s->overlap > g->n[k]) return PFNKS_EINVAL;
  }
  if (g->dim == 2 && g->n[2] != 1) return PFNKS_EINVAL;
  if (s->overlap < 0 || s->overlap > 4) return PFNKS_EINVAL;
  if (s->gmres_restart < 1 || s->gmres_restart > 64) return PFNKS_EINVAL;
  if (s->sweeps < 1 || s->sweeps > 16) return PFNKS_EINVAL;
  if (s->newton_maxit < 1 || s->gmres_maxit < 1) return PFNKS_EINVAL;
  if (!(s->newton_stol >= 0.0)) return PFNKS_EINVAL;
  if (s->pc_refresh != 0 && s->pc_refresh != 1) return PFNKS_EINVAL;
  if (!(s->sor_omega > 0.0 && s->sor_omega < 2.0)) return PFNKS_EINVAL;
  if (s->pc < PFNKS_PC_RAS || s->pc > PFNKS_PC_RRAS) return PFNKS_EINVAL;
  if (sums_overlap(s->pc))
    for (int k = 0; k < g->dim; ++k)
      if (s->overlap > s->tile[k]) return PFNKS_EINVAL;  // at most three tiles per direction cover a node
  if (s->precision != PFNKS_FP64 && s->precision != PFNKS_MIXED) return PFNKS_EINVAL;
  if (m->S < 1 || m->S > pf::kMaxS) return PFNKS_EINVAL;
  if (!(m->kappa >= 0.0) || !(m->L_eta > 0.0) || m->Lscale < 0.0) return PFNKS_EINVAL;
  // extended tile must fit the kernel's registers (<= 3 nodes per thread of 512) and the
  // 160 KiB of LDS of one compute unit
  // (the iterate's LDS planes: all 4 + dim fields with a ring of two when the tiles solve the
  // displacement too, else the three eta fields with a ring of one)
  const bool all = tiles_all_fields(s->pc);
  long long ext = 1, zpad = 1, dpad = 1;
  for (int k = 0; k < g->dim; ++k) {
    ext *= s->tile[k] + 2 * s->overlap;
    zpad *= s->tile[k] + 2 * s->overlap + (all ? 4 : 2);
    dpad *= s->tile[k] + 2 * s->overlap + 2;
  }
  if (ext > 3 * 512) return PFNKS_EINVAL;
  const int nfz = all ? 4 + g->dim : 3;
  const long long kb = (long long)krylov_bytes(s->precision);
  if (uses_tiles(s->pc) && kb * (nfz * zpad + 2 * dpad + 4 * ext) > 160 * 1024) return PFNKS_EINVAL;
  return PFNKS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// problem
// ---------------------------------------------------------------------------------------
struct pfnks_problem {
  pfnks_grid grid;
  pfnks_model model;
  pfnks_solver solver;
  Consts K;
  pf::TileCfg T;
  pf::FftPlan plan;
  int nf;
  long long N, nvec;
  hipStream_t stream;
  char* ws;
  double *X, *Xn, *Xt, *F, *Ft, *S, *B, *G4, *w, *tmp, *part, *red;
  void *Bpc, *V, *Zb, *z, *tmpv;  // Krylov element type: double (PFNKS_FP64) or float (PFNKS_MIXED)
  size_t kb;                 // bytes of that element
  double2 *fft0, *fft1;
  double* hbuf;   // pinned host scalars (written directly by the finalize kernels)
  double* hdev;   // device Gram-Schmidt columns [h_0..h_j, <w,w>], one slot of m+2 per j
  double* hhost;  // pinned host mirror of hdev
  double* giv;    // device GMRES cycle state (GivLayout), used by problem groups
  std::vector<hipEvent_t> hev;  // one per Arnoldi column
  double t;
  long long launches, syncs;
  // live kernel timing (HIP events on the problem's stream), off unless enabled
  int prof;
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  long long kcount[PFNKS_KERNEL_KINDS];
  double kms[PFNKS_KERNEL_KINDS], kbytes[PFNKS_KERNEL_KINDS];
};

namespace {

Consts consts_of(const pfnks_grid& g, const pfnks_model& m) {
  Consts K;
  std::memset(&K, 0, sizeof(K));
  K.dim = g.dim;
  K.nx = g.n[0];
  K.ny = g.n[1];
  K.nz = (g.dim == 3) ? g.n[2] : 1;
  K.N = (long long)K.nx * K.ny * K.nz;
  K.h = g.h;
  K.ih = 1.0 / g.h;
  K.ih2 = 1.0 / (g.h * g.h);
  K.i2h = 0.5 / g.h;
  // p(c) = e0 c + c (1 - c) sum_k L_k (2c - 1)^k, expanded to monomials
  double poly[6] = {0, 0, 0, 0, 0, 0};
  double pw[6] = {1, 0, 0, 0, 0, 0};  // (2c - 1)^k
  for (int k = 0; k < 4; ++k) {
    // add L_k * (c - c^2) * pw
    for (int a = 0; a < 4; ++a) {
      poly[a + 1] += m.L[k] * pw[a];
      poly[a + 2] -= m.L[k] * pw[a];
    }
    double nxt[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 5; ++a) {
      nxt[a + 1] += 2.0 * pw[a];
      nxt[a] -= pw[a];
    }
    std::memcpy(pw, nxt, sizeof(pw));
  }
  poly[1] += m.e0;
  for (int a = 0; a < 6; ++a) K.pc[a] = poly[a];
  K.A2 = 4.0 * m.U1 + 12.0 * m.U4;
  K.A3 = -24.0 * m.U4;
  K.B3 = -48.0 * m.U4;
  K.theta = m.theta;
  K.w_c = m.w_c;
  K.gamma_c = m.gamma_c;
  K.gamma_eta = m.gamma_eta;
  K.kappa = m.kappa;
  K.L_eta = m.L_eta;
  K.eps0 = m.eps0;
  K.C11 = m.Lscale * m.C11;
  K.C12 = m.Lscale * m.C12;
  K.C44 = m.Lscale * m.C44;
  K.Ctr = K.C11 + (g.dim - 1) * K.C12;
  K.kel = 0.5 * g.dim * m.eps0 * m.eps0 * K.Ctr;
  K.elastic = (m.Lscale != 0.0) ? 1 : 0;
  K.S = m.S;
  for (int j = 1; j <= m.S - 1; ++j) {
    K.qs[j - 1] = 1.0 / (2.0 * j * (2.0 * j + 1.0));
    K.qd[j - 1] = 1.0 / (2.0 * (2.0 * j + 1.0));
  }
  return K;
}

void make_consts(pfnks_problem* p) { p->K = consts_of(p->grid, p->model); }

hipEvent_t prof_event(pfnks_problem* p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  // timing only: no system-scope fence (L2 write-back) when the event is recorded, so that
  // bracketing a kernel adds no cache flush between it and the next one
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// bracket the launches of one kernel kind with events (when profiling is on)
struct Prof {
  pfnks_problem* p;
  int kind;
  double bytes;
  hipEvent_t a;
  Prof(pfnks_problem* p_, int kind_, double bytes_) : p(p_), kind(kind_), bytes(bytes_), a(nullptr) {
    if (p->prof & (1 << kind)) {
      a = prof_event(p);
      if (a) (void)hipEventRecord(a, p->stream);
    }
  }
  ~Prof() {
    if (!a) return;
    hipEvent_t b = prof_event(p);
    if (!b) return;
    (void)hipEventRecord(b, p->stream);
    p->pending.push_back({kind, a, b, bytes});
  }
};

// turn finished event pairs into per-kind totals; pairs still in flight (recorded in stream
// order after the last completed work) stay pending
void prof_resolve(pfnks_problem* p) {
  size_t done = 0;
  for (; done < p->pending.size(); ++done) {
    auto& r = p->pending[done];
    if (hipEventQuery(r.b) != hipSuccess) break;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      p->kcount[r.kind] += 1;
      p->kms[r.kind] += ms;
      p->kbytes[r.kind] += r.bytes;
    }
    p->pool.push_back(r.a);
    p->pool.push_back(r.b);
  }
  p->pending.erase(p->pending.begin(), p->pending.begin() + done);
}

// slot of the two mass-projection sums in p->red, kept on the device for the line search's
// trials; every other reduction into p->red writes fewer values (at most 3 * 2^3 = 24)
constexpr int kRedMassSlot = pf::kMaxRed - 2;
// slots (device p->red and pinned host p->hbuf) of the update test's 2 nf per-field maxima
constexpr int kHostUpd = 8;

// finalize partial sums of nvals values and copy them to p->hbuf
int reduce_to_host(pfnks_problem* p, int nvals) {
  pf::launch_finalize(p->part, nvals, p->red, p->stream, p->hbuf);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(p->stream));
  p->launches += 1;
  p->syncs += 1;
  if (!p->pending.empty()) prof_resolve(p);
  return PFNKS_OK;
}

// kernels of one residual: two stencil passes, three in 3D with elasticity (the stress pass)
int residual_launches(const pfnks_problem* p) { return (p->K.dim == 3 && p->K.elastic) ? 3 : 2; }

// F = F(X; Xn, dt); returns ||F|| and the count of out-of-domain nodes
int residual(pfnks_problem* p, const double* X, double dt, double* F, double* nrm, double* bad) {
  {
    Prof pr(p, PFNKS_K_RESIDUAL, 8.0 * 3 * p->nvec);
    // 3D: the stress passes between the two stencil passes through w (free outside GMRES)
    pf::launch_residual(p->K, dt, X, p->Xn, p->G4, F, p->part, p->stream, pf::Bat(), p->w);
  }
  p->launches += residual_launches(p);
  int st = reduce_to_host(p, 2);
  if (st) return st;
  *nrm = std::sqrt(p->hbuf[0]);
  *bad = p->hbuf[1];
  return PFNKS_OK;
}

int dot_norm(pfnks_problem* p, const double* x, double* nrm) {
  pf::launch_multidot(p->nvec, 0, x, 0, x, p->part, p->stream);
  p->launches += 1;
  int st = reduce_to_host(p, 1);
  if (st) return st;
  *nrm = std::sqrt(p->hbuf[0]);
  return PFNKS_OK;
}

// bt with every instance's scalar set to 1 (a plain copy through axpby)
pf::Bat bat_ones(const pf::Bat& bt) {
  pf::Bat b = bt;
  for (int i = 0; i < pf::kMaxBatch; ++i) b.s[i] = 1.0;
  return b;
}

// algorithmic bytes of the per-step tile set-up: every extended tile node reads its chemical
// block (16) in the Krylov element type and c^n (double) and writes 13 node-block values
double pack_bytes(pfnks_problem* p) {
  if (!uses_tiles(p->solver.pc)) return 0.0;
  double rho = 1.0;
  for (int k = 0; k < p->K.dim; ++k) {
    const int t = p->solver.tile[k];
    rho *= (double)(t + 2 * p->solver.overlap) / t;
  }
  const double kb = (double)p->kb;
  return p->N * rho * (29.0 * kb + 8.0);
}

// algorithmic bytes of one Schwarz apply: every extended tile node reads r (nfz planes), its
// node-block pieces (13, formed once per step) and the c row of its chemical block (4), in
// the Krylov element type, and c^n (double); the owned nodes write z
double ras_bytes(pfnks_problem* p, int nfz) {
  double rho = 1.0;
  for (int k = 0; k < p->K.dim; ++k) {
    const int t = p->solver.tile[k];
    rho *= (double)(t + 2 * p->solver.overlap) / t;
  }
  const double kb = (double)p->kb;
  return p->N * (rho * ((nfz + 17) * kb + 8.0) + nfz * kb);
}

// once per time step, after the lagged preconditioner blocks Bpc: the tile solve's node blocks
void pc_setup(pfnks_problem* p, double dt, const pf::Bat& bt = pf::Bat()) {
  if (!uses_tiles(p->solver.pc)) return;
  if (p->solver.precision == PFNKS_MIXED)
    pf::launch_ras_pack<float>(p->K, p->T, dt, (const float*)p->Bpc, p->Xn, p->stream, bt);
  else
    pf::launch_ras_pack<double>(p->K, p->T, dt, (const double*)p->Bpc, p->Xn, p->stream, bt);
  p->launches += 1;
}

// z = M^{-1} r with the lagged preconditioner blocks Bpc; T is the Krylov element type
template <typename T>
void pc_apply(pfnks_problem* p, double dt, const T* r, T* z, const pf::Bat& bt = pf::Bat()) {
  const long long N = p->N;
  const int pc = p->solver.pc;
  const T* Bpc = static_cast<const T*>(p->Bpc);
  if (tiles_all_fields(pc)) {
    pf::TileCfg T_ = p->T;
    T_.with_u = 1;
    T_.mode = (pc == PFNKS_PC_AS) ? 1 : (pc == PFNKS_PC_RRAS) ? 2 : 0;
    Prof pr(p, PFNKS_K_RAS, ras_bytes(p, 4 + p->K.dim));
    pf::launch_ras<T>(p->K, T_, dt, Bpc, p->Xn, r, z, p->stream, bt);
    p->launches += sums_overlap(pc) ? 2 : 1;
    return;
  }
  if (pc == PFNKS_PC_RAS_SPECTRAL) {
    pf::TileCfg T_ = p->T;
    T_.with_u = 0;
    Prof pr(p, PFNKS_K_RAS, ras_bytes(p, 4));
    pf::launch_ras<T>(p->K, T_, dt, Bpc, p->Xn, r, z, p->stream, bt);
    p->launches += 1;
  } else {
    // PFNKS_PC_NONE and PFNKS_PC_SPECTRAL: z_w = r_w (a copy: every instance's scale is 1)
    pf::launch_axpby<T, T, T>(4 * N, 1.0, r, 0.0, nullptr, z, p->stream, bat_ones(bt));
    p->launches += 1;
  }
  if (pc == PFNKS_PC_NONE) {
    pf::launch_axpby<T, T, T>((long long)p->K.dim * N, 1.0, r + 4 * N, 0.0, nullptr, z + 4 * N, p->stream,
                              bat_ones(bt));
    p->launches += 1;
    return;
  }
  // displacement block: z_u = K^{-1} (r_u - J_uc z_c) = K^{-1} (r_u + eps0 Ctr Dhat z_c)
  Prof pr(p, PFNKS_K_SPECTRAL, (double)p->kb * (2 * p->K.dim + 1) * N);
  pf::launch_spectral_solve<T>(p->K, p->plan, r + 4 * N, p->K.eps0 * p->K.Ctr, z, p->fft0, p->fft1,
                               z + 4 * N, p->stream, bt);
  p->launches += 3 + 4 * p->K.dim * (p->K.dim == 3 ? 2 : 1);
}

// w = J v (v in element type Tv; arithmetic and w in double)
template <typename Tv>
void jv(pfnks_problem* p, double dt, const double* Bm, const Tv* v, double* w, const pf::Bat& bt = pf::Bat()) {
  Prof pr(p, PFNKS_K_JV, (double)p->nvec * (sizeof(Tv) + 8.0) + 136.0 * p->N);
  // 3D: two passes, dG and the stress through seven scratch planes (the trial residual Ft,
  // which holds nothing while a linear system is solved)
  pf::launch_jv<Tv>(p->K, dt, Bm, p->Xn, v, w, p->Ft, p->stream, bt);
  p->launches += (p->K.dim == 3) ? 2 : 1;
}

// Solve J S = -F: right-preconditioned restarted GMRES with classical Gram-Schmidt, in the
// flexible form: the preconditioned vectors z_j = M^{-1} v_j are kept (Z) and the correction
// is S += Z y, so J Z = V H holds up to the rounding of the stored v_{j+1} even when M^{-1}
// is applied in float (rounding makes it slightly nonlinear), and no preconditioner apply
// is needed at the end of a cycle.
// The Gram-Schmidt coefficients stay on the device (the update kernel reads them and forms
// h_{j+1,j} = sqrt(<w,w> - sum h_i^2)); the finalize kernel also writes them to pinned host
// memory.  The host enqueues Arnoldi step j+1 before it reads column j (Givens rotations,
// convergence test), so the device never waits for the host; at most one step per cycle is
// computed and discarded.  When <w,w> - sum h^2 has lost more than two digits, the cycle ends
// there and GMRES restarts from the true residual.
// T: element type of the basis, of z and of the preconditioner (float in mixed precision:
// every inner product, the Hessenberg matrix, S, F and the restart residual stay double).
template <typename T>
int gmres(pfnks_problem* p, double dt, const double* Bm, double fnorm, double tol, int* its,
          int* ok) {
  const long long n = p->nvec;
  const int m = p->solver.gmres_restart;
  const int maxit = p->solver.gmres_maxit;
  const int ld = m + 2;
  const double kb = (double)sizeof(T);
  T* V = static_cast<T*>(p->V);
  T* Z = static_cast<T*>(p->Zb);
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m);
  int total = 0;
  *ok = 0;
  *its = 0;
  HIPCHK(hipMemsetAsync(p->S, 0, sizeof(double) * n, p->stream));
  // r = -F
  pf::launch_axpby<double, double, double>(n, -1.0, p->F, 0.0, nullptr, p->tmp, p->stream);
  double beta = fnorm;
  p->launches += 1;
  auto launch_step = [&](int j) {
    pc_apply<T>(p, dt, V + j * n, Z + j * n);
    jv<T>(p, dt, Bm, Z + j * n, p->w);
    {
      Prof pr(p, PFNKS_K_MULTIDOT, (kb * (j + 1) + 8.0) * n);
      pf::launch_multidot<T>(n, j + 1, V, n, p->w, p->part, p->stream);
    }
    pf::launch_finalize(p->part, j + 2, p->hdev + j * ld, p->stream, p->hhost + j * ld);
    (void)hipEventRecord(p->hev[j], p->stream);
    {
      Prof pr(p, PFNKS_K_UPDATE, (kb * (j + 2) + 8.0) * n);
      pf::launch_update_dev<T>(n, j + 1, V, n, p->hdev + j * ld, p->w, V + (j + 1) * n, p->stream);
    }
    p->launches += 3;
  };
  while (true) {
    if (beta <= tol) {
      *ok = 1;
      break;
    }
    pf::launch_axpby<double, double, T>(n, 1.0 / beta, p->tmp, 0.0, nullptr, V, p->stream);
    p->launches += 1;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int launched = 1, k = 0;
    double resid = beta;
    launch_step(0);
    for (int j = 0;; ++j) {
      if (launched == j + 1 && j + 1 < m && total + launched < maxit) {
        launch_step(j + 1);
        ++launched;
      }
      HIPCHK(hipEventSynchronize(p->hev[j]));
      p->syncs += 1;
      if (!p->pending.empty()) prof_resolve(p);
      const double* hj = p->hhost + j * ld;
      double* h = &H[(size_t)j * (m + 1)];  // column j
      double hh = 0.0;
      for (int i = 0; i <= j; ++i) {
        h[i] = hj[i];
        hh += h[i] * h[i];
      }
      const double ww = hj[j + 1];
      const double nrm2 = ww - hh;
      const bool cancel = !(nrm2 > 1e-2 * ww);
      const double hnext = std::sqrt(std::fmax(nrm2, 0.0));
      h[j + 1] = hnext;
      for (int i = 0; i < j; ++i) {
        const double a = h[i], b = h[i + 1];
        h[i] = cs[i] * a + sn[i] * b;
        h[i + 1] = -sn[i] * a + cs[i] * b;
      }
      const double a = h[j], b = h[j + 1];
      const double r = std::hypot(a, b);
      cs[j] = (r == 0.0) ? 1.0 : a / r;
      sn[j] = (r == 0.0) ? 0.0 : b / r;
      h[j] = r;
      h[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      resid = std::fabs(g[j + 1]);
      ++total;
      k = j + 1;
      if (!std::isfinite(resid)) {
        (void)hipStreamSynchronize(p->stream);
        return PFNKS_ENOCONV;
      }
      if (resid <= tol) break;
      if (cancel || hnext == 0.0 || j + 1 == m || total >= maxit) break;
    }
    // y = H^{-1} g (upper triangular k x k)
    for (int i = k - 1; i >= 0; --i) {
      double s_ = g[i];
      for (int c = i + 1; c < k; ++c) s_ -= H[(size_t)c * (m + 1) + i] * y[c];
      y[i] = s_ / H[(size_t)i * (m + 1) + i];
    }
    // S += Z y
    pf::launch_lincomb<T, double>(n, k, Z, n, y.data(), 1.0, p->S, p->stream);
    p->launches += 1;
    // With a double basis the Hessenberg estimate |g_k| is the residual of the correction up
    // to rounding and decides convergence, as GMRES's recursive residual does.  A float basis
    // can make it optimistic by its rounding (2^-24), so there the true residual
    // r = -F - J S decides; a cycle that ends unconverged restarts from the true residual.
    if (sizeof(T) == sizeof(double) && resid <= tol) {
      *ok = 1;
      break;
    }
    jv<double>(p, dt, Bm, p->S, p->w);
    pf::launch_axpby<double, double, double>(n, -1.0, p->F, -1.0, p->w, p->tmp, p->stream);
    p->launches += 1;
    int st = dot_norm(p, p->tmp, &beta);
    if (st) return st;
    if (beta <= tol) {
      *ok = 1;
      break;
    }
    if (total >= maxit) break;
  }
  *its = total;
  return PFNKS_OK;
}

int step_close(pfnks_problem* p, pfnks_step_stats* st, const double* X, double dt_unused) {
  (void)dt_unused;
  // energy parts and mass at X
  pf::launch_energy(p->K, X, p->part, p->stream);
  p->launches += 1;
  int s = reduce_to_host(p, 4);
  if (s) return s;
  const double hd = std::pow(p->grid.h, p->grid.dim);
  if (st) {
    st->energy_parts[0] = p->hbuf[0] * hd;
    st->energy_parts[1] = p->hbuf[1] * hd;
    st->energy_parts[2] = p->hbuf[2] * hd;
    st->energy = st->energy_parts[0] + st->energy_parts[1] + st->energy_parts[2];
    st->mass = p->hbuf[3] * hd;
  }
  return PFNKS_OK;
}

int project_gauge(pfnks_problem* p, double* X) {
  pf::launch_class_sums(p->K, X + 4 * p->N, p->part, p->stream);
  const int ncls = 1 << p->grid.dim;
  pf::launch_finalize(p->part, p->grid.dim * ncls, p->red, p->stream);
  pf::launch_class_shift(p->K, X + 4 * p->N, p->red, p->stream);
  p->launches += 3;
  return PFNKS_OK;
}

int check_domain_host(const double* c, const double* eta, long long N) {
  for (long long i = 0; i < N; ++i) {
    const double cc = c[i];
    if (!(cc > 0.0 && cc < 1.0)) return PFNKS_EDOMAIN;
    double es = 0.0;
    for (int q = 0; q < 3; ++q) {
      const double y = cc * eta[q * N + i];
      es += eta[q * N + i];
      if (!(y > 0.0 && y < 1.0)) return PFNKS_EDOMAIN;
    }
    const double y4 = cc * (4.0 - es);
    if (!(y4 > 0.0 && y4 < 1.0)) return PFNKS_EDOMAIN;
  }
  return PFNKS_OK;
}

// ---------------------------------------------------------------------------------------
// allocation-free residual: file-scope device scratch
// ---------------------------------------------------------------------------------------
// Largest grid of pfnks_residual_static, and its scratch: the four G planes of the residual's
// first pass, then the reductions' per-block partial sums (two values) and their two sums.
constexpr long long kStaticMaxNodes = 1LL << 21;
constexpr size_t kStaticG = 4 * (size_t)kStaticMaxNodes;
constexpr size_t kStaticDoubles = kStaticG + 2 * (size_t)pf::kRedBlocks + 64;
static __device__ __align__(256) double scratch[kStaticDoubles];

// Device address of `scratch` on each GPU (each holds its own copy), taken once per device
// with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return PFNKS_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return PFNKS_OK;
}

int validate_grid_model(const pfnks_grid* g, const pfnks_model* m) {
  if (!g || !m) return PFNKS_EINVAL;
  if (g->dim != 2 && g->dim != 3) return PFNKS_EINVAL;
  if (!(g->h > 0.0)) return PFNKS_EINVAL;
  for (int k = 0; k < g->dim; ++k)
    if (!fft_side(g->n[k])) return PFNKS_EINVAL;
  if (g->dim == 2 && g->n[2] != 1) return PFNKS_EINVAL;
  if (m->S < 1 || m->S > pf::kMaxS) return PFNKS_EINVAL;
  if (!(m->kappa >= 0.0) || !(m->L_eta > 0.0) || m->Lscale < 0.0) return PFNKS_EINVAL;
  return PFNKS_OK;
}

}  // namespace

extern "C" {

int pfnks_residual_static(const pfnks_grid* grid, const pfnks_model* model, double cbar0, double dt,
                          const double* d_X, const double* d_Xn, double* d_F, double* norm, double* bad,
                          void* hip_stream) {
  int st = validate_grid_model(grid, model);
  if (st) return st;
  if (!d_X || !d_Xn || !d_F || !(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(cbar0)) return PFNKS_EINVAL;
  const long long N = (long long)grid->n[0] * grid->n[1] * (grid->dim == 3 ? grid->n[2] : 1);
  if (N > kStaticMaxNodes) return PFNKS_ENOSPACE;
  double* scr = nullptr;
  st = static_scratch(&scr);
  if (st) return st;
  pfnks_grid g = *grid;
  if (g.dim == 2) g.n[2] = 1;
  Consts K = consts_of(g, *model);
  K.cbar0 = cbar0;
  hipStream_t s = (hipStream_t)hip_stream;
  double* G4 = scr;
  double* part = scr + kStaticG;
  double* red = part + 2 * pf::kRedBlocks;
  pf::launch_residual(K, dt, d_X, d_Xn, G4, d_F, part, s);
  HIPCHK(hipGetLastError());
  if (norm || bad) {
    pf::launch_finalize(part, 2, red, s);
    HIPCHK(hipGetLastError());
    double h[2];
    HIPCHK(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (norm) *norm = std::sqrt(h[0]);
    if (bad) *bad = h[1];
  }
  return PFNKS_OK;
}

}  // extern "C"

namespace {

// the problem object over a workspace laid out by L: device pointers, pinned host scalars,
// events, twiddle and symbol tables and the tile colour order (no state yet)
int setup_problem(const pfnks_grid* grid, const pfnks_model* model, const pfnks_solver* solver, const Layout& L,
                  long long N, char* ws, hipStream_t stream, pfnks_problem** out) {
  pfnks_problem* p = new pfnks_problem();
  p->prof = 0;
  p->hbuf = nullptr;
  p->hhost = nullptr;
  for (int k = 0; k < PFNKS_KERNEL_KINDS; ++k) {
    p->kcount[k] = 0;
    p->kms[k] = 0.0;
    p->kbytes[k] = 0.0;
  }
  p->grid = *grid;
  if (grid->dim == 2) p->grid.n[2] = 1;
  p->model = *model;
  p->solver = *solver;
  p->nf = 4 + grid->dim;
  p->N = N;
  p->nvec = (long long)p->nf * N;
  p->stream = stream;
  p->ws = ws;
  make_consts(p);
  p->T.tx = solver->tile[0];
  p->T.ty = solver->tile[1];
  p->T.tz = (grid->dim == 3) ? solver->tile[2] : 1;
  p->T.ov = solver->overlap;
  p->T.sweeps = solver->sweeps;
  p->T.omega = solver->sor_omega;
  p->T.with_u = 0;
  p->T.perm = (const int*)(p->ws + L.off[B_PERM]);
  p->T.mode = 0;
  p->T.scratch = p->ws + L.off[B_ASX];
  p->T.pack = p->ws + L.off[B_PACK];
  pf::TileCfg tcheck = p->T;
  tcheck.with_u = tiles_all_fields(solver->pc) ? 1 : 0;
  if (uses_tiles(solver->pc) && (pf::ras_threads(p->K, tcheck, krylov_bytes(solver->precision), nullptr) == 0 ||
                                 pf::ras_lds_bytes(p->K, tcheck, krylov_bytes(solver->precision)) > 160 * 1024)) {
    delete p;
    return PFNKS_EINVAL;  // tile shape beyond what the tile kernel holds per thread or in LDS
  }
  auto ptr = [&](int b) { return (double*)(p->ws + L.off[b]); };
  p->kb = krylov_bytes(solver->precision);
  p->X = ptr(B_X);
  p->Xn = ptr(B_XN);
  p->Xt = ptr(B_XT);
  p->F = ptr(B_F);
  p->Ft = ptr(B_FT);
  p->S = ptr(B_S);
  p->B = ptr(B_B);
  p->Bpc = ptr(B_BPC);
  p->G4 = ptr(B_G4);
  p->V = ptr(B_V);
  p->Zb = ptr(B_ZB);
  p->w = ptr(B_W);
  p->z = ptr(B_Z);
  p->tmp = ptr(B_TMP);
  p->tmpv = (solver->precision == PFNKS_MIXED) ? (void*)ptr(B_TMPV) : (void*)p->tmp;
  p->part = ptr(B_PART);
  p->red = ptr(B_RED);
  p->fft0 = (double2*)(p->ws + L.off[B_FFT0]);
  p->fft1 = (double2*)(p->ws + L.off[B_FFT1]);
  p->giv = ptr(B_GIV);
  p->t = 0.0;

  auto fail = [&](int code) {
    if (p->hbuf) (void)hipHostFree(p->hbuf);
    if (p->hhost) (void)hipHostFree(p->hhost);
    for (auto ev : p->hev)
      if (ev) (void)hipEventDestroy(ev);
    delete p;
    return code;
  };
  hipError_t e = hipHostMalloc((void**)&p->hbuf, sizeof(double) * pf::kMaxRed, hipHostMallocDefault);
  if (e != hipSuccess) return fail(device_error(e, "hipHostMalloc"));
  const int mres = solver->gmres_restart;
  e = hipHostMalloc((void**)&p->hhost, sizeof(double) * (mres + 1) * (mres + 2), hipHostMallocDefault);
  if (e != hipSuccess) return fail(device_error(e, "hipHostMalloc"));
  p->hdev = (double*)(p->ws + L.off[B_HDEV]);
  p->hev.resize(mres + 1, nullptr);
  for (auto& ev : p->hev) {
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return fail(device_error(e, "hipEventCreate"));
  }

  // twiddle tables exp(-2 pi i k / n), k <= n (the power-of-two transforms read k < n/2, the
  // mixed-radix ones every k < n)
  for (int d = 0; d < 3; ++d) {
    const int nd = (d < grid->dim) ? grid->n[d] : 2;
    std::vector<double2> tw(nd + 1);
    for (int k = 0; k <= nd; ++k) {
      const double ang = -2.0 * M_PI * (double)k / (double)nd;
      tw[k] = make_double2(std::cos(ang), std::sin(ang));
    }
    double2* dst = (double2*)(p->ws + L.off[B_TW0 + d]);
    e = hipMemcpy(dst, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(device_error(e, "hipMemcpy twiddles"));
    p->plan.tw[d] = dst;
    p->plan.n[d] = nd;
    // Fourier symbol of the central difference: i sin(2 pi m / n) / h
    std::vector<double> sn(nd);
    for (int m = 0; m < nd; ++m)
      sn[m] = (m == 0 || 2 * m == nd) ? 0.0 : std::sin(2.0 * M_PI * (double)m / (double)nd) / grid->h;
    double* sdst = (double*)(p->ws + L.off[B_SN0 + d]);
    e = hipMemcpy(sdst, sn.data(), sizeof(double) * nd, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(device_error(e, "hipMemcpy symbols"));
    p->plan.sn[d] = sdst;
  }
  // colour order of the extended tile (the same for every tile) and its inverse (the colour
  // position of each node), for the Schwarz kernels
  {
    const size_t ne = (size_t)pf::ras_ext_nodes(p->K, p->T);
    std::vector<int> order(2 * ne);
    pf::ras_colour_order(p->K, p->T, order.data());
    for (size_t pos = 0; pos < ne; ++pos) order[ne + (size_t)order[pos]] = (int)pos;
    e = hipMemcpy((void*)p->T.perm, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(device_error(e, "hipMemcpy colour order"));
  }
  *out = p;
  return PFNKS_OK;
}

void destroy_problem(pfnks_problem* p) {
  if (!p) return;
  for (auto& r : p->pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto ev : p->pool) (void)hipEventDestroy(ev);
  for (auto ev : p->hev)
    if (ev) (void)hipEventDestroy(ev);
  if (p->hbuf) (void)hipHostFree(p->hbuf);
  if (p->hhost) (void)hipHostFree(p->hhost);
  delete p;
}

}  // namespace

extern "C" {

int pfnks_workspace_bytes(const pfnks_grid* grid, const pfnks_model* model, const pfnks_solver* solver,
                          size_t* bytes) {
  if (!bytes) return PFNKS_EINVAL;
  int st = validate(grid, model, solver);
  if (st) return st;
  const long long N = (long long)grid->n[0] * grid->n[1] * (grid->dim == 3 ? grid->n[2] : 1);
  *bytes = make_layout(grid->dim, N, solver->gmres_restart, grid->n, solver->precision, ext_nodes(grid, solver),
                       tiles_summed(grid, solver), tiles_packed(grid, solver)).total;
  return PFNKS_OK;
}

int pfnks_create_problem(const pfnks_grid* grid, const pfnks_model* model, const pfnks_solver* solver,
                         const double* c0, const double* eta0, void* d_workspace, size_t ws_bytes,
                         void* hip_stream, pfnks_problem** out) {
  if (!out || !c0 || !eta0 || !d_workspace) return PFNKS_EINVAL;
  *out = nullptr;
  int st = validate(grid, model, solver);
  if (st) return st;
  if (((uintptr_t)d_workspace & 255) != 0) return PFNKS_EINVAL;
  const long long N = (long long)grid->n[0] * grid->n[1] * (grid->dim == 3 ? grid->n[2] : 1);
  const Layout L = make_layout(grid->dim, N, solver->gmres_restart, grid->n, solver->precision, ext_nodes(grid, solver),
                               tiles_summed(grid, solver), tiles_packed(grid, solver));
  if (ws_bytes < L.total) return PFNKS_ENOSPACE;
  st = check_domain_host(c0, eta0, N);
  if (st) return st;

  pfnks_problem* p = nullptr;
  st = setup_problem(grid, model, solver, L, N, (char*)d_workspace, (hipStream_t)hip_stream, &p);
  if (st) return st;
  auto fail = [&](int code) {
    destroy_problem(p);
    return code;
  };
  hipError_t e = hipSuccess;
  // state: c, eta, u = 0
  e = hipMemcpy(p->Xn, c0, sizeof(double) * N, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->Xn + N, eta0, sizeof(double) * 3 * N, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p->Xn + 4 * N, 0, sizeof(double) * grid->dim * N);
  if (e != hipSuccess) return fail(device_error(e, "state upload"));
  // cbar0 = mean(c0) by a grid reduction
  pf::launch_sum2(N, p->Xn, p->Xn, p->Xn, p->part, p->stream);
  st = reduce_to_host(p, 1);
  if (st) return fail(st);
  p->K.cbar0 = p->hbuf[0] / (double)N;
  // u0 from the discrete equilibrium at c0: K u = eps0 Ctr Dhat c0 (the cbar0 shift drops out)
  pf::launch_spectral_solve<double>(p->K, p->plan, nullptr, p->K.eps0 * p->K.Ctr, p->Xn, p->fft0, p->fft1,
                            p->Xn + 4 * N, p->stream);
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return fail(device_error(e, "elastic init"));
  *out = p;
  return PFNKS_OK;
}

int pfnks_step(pfnks_problem* p, double dt, pfnks_step_stats* stats) {
  if (!p || !(dt > 0.0) || !std::isfinite(dt)) return PFNKS_EINVAL;
  pfnks_step_stats st{};
  p->launches = 0;
  p->syncs = 0;
  const long long n = p->nvec, N = p->N;
  const pfnks_solver& sv = p->solver;
  const double sq = std::sqrt((double)n);
  const double eps_a = sv.newton_atol_rms * sq, xi_a = sv.gmres_atol_rms * sq;
  // X_0 = X^n
  HIPCHK(hipMemcpyAsync(p->X, p->Xn, sizeof(double) * n, hipMemcpyDeviceToDevice, p->stream));
  double fn, bad;
  int s = residual(p, p->X, dt, p->F, &fn, &bad);
  if (s) return s;
  st.res0 = fn;
  const double r0 = fn;
  int converged = (fn <= eps_a) || fn == 0.0;
  int newton = 0, gm_total = 0, backtracks = 0;
  double upd_rel = 0.0;
  double ds_prev[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // per-field max|lambda S_f| of the last correction
  for (; !converged && newton < sv.newton_maxit; ++newton) {
    // linearise at X; the preconditioner blocks are set up once per step (lagged over the
    // Newton iterations, the paper's factorisation reuse) or, with pc_refresh, at every
    // Newton iteration
    double* Bm = p->B;
    {
      const bool mixed = sv.precision == PFNKS_MIXED;
      const bool build_pc = (newton == 0) || sv.pc_refresh;
      Prof pr(p, PFNKS_K_LINEARISE,
              8.0 * 24 * N + ((build_pc && mixed) ? 64.0 * N : 0.0) + (build_pc ? pack_bytes(p) : 0.0));
      if (build_pc && !mixed) {
        pf::launch_linearise(p->K, p->X, p->Xn, (double*)p->Bpc, nullptr, p->stream);
        Bm = (double*)p->Bpc;
      } else {
        pf::launch_linearise(p->K, p->X, p->Xn, p->B, build_pc ? (float*)p->Bpc : nullptr, p->stream);
      }
      if (build_pc) pc_setup(p, dt);
    }
    p->launches += 1;
    const double tol = std::fmax(sv.gmres_rtol * fn, xi_a);
    int its = 0, ok = 0;
    s = (sv.precision == PFNKS_MIXED) ? gmres<float>(p, dt, Bm, fn, tol, &its, &ok)
                                      : gmres<double>(p, dt, Bm, fn, tol, &its, &ok);
    gm_total += its;
    if (s == PFNKS_ENOCONV) break;
    if (s) return s;
    // mass projection of the update: sum S_c = -sum (c - c^n); the two sums stay on the
    // device (a slot of red no other reduction writes) and the trial kernel forms the shift
    double* msums = p->red + kRedMassSlot;
    pf::launch_sum2(N, p->S, p->X, p->Xn, p->part, p->stream);
    pf::launch_finalize(p->part, 2, msums, p->stream);
    p->launches += 2;
    // backtracking line search (Armijo).  One host synchronisation per trial: the trial's
    // count of nodes outside the log domain goes to host memory without one, and the residual
    // is evaluated at the trial point whatever it is (outside the domain it is not finite and
    // counts the same nodes, and the point is rejected either way).
    // The first trial also takes the per-field maxima |S_f| and |X_f| of the update test
    // (host slots kHostUpd.., read after that trial's residual synchronisation).
    double lam = 1.0, ft = 0.0;
    bool accepted = false;
    for (int hv = 0; hv <= sv.ls_max_halvings; ++hv) {
      pf::launch_trial(p->K, p->nf, p->X, p->S, lam, msums, p->Xt, p->part,
                       hv == 0 ? p->part + pf::kRedBlocks : nullptr, p->stream);
      pf::launch_finalize(p->part, 1, p->red, p->stream, p->hbuf + 2);
      p->launches += 2;
      if (hv == 0) {
        pf::launch_finalize_max(p->part + pf::kRedBlocks, 2 * p->nf, p->red + kHostUpd, p->stream,
                                p->hbuf + kHostUpd);
        p->launches += 1;
      }
      s = residual(p, p->Xt, dt, p->Ft, &ft, &bad);
      if (s) return s;
      const double trial_bad = p->hbuf[2];
      if (trial_bad == 0.0 && bad == 0.0 && std::isfinite(ft) &&
          ft * ft <= (1.0 - 2.0 * sv.ls_alpha * lam) * fn * fn) {
        accepted = true;
        break;
      }
      lam *= 0.5;
      ++backtracks;
    }
    if (!accepted) break;
    std::swap(p->X, p->Xt);
    std::swap(p->F, p->Ft);
    fn = ft;
    // update test: the error left after this correction, estimated from the contraction of
    // consecutive corrections theta = max_f |dS_f|_k / |dS_f|_{k-1} as theta / (1 - theta)
    // |dS_f|_k, must be <= stol max|X_f| in every field.  The first correction has no
    // estimate (one more iteration is needed); a field whose correction is exactly zero
    // passes (e.g. the displacement without elasticity).
    double ds[8], xs[8], theta = 0.0;
    for (int f = 0; f < p->nf; ++f) {
      ds[f] = lam * p->hbuf[kHostUpd + 2 * f];
      xs[f] = p->hbuf[kHostUpd + 2 * f + 1];
      if (ds[f] > 0.0) theta = std::fmax(theta, ds_prev[f] > 0.0 ? ds[f] / ds_prev[f] : HUGE_VAL);
    }
    const double amp = (theta < 1.0) ? theta / (1.0 - theta) : HUGE_VAL;
    bool small_update = true;
    upd_rel = 0.0;
    for (int f = 0; f < p->nf; ++f) {
      if (ds[f] == 0.0) continue;
      const double est = ds[f] * amp;
      upd_rel = std::fmax(upd_rel, xs[f] > 0.0 ? est / xs[f] : HUGE_VAL);
      if (!(est <= sv.newton_stol * xs[f])) small_update = false;
    }
    for (int f = 0; f < p->nf; ++f) ds_prev[f] = ds[f];
    if (sv.newton_stol <= 0.0) small_update = true;
    if (fn <= eps_a || (fn <= sv.newton_rtol * r0 && small_update)) {
      converged = 1;
      ++newton;
      break;
    }
  }
  st.newton_its = newton;
  st.gmres_its = gm_total;
  st.ls_backtracks = backtracks;
  st.res_final = fn;
  st.update_rel = upd_rel;
  if (!converged) {
    st.status = PFNKS_ENOCONV;
    if (stats) *stats = st;
    HIPCHK(hipStreamSynchronize(p->stream));
    return PFNKS_ENOCONV;
  }
  // zero mean of u on every parity class (the gauge Dhat leaves free): the Fourier block
  // already returns updates without those modes, but only up to the rounding of the Krylov
  // element type, and the other preconditioners do not remove them at all
  project_gauge(p, p->X);
  // step close: ||X - X^n|| over c and eta (to host memory, read after the energy's
  // synchronisation), energy, mass
  pf::launch_dx2(4 * N, p->X, p->Xn, p->part, p->stream);
  pf::launch_finalize(p->part, 1, p->red, p->stream, p->hbuf + 4);
  p->launches += 2;
  s = step_close(p, &st, p->X, dt);
  if (s) return s;
  st.dx_rms = std::sqrt(p->hbuf[4] / (4.0 * N));
  std::swap(p->X, p->Xn);
  p->t += dt;
  st.status = PFNKS_OK;
  if (stats) *stats = st;
  return PFNKS_OK;
}

int pfnks_batch_step(pfnks_problem* const* problems, int k, const double* dts, int threads,
                     pfnks_step_stats* stats, int* status) {
  if (!problems || !dts || k < 0 || threads < 0) return PFNKS_EINVAL;
  for (int i = 0; i < k; ++i) {
    if (!problems[i]) return PFNKS_EINVAL;
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i]) return PFNKS_EINVAL;
  }
  std::vector<int> st(k, PFNKS_OK);
  // the worker's text of a PFNKS_EDEVICE (g_last_error is per thread), handed to the caller
  std::vector<std::string> err(k);
  std::atomic<int> next{0};
  auto work = [&]() {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= k) break;
      st[i] = pfnks_step(problems[i], dts[i], stats ? &stats[i] : nullptr);
      if (st[i] == PFNKS_EDEVICE) err[i] = g_last_error;
    }
  };
  const int nth = std::min(k, threads > 0 ? threads : 16);
  if (nth <= 1) {
    work();
  } else {
    std::vector<std::thread> pool;
    pool.reserve(nth);
    for (int t = 0; t < nth; ++t) pool.emplace_back(work);
    for (auto& t : pool) t.join();
  }
  int first = PFNKS_OK;
  for (int i = 0; i < k; ++i) {
    if (status) status[i] = st[i];
    if (first == PFNKS_OK && st[i] != PFNKS_OK) {
      first = st[i];
      if (st[i] == PFNKS_EDEVICE) g_last_error = "problem " + std::to_string(i) + ": " + err[i];
    }
  }
  return first;
}

// ---------------------------------------------------------------------------------------
// lockstep problem groups
// ---------------------------------------------------------------------------------------
// A group is `count` problems of one grid, model and solver in one workspace: instance i's
// workspace is instance 0's layout, i * stride bytes further on.  Every kernel launch covers
// all instances still working in that phase (pf::Bat), so a Newton iteration costs one
// launch per kernel kind however many instances there are, and the host synchronises once
// per Arnoldi step, residual evaluation and cycle end for all of them together.  The
// Hessenberg columns, Givens rotations and the cycle's triangular solve run on the device
// (launch_arnoldi, launch_ysolve), so the host reads only each instance's status.
}  // extern "C"

namespace {

// pinned host slots of one instance: the single problem's reduction slots, then the GMRES
// cycle status (ended, |g_{j+1}|, columns, not finite)
constexpr int kHostGiv = pf::kMaxRed;
constexpr int kHostSlot = pf::kMaxRed + 8;

unsigned all_mask(int count) { return count >= 32 ? 0xffffffffu : ((1u << count) - 1u); }

}  // namespace

struct pfnks_group {
  pfnks_problem* p;  // instance 0: grid, model, solver, kernel constants, pointers into its workspace
  int count;
  long long stride;  // bytes between the instances' workspaces
  double* hs;        // pinned host slots, kHostSlot per instance
  std::vector<double> cbar0, t, dt;
  long long launches, syncs;
};

namespace {

// launch descriptor over the instances in mask (only those are launched: the grid's z parts
// map to them in order); the per-instance scalar is the time step
pf::Bat gbat(const pfnks_group* G, unsigned mask) {
  pf::Bat b;
  b.stride = G->stride;
  b.hstride = (long long)sizeof(double) * kHostSlot;
  b.per = 1;
  b.mask = mask;
  b.count = 0;
  for (int i = 0; i < G->count; ++i)
    if ((mask >> i) & 1u) b.map[b.count++] = (unsigned char)i;
  if (b.count == 0) b.count = 1;  // an empty launch: its one part has a clear mask bit and returns
  for (int i = 0; i < G->count; ++i) {
    b.s[i] = G->dt[i];
    b.cb[i] = G->cbar0[i];
  }
  return b;
}

// the same with every instance's scalar v (the coefficient of axpby)
pf::Bat gbat_s(const pfnks_group* G, unsigned mask, double v) {
  pf::Bat b = gbat(G, mask);
  for (int i = 0; i < G->count; ++i) b.s[i] = v;
  return b;
}

inline bool has(unsigned mask, int i) { return (mask >> i) & 1u; }
inline double* gslot(pfnks_group* G, int i) { return G->hs + (size_t)i * kHostSlot; }

int gsync(pfnks_group* G) {
  HIPCHK(hipStreamSynchronize(G->p->stream));
  G->syncs += 1;
  return PFNKS_OK;
}

void gcopy(pfnks_group* G, unsigned mask, const double* src, double* dst) {
  pf::launch_axpby<double, double, double>(G->p->nvec, 1.0, src, 0.0, nullptr, dst, G->p->stream,
                                           gbat_s(G, mask, 1.0));
  G->launches += 1;
}

// F = F(X) for the instances in mask; their ||F|| and counts of nodes outside the log domain
int gresidual(pfnks_group* G, unsigned mask, const double* X, double* F, double* nrm, double* bad) {
  pfnks_problem* p = G->p;
  const pf::Bat bt = gbat(G, mask);
  pf::launch_residual(p->K, 0.0, X, p->Xn, p->G4, F, p->part, p->stream, bt, p->w);
  pf::launch_finalize(p->part, 2, p->red, p->stream, G->hs, bt);
  G->launches += residual_launches(p) + 1;
  int st = gsync(G);
  if (st) return st;
  for (int i = 0; i < G->count; ++i)
    if (has(mask, i)) {
      nrm[i] = std::sqrt(gslot(G, i)[0]);
      bad[i] = gslot(G, i)[1];
    }
  return PFNKS_OK;
}

// GMRES of gmres() for the instances in act, in lockstep: every Arnoldi step is launched for
// the instances whose cycle is still running (as far as the host knows: one step is launched
// ahead, and the device leaves an instance whose cycle has ended untouched).  its: total
// iterations; *bad: instances whose residual estimate became non-finite.
template <typename T>
int gmres_group(pfnks_group* G, unsigned act, const double* Bm, const double* fnorm, const double* tol, int* its,
                unsigned* bad) {
  pfnks_problem* p = G->p;
  const long long n = p->nvec;
  const int m = p->solver.gmres_restart, maxit = p->solver.gmres_maxit, ld = m + 2;
  T* V = static_cast<T*>(p->V);
  T* Z = static_cast<T*>(p->Zb);
  const int B = G->count;
  std::vector<double> beta(B, 0.0);
  std::vector<int> total(B, 0), cols(B, 0);
  *bad = 0;
  pf::launch_fill_zero<double>(n, p->S, p->stream, gbat(G, act));
  pf::launch_axpby<double, double, double>(n, -1.0, p->F, 0.0, nullptr, p->tmp, p->stream, gbat_s(G, act, -1.0));
  G->launches += 2;
  for (int i = 0; i < B; ++i)
    if (has(act, i)) {
      beta[i] = fnorm[i];
      its[i] = 0;
    }
  auto launch_step = [&](int j, unsigned mask) {
    const pf::Bat bt = gbat(G, mask);  // per-instance time step of the tile solve and J v
    pc_apply<T>(p, 0.0, V + j * n, Z + j * n, bt);
    jv<T>(p, 0.0, Bm, Z + j * n, p->w, bt);
    pf::launch_multidot<T>(n, j + 1, V, n, p->w, p->part, p->stream, bt);
    pf::launch_arnoldi(p->part, j, m, p->hdev + j * ld, p->giv, G->hs + kHostGiv, p->stream, bt);
    (void)hipEventRecord(p->hev[j], p->stream);
    pf::launch_update_dev<T>(n, j + 1, V, n, p->hdev + j * ld, p->w, V + (j + 1) * n, p->stream, bt);
    G->launches += 3;
  };
  unsigned live = act;
  while (true) {
    for (int i = 0; i < B; ++i)
      if (has(live, i) && beta[i] <= tol[i]) live &= ~(1u << i);
    if (!live) break;
    // v_0 = r / beta and the start of the cycle on the device: g = beta e_1, its tolerance
    // and column limit
    int lim_max = 0;
    {
      pf::Bat bv = gbat(G, live), bg = gbat(G, live);
      for (int i = 0; i < B; ++i)
        if (has(live, i)) {
          const int lim = std::min(m, maxit - total[i]);
          bv.s[i] = 1.0 / beta[i];
          bg.s[i] = beta[i];
          bg.s2[i] = tol[i];
          bg.s3[i] = (double)lim;
          lim_max = std::max(lim_max, lim);
        }
      pf::launch_axpby<double, double, T>(n, 0.0, p->tmp, 0.0, nullptr, V, p->stream, bv);
      pf::launch_giv_init(p->giv, m, p->stream, bg);
      G->launches += 2;
    }
    unsigned run = live;
    launch_step(0, run);
    int launched = 1;
    for (int j = 0;; ++j) {
      if (launched == j + 1 && j + 1 < lim_max) {
        launch_step(j + 1, run);
        ++launched;
      }
      HIPCHK(hipEventSynchronize(p->hev[j]));
      G->syncs += 1;
      for (int i = 0; i < B; ++i) {
        if (!has(run, i)) continue;
        const double* h = gslot(G, i) + kHostGiv;
        if (h[0] != 0.0) {
          run &= ~(1u << i);
          cols[i] = (int)h[2];
          if (h[3] != 0.0) *bad |= 1u << i;
        }
      }
      if (!run) break;
      if (j + 1 >= launched) {
        // every cycle ends by its column limit, which no launched step exceeds
        g_last_error = "GMRES cycle of a problem group did not end at its column limit";
        return PFNKS_EDEVICE;
      }
    }
    // S += Z y per instance; then the true residual r = -F - J S decides and restarts for the
    // instances whose estimate does not settle it
    const unsigned fin = live & ~*bad;
    if (fin) {
      int kmax = 1;
      for (int i = 0; i < B; ++i)
        if (has(fin, i)) kmax = std::max(kmax, cols[i]);
      const pf::Bat bf = gbat(G, fin);
      pf::launch_ysolve(p->giv, m, p->stream, bf);
      pf::launch_lincomb_dev<T, double>(n, kmax, Z, n, p->giv, m, p->S, p->stream, bf);
      G->launches += 2;
      // as in gmres(): with a double basis an instance whose estimate met its tolerance has
      // converged; the others (and every instance with a float basis) take the true residual
      unsigned rest = fin;
      for (int i = 0; i < B; ++i) {
        if (!has(fin, i)) continue;
        total[i] += cols[i];
        its[i] = total[i];
        if (sizeof(T) == sizeof(double) && gslot(G, i)[kHostGiv + 1] <= tol[i]) {
          rest &= ~(1u << i);
          live &= ~(1u << i);
        }
      }
      if (rest) {
        const pf::Bat br = gbat(G, rest);
        jv<double>(p, 0.0, Bm, p->S, p->w, br);
        pf::launch_axpby<double, double, double>(n, -1.0, p->F, -1.0, p->w, p->tmp, p->stream,
                                                 gbat_s(G, rest, -1.0));
        pf::launch_multidot<double>(n, 0, p->tmp, 0, p->tmp, p->part, p->stream, br);
        pf::launch_finalize(p->part, 1, p->red, p->stream, G->hs, br);
        G->launches += 3;
        int st = gsync(G);
        if (st) return st;
        for (int i = 0; i < B; ++i) {
          if (!has(rest, i)) continue;
          beta[i] = std::sqrt(gslot(G, i)[0]);
          if (beta[i] <= tol[i] || total[i] >= maxit) live &= ~(1u << i);
        }
      }
    }
    live &= ~*bad;
  }
  return PFNKS_OK;
}

}  // namespace

extern "C" {

int pfnks_group_workspace_bytes(const pfnks_grid* grid, const pfnks_model* model, const pfnks_solver* solver,
                                int count, size_t* bytes) {
  if (!bytes || count < 1 || count > pf::kMaxBatch) return PFNKS_EINVAL;
  size_t one = 0;
  int st = pfnks_workspace_bytes(grid, model, solver, &one);
  if (st) return st;
  *bytes = one * (size_t)count;
  return PFNKS_OK;
}

int pfnks_group_create(const pfnks_grid* grid, const pfnks_model* model, const pfnks_solver* solver, int count,
                       const double* c0, const double* eta0, void* d_workspace, size_t ws_bytes, void* hip_stream,
                       pfnks_group** out) {
  if (!out || !c0 || !eta0 || !d_workspace || count < 1 || count > pf::kMaxBatch) return PFNKS_EINVAL;
  *out = nullptr;
  int st = validate(grid, model, solver);
  if (st) return st;
  if (((uintptr_t)d_workspace & 255) != 0) return PFNKS_EINVAL;
  const long long N = (long long)grid->n[0] * grid->n[1] * (grid->dim == 3 ? grid->n[2] : 1);
  const Layout L = make_layout(grid->dim, N, solver->gmres_restart, grid->n, solver->precision, ext_nodes(grid, solver),
                               tiles_summed(grid, solver), tiles_packed(grid, solver));
  if (ws_bytes / (size_t)count < L.total) return PFNKS_ENOSPACE;
  for (int i = 0; i < count; ++i) {
    st = check_domain_host(c0 + (size_t)i * N, eta0 + (size_t)i * 3 * N, N);
    if (st) return st;
  }
  pfnks_problem* p = nullptr;
  st = setup_problem(grid, model, solver, L, N, (char*)d_workspace, (hipStream_t)hip_stream, &p);
  if (st) return st;
  pfnks_group* G = new pfnks_group();
  G->p = p;
  G->count = count;
  G->stride = (long long)L.total;
  G->hs = nullptr;
  G->cbar0.assign(count, 0.0);
  G->t.assign(count, 0.0);
  G->dt.assign(count, 0.0);
  G->launches = G->syncs = 0;
  auto fail = [&](int code) {
    destroy_problem(p);
    if (G->hs) (void)hipHostFree(G->hs);
    delete G;
    return code;
  };
  hipError_t e = hipHostMalloc((void**)&G->hs, sizeof(double) * kHostSlot * count, hipHostMallocDefault);
  if (e != hipSuccess) return fail(device_error(e, "hipHostMalloc"));
  // states: c, eta, u = 0
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    double* Xn = pf::bat_at(p->Xn, i * G->stride);
    e = hipMemcpy(Xn, c0 + (size_t)i * N, sizeof(double) * N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(Xn + N, eta0 + (size_t)i * 3 * N, sizeof(double) * 3 * N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(Xn + 4 * N, 0, sizeof(double) * grid->dim * N);
  }
  if (e != hipSuccess) return fail(device_error(e, "state upload"));
  // cbar0 of every instance, then u0 from the discrete equilibrium at c0 (as pfnks_create_problem)
  const pf::Bat ball = gbat(G, all_mask(count));
  pf::launch_sum2(N, p->Xn, p->Xn, p->Xn, p->part, p->stream, ball);
  pf::launch_finalize(p->part, 1, p->red, p->stream, G->hs, ball);
  st = gsync(G);
  if (st) return fail(st);
  for (int i = 0; i < count; ++i) G->cbar0[i] = gslot(G, i)[0] / (double)N;
  pf::launch_spectral_solve<double>(p->K, p->plan, nullptr, p->K.eps0 * p->K.Ctr, p->Xn, p->fft0, p->fft1,
                                    p->Xn + 4 * N, p->stream, ball);
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return fail(device_error(e, "elastic init"));
  *out = G;
  return PFNKS_OK;
}

int pfnks_group_step(pfnks_group* G, const double* dts, pfnks_step_stats* stats, int* status) {
  if (!G || !dts) return PFNKS_EINVAL;
  const int B = G->count;
  for (int i = 0; i < B; ++i)
    if (!(dts[i] >= 0.0) || !std::isfinite(dts[i])) return PFNKS_EINVAL;
  pfnks_problem* p = G->p;
  // instances with dt = 0 sit this step out
  unsigned all = 0;
  for (int i = 0; i < B; ++i) {
    G->dt[i] = dts[i];
    if (dts[i] > 0.0) all |= 1u << i;
  }
  G->launches = 0;
  G->syncs = 0;
  const long long n = p->nvec, N = p->N;
  const pfnks_solver& sv = p->solver;
  const double sq = std::sqrt((double)n);
  const double eps_a = sv.newton_atol_rms * sq, xi_a = sv.gmres_atol_rms * sq;
  const bool mixed = sv.precision == PFNKS_MIXED;
  std::vector<pfnks_step_stats> st(B);
  for (int i = 0; i < B; ++i) st[i] = pfnks_step_stats{};
  if (!all) {
    for (int i = 0; i < B; ++i) {
      if (stats) stats[i] = st[i];
      if (status) status[i] = PFNKS_OK;
    }
    return PFNKS_OK;
  }
  std::vector<double> fn(B), r0(B), bad(B), ft(B), badt(B), lam(B, 1.0), tol(B), upd(B, 0.0), ds_prev((size_t)B * 8, 0.0);
  std::vector<int> its(B, 0), newton(B, 0), gm(B, 0), backs(B, 0);
  unsigned conv = 0, failed = 0;
  // X_0 = X^n
  gcopy(G, all, p->Xn, p->X);
  int s = gresidual(G, all, p->X, p->F, fn.data(), bad.data());
  if (s) return s;
  for (int i = 0; i < B; ++i) {
    if (!has(all, i)) continue;
    st[i].res0 = r0[i] = fn[i];
    if (fn[i] <= eps_a || fn[i] == 0.0) conv |= 1u << i;
  }
  for (int it = 0; it < sv.newton_maxit; ++it) {
    const unsigned act = all & ~conv & ~failed;
    if (!act) break;
    // linearise; the preconditioner blocks as in pfnks_step (lagged unless pc_refresh)
    const pf::Bat ba = gbat(G, act);
    const bool build_pc = (it == 0) || sv.pc_refresh;
    double* Bm = p->B;
    if (build_pc && !mixed) {
      pf::launch_linearise(p->K, p->X, p->Xn, (double*)p->Bpc, nullptr, p->stream, ba);
      Bm = (double*)p->Bpc;
    } else {
      pf::launch_linearise(p->K, p->X, p->Xn, p->B, build_pc ? (float*)p->Bpc : nullptr, p->stream, ba);
    }
    G->launches += 1;
    if (build_pc) pc_setup(p, 0.0, ba);
    for (int i = 0; i < B; ++i)
      if (has(act, i)) tol[i] = std::fmax(sv.gmres_rtol * fn[i], xi_a);
    unsigned gbad = 0;
    s = mixed ? gmres_group<float>(G, act, Bm, fn.data(), tol.data(), its.data(), &gbad)
              : gmres_group<double>(G, act, Bm, fn.data(), tol.data(), its.data(), &gbad);
    if (s) return s;
    for (int i = 0; i < B; ++i)
      if (has(act, i)) gm[i] += its[i];
    failed |= gbad;
    const unsigned lsm = act & ~gbad;
    if (!lsm) continue;
    // mass projection sums (device), then the backtracking line search of pfnks_step
    double* msums = p->red + kRedMassSlot;
    pf::launch_sum2(N, p->S, p->X, p->Xn, p->part, p->stream, gbat(G, lsm));
    pf::launch_finalize(p->part, 2, msums, p->stream, nullptr, gbat(G, lsm));
    G->launches += 2;
    unsigned ls = lsm, accepted = 0;
    for (int i = 0; i < B; ++i) lam[i] = 1.0;
    for (int hv = 0; hv <= sv.ls_max_halvings && ls; ++hv) {
      pf::Bat bl = gbat(G, ls);
      for (int i = 0; i < B; ++i) bl.s[i] = lam[i];
      pf::launch_trial(p->K, p->nf, p->X, p->S, 0.0, msums, p->Xt, p->part, hv == 0 ? p->part + pf::kRedBlocks : nullptr,
                       p->stream, bl);
      pf::launch_finalize(p->part, 1, p->red, p->stream, G->hs + 2, bl);
      G->launches += 2;
      if (hv == 0) {
        pf::launch_finalize_max(p->part + pf::kRedBlocks, 2 * p->nf, p->red + kHostUpd, p->stream, G->hs + kHostUpd, bl);
        G->launches += 1;
      }
      s = gresidual(G, ls, p->Xt, p->Ft, ft.data(), badt.data());
      if (s) return s;
      for (int i = 0; i < B; ++i) {
        if (!has(ls, i)) continue;
        const double trial_bad = gslot(G, i)[2];
        if (trial_bad == 0.0 && badt[i] == 0.0 && std::isfinite(ft[i]) &&
            ft[i] * ft[i] <= (1.0 - 2.0 * sv.ls_alpha * lam[i]) * fn[i] * fn[i]) {
          accepted |= 1u << i;
          ls &= ~(1u << i);
        } else {
          lam[i] *= 0.5;
          ++backs[i];
        }
      }
    }
    failed |= lsm & ~accepted;
    if (!accepted) continue;
    gcopy(G, accepted, p->Xt, p->X);
    gcopy(G, accepted, p->Ft, p->F);
    for (int i = 0; i < B; ++i) {
      if (!has(accepted, i)) continue;
      fn[i] = ft[i];
      ++newton[i];
      // update test of pfnks_step, on this instance's maxima
      const double* h = gslot(G, i);
      double ds[8], xs[8], theta = 0.0;
      for (int f = 0; f < p->nf; ++f) {
        ds[f] = lam[i] * h[kHostUpd + 2 * f];
        xs[f] = h[kHostUpd + 2 * f + 1];
        const double prev = ds_prev[(size_t)i * 8 + f];
        if (ds[f] > 0.0) theta = std::fmax(theta, prev > 0.0 ? ds[f] / prev : HUGE_VAL);
      }
      const double amp = (theta < 1.0) ? theta / (1.0 - theta) : HUGE_VAL;
      bool small_update = true;
      upd[i] = 0.0;
      for (int f = 0; f < p->nf; ++f) {
        if (ds[f] == 0.0) continue;
        const double est = ds[f] * amp;
        upd[i] = std::fmax(upd[i], xs[f] > 0.0 ? est / xs[f] : HUGE_VAL);
        if (!(est <= sv.newton_stol * xs[f])) small_update = false;
      }
      for (int f = 0; f < p->nf; ++f) ds_prev[(size_t)i * 8 + f] = ds[f];
      if (sv.newton_stol <= 0.0) small_update = true;
      if (fn[i] <= eps_a || (fn[i] <= sv.newton_rtol * r0[i] && small_update)) conv |= 1u << i;
    }
  }
  const unsigned ok = conv & ~failed;
  for (int i = 0; i < B; ++i) {
    if (!has(all, i)) {
      st[i].status = PFNKS_OK;  // sat the step out
      continue;
    }
    st[i].newton_its = newton[i];
    st[i].gmres_its = gm[i];
    st[i].ls_backtracks = backs[i];
    st[i].res_final = fn[i];
    st[i].update_rel = upd[i];
    st[i].status = has(ok, i) ? PFNKS_OK : PFNKS_ENOCONV;
  }
  if (ok) {
    // step close of the converged instances: gauge projection, ||X - X^n||, energy, mass
    const pf::Bat bo = gbat(G, ok);
    const int ncls = 1 << p->grid.dim;
    pf::launch_class_sums(p->K, p->X + 4 * N, p->part, p->stream, bo);
    pf::launch_finalize(p->part, p->grid.dim * ncls, p->red, p->stream, nullptr, bo);
    pf::launch_class_shift(p->K, p->X + 4 * N, p->red, p->stream, bo);
    pf::launch_dx2(4 * N, p->X, p->Xn, p->part, p->stream, bo);
    pf::launch_finalize(p->part, 1, p->red, p->stream, G->hs + 4, bo);
    pf::launch_energy(p->K, p->X, p->part, p->stream, bo);
    pf::launch_finalize(p->part, 4, p->red, p->stream, G->hs, bo);
    G->launches += 7;
    gcopy(G, ok, p->X, p->Xn);
  }
  s = gsync(G);
  if (s) return s;
  const double hd = std::pow(p->grid.h, p->grid.dim);
  for (int i = 0; i < B; ++i) {
    if (!has(ok, i)) continue;
    const double* h = gslot(G, i);
    st[i].energy_parts[0] = h[0] * hd;
    st[i].energy_parts[1] = h[1] * hd;
    st[i].energy_parts[2] = h[2] * hd;
    st[i].energy = st[i].energy_parts[0] + st[i].energy_parts[1] + st[i].energy_parts[2];
    st[i].mass = h[3] * hd;
    st[i].dx_rms = std::sqrt(h[4] / (4.0 * N));
    G->t[i] += dts[i];
  }
  int first = PFNKS_OK;
  for (int i = 0; i < B; ++i) {
    if (stats) stats[i] = st[i];
    if (status) status[i] = st[i].status;
    if (first == PFNKS_OK && st[i].status != PFNKS_OK) first = st[i].status;
  }
  return first;
}

int pfnks_group_set_instance(pfnks_group* G, int i, const double* c0, const double* eta0) {
  if (!G || !c0 || !eta0 || i < 0 || i >= G->count) return PFNKS_EINVAL;
  pfnks_problem* p = G->p;
  const long long N = p->N;
  int st = check_domain_host(c0, eta0, N);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(p->stream));
  double* Xn = pf::bat_at(p->Xn, i * G->stride);
  HIPCHK(hipMemcpyAsync(Xn, c0, sizeof(double) * N, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(Xn + N, eta0, sizeof(double) * 3 * N, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemsetAsync(Xn + 4 * N, 0, sizeof(double) * p->grid.dim * N, p->stream));
  // its mean composition, then u0 from the discrete equilibrium at c0 (as at creation)
  const pf::Bat bi = gbat(G, 1u << i);
  pf::launch_sum2(N, p->Xn, p->Xn, p->Xn, p->part, p->stream, bi);
  pf::launch_finalize(p->part, 1, p->red, p->stream, G->hs, bi);
  st = gsync(G);
  if (st) return st;
  G->cbar0[i] = gslot(G, i)[0] / (double)N;
  pf::launch_spectral_solve<double>(p->K, p->plan, nullptr, p->K.eps0 * p->K.Ctr, p->Xn, p->fft0, p->fft1,
                                    p->Xn + 4 * N, p->stream, gbat(G, 1u << i));
  HIPCHK(hipStreamSynchronize(p->stream));
  G->t[i] = 0.0;
  return PFNKS_OK;
}

int pfnks_group_get_state(pfnks_group* G, int i, double* X, double* t) {
  if (!G || !X || i < 0 || i >= G->count) return PFNKS_EINVAL;
  pfnks_problem* p = G->p;
  HIPCHK(hipMemcpyAsync(X, pf::bat_at(p->Xn, i * G->stride), sizeof(double) * p->nvec, hipMemcpyDeviceToHost,
                        p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  if (t) *t = G->t[i];
  return PFNKS_OK;
}

int pfnks_group_counters(pfnks_group* G, long long* launches, long long* syncs) {
  if (!G) return PFNKS_EINVAL;
  if (launches) *launches = G->launches;
  if (syncs) *syncs = G->syncs;
  return PFNKS_OK;
}

int pfnks_group_destroy(pfnks_group* G) {
  if (!G) return PFNKS_EINVAL;
  if (G->p->stream) (void)hipStreamSynchronize(G->p->stream);
  destroy_problem(G->p);
  if (G->hs) (void)hipHostFree(G->hs);
  delete G;
  return PFNKS_OK;
}

int pfnks_energy(pfnks_problem* p, double* total, double parts[3]) {
  if (!p || !total) return PFNKS_EINVAL;
  pfnks_step_stats st{};
  int s = step_close(p, &st, p->Xn, 0.0);
  if (s) return s;
  *total = st.energy;
  if (parts)
    for (int k = 0; k < 3; ++k) parts[k] = st.energy_parts[k];
  return PFNKS_OK;
}

int pfnks_mass(pfnks_problem* p, double* mass) {
  if (!p || !mass) return PFNKS_EINVAL;
  pfnks_step_stats st{};
  int s = step_close(p, &st, p->Xn, 0.0);
  if (s) return s;
  *mass = st.mass;
  return PFNKS_OK;
}

int pfnks_get_state(pfnks_problem* p, double* X, double* t) {
  if (!p || !X) return PFNKS_EINVAL;
  HIPCHK(hipMemcpyAsync(X, p->Xn, sizeof(double) * p->nvec, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  if (t) *t = p->t;
  return PFNKS_OK;
}

int pfnks_set_state(pfnks_problem* p, const double* X, double t) {
  if (!p || !X) return PFNKS_EINVAL;
  int s = check_domain_host(X, X + p->N, p->N);
  if (s) return s;
  HIPCHK(hipMemcpyAsync(p->Xn, X, sizeof(double) * p->nvec, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  p->t = t;
  return PFNKS_OK;
}

int pfnks_destroy(pfnks_problem* p) {
  if (!p) return PFNKS_EINVAL;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  prof_resolve(p);
  destroy_problem(p);
  return PFNKS_OK;
}

int pfnks_debug_profile(pfnks_problem* p, int enable) {
  if (!p) return PFNKS_EINVAL;
  HIPCHK(hipStreamSynchronize(p->stream));
  prof_resolve(p);
  p->prof = enable & ((1 << PFNKS_KERNEL_KINDS) - 1);
  for (int k = 0; k < PFNKS_KERNEL_KINDS; ++k) {
    p->kcount[k] = 0;
    p->kms[k] = 0.0;
    p->kbytes[k] = 0.0;
  }
  return PFNKS_OK;
}

int pfnks_debug_kernel_time(pfnks_problem* p, int kind, long long* launches, double* ms_total,
                            double* bytes_total) {
  if (!p || kind < 0 || kind >= PFNKS_KERNEL_KINDS) return PFNKS_EINVAL;
  HIPCHK(hipStreamSynchronize(p->stream));
  prof_resolve(p);
  if (launches) *launches = p->kcount[kind];
  if (ms_total) *ms_total = p->kms[kind];
  if (bytes_total) *bytes_total = p->kbytes[kind];
  return PFNKS_OK;
}

const char* pfnks_strerror(int status) {
  switch (status) {
    case PFNKS_OK: return "ok";
    case PFNKS_EINVAL: return "invalid argument";
    case PFNKS_EDOMAIN: return "state outside the log domain (need 0 < c < 1 and 0 < c*eta_i < 1)";
    case PFNKS_ENOSPACE: return "workspace too small";
    case PFNKS_ENOCONV: return "Newton iteration did not converge";
    case PFNKS_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* pfnks_last_error(void) { return g_last_error.c_str(); }

int pfnks_debug_residual(pfnks_problem* p, const double* X, double dt, double* F) {
  if (!p || !X || !F || !(dt > 0.0)) return PFNKS_EINVAL;
  HIPCHK(hipMemcpyAsync(p->Xt, X, sizeof(double) * p->nvec, hipMemcpyHostToDevice, p->stream));
  double fn, bad;
  int s = residual(p, p->Xt, dt, p->Ft, &fn, &bad);
  if (s) return s;
  HIPCHK(hipMemcpyAsync(F, p->Ft, sizeof(double) * p->nvec, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return PFNKS_OK;
}

int pfnks_debug_jv(pfnks_problem* p, const double* X, double dt, const double* v, double* w) {
  if (!p || !X || !v || !w || !(dt > 0.0)) return PFNKS_EINVAL;
  HIPCHK(hipMemcpyAsync(p->Xt, X, sizeof(double) * p->nvec, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(p->tmp, v, sizeof(double) * p->nvec, hipMemcpyHostToDevice, p->stream));
  pf::launch_linearise(p->K, p->Xt, p->Xn, p->B, nullptr, p->stream);
  jv<double>(p, dt, p->B, p->tmp, p->w);
  HIPCHK(hipMemcpyAsync(w, p->w, sizeof(double) * p->nvec, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return PFNKS_OK;
}

int pfnks_debug_pc(pfnks_problem* p, const double* X, double dt, const double* r, double* z) {
  if (!p || !X || !r || !z || !(dt > 0.0)) return PFNKS_EINVAL;
  HIPCHK(hipMemcpyAsync(p->Xt, X, sizeof(double) * p->nvec, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(p->tmp, r, sizeof(double) * p->nvec, hipMemcpyHostToDevice, p->stream));
  if (p->solver.precision == PFNKS_MIXED) {
    // the preconditioner in float: r rounded to float, z widened back to double
    pf::launch_linearise(p->K, p->Xt, p->Xn, p->B, (float*)p->Bpc, p->stream);
    pc_setup(p, dt);
    pf::launch_axpby<double, double, float>(p->nvec, 1.0, p->tmp, 0.0, nullptr, (float*)p->tmpv, p->stream);
    pc_apply<float>(p, dt, (const float*)p->tmpv, (float*)p->z);
    pf::launch_axpby<float, float, double>(p->nvec, 1.0, (const float*)p->z, 0.0, nullptr, p->w, p->stream);
  } else {
    pf::launch_linearise(p->K, p->Xt, p->Xn, (double*)p->Bpc, nullptr, p->stream);
    pc_setup(p, dt);
    pc_apply<double>(p, dt, p->tmp, (double*)p->z);
    HIPCHK(hipMemcpyAsync(p->w, p->z, sizeof(double) * p->nvec, hipMemcpyDeviceToDevice, p->stream));
  }
  HIPCHK(hipMemcpyAsync(z, p->w, sizeof(double) * p->nvec, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return PFNKS_OK;
}

int pfnks_debug_counters(pfnks_problem* p, long long* launches, long long* syncs) {
  if (!p) return PFNKS_EINVAL;
  if (launches) *launches = p->launches;
  if (syncs) *syncs = p->syncs;
  return PFNKS_OK;
}

}  // extern "C"
