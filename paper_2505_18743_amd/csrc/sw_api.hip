// Host side of the C ABI declared in include/sw.h: validation, quadtree faces,
// reference tables, device memory, and the per-step launch sequence.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "sw.h"
#include "sw_internal.h"

namespace swk {
hipError_t launch_stage_r1(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_stage_r2(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_stage_r3(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);

hipError_t launch_stage(int r, int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_stage_r1(P, mode, a, nblk, s);
    case 2: return launch_stage_r2(P, mode, a, nblk, s);
    case 3: return launch_stage_r3(P, mode, a, nblk, s);
  }
  return hipErrorInvalidValue;
}

__global__ void k_bathy(const double*, const double*, double*, int, int, int, size_t);
__global__ void k_facez(const int*, const int*, const int*, int, int, int, int, int, size_t, const double*,
                        const double*, const double*, double*, int*, int);
__global__ void k_cellinit(LevelTabs, int, int, size_t, int, const double*, double*, double*);
__global__ void k_lake(LevelTabs, int, int, size_t, int, const double*, const double*, const double*, double*,
                       double*, double*);
__global__ void k_set(double*, int, double);
__global__ void k_fill(double*, size_t, double);
__global__ void k_fill8(int8_t*, size_t, int8_t);
__global__ void k_copy(const double*, double*, size_t);
__global__ void k_minred(const double*, int, double*);
__global__ void k_dt(const double*, int, double, double, double*);
__global__ void k_diag_part(const double*, const int8_t*, int, double*);
__global__ void k_diag(const double*, int, double*, double*);

hipError_t launch_elem_r1(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_elem_r2(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_elem_r3(int P, int mode, const StageArgs& a, int nblk, hipStream_t s);

hipError_t launch_elem(int r, int P, int mode, const StageArgs& a, int nblk, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  switch (r) {
    case 1: return launch_elem_r1(P, mode, a, nblk, s);
    case 2: return launch_elem_r2(P, mode, a, nblk, s);
    case 3: return launch_elem_r3(P, mode, a, nblk, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace swk

using namespace swk;

namespace {

thread_local std::string g_err;

sw_status fail(sw_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) return fail(SW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// 1-D reference data: Legendre polynomials, GLL / GL / equispaced rules on [0,1],
// Lagrange basis on the GLL support points (Sec. 3.2).
// ---------------------------------------------------------------------------
void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = (std::fabs(x) < 1.0) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.5 * n * (n + 1.0) * (x > 0 ? 1.0 : (n % 2 ? 1.0 : -1.0));
}

// n-point Lobatto rule: end points and the roots of P'_{n-1}, weights 2/(N(N+1)P_N^2)
void gll(int n, std::vector<double>& x, std::vector<double>& w) {
  const int N = n - 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  std::vector<double> t(n);
  t[0] = -1.0;
  t[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double xi = -std::cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(N, xi, p, dp);
      const double d2 = (2.0 * xi * dp - N * (N + 1.0) * p) / (1.0 - xi * xi);
      const double dx = dp / d2;
      xi -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    t[i] = xi;
  }
  for (int i = 0; i < n; ++i) {
    double p, dp;
    legendre(N, t[i], p, dp);
    x[i] = (t[i] + 1.0) * 0.5;
    w[i] = 1.0 / (N * (N + 1.0) * p * p);   // 2/(N(N+1)P^2) halved for [0,1]
  }
  x[0] = 0.0;
  x[N] = 1.0;
}

void gl(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double xi = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, xi, p, dp);
      const double dx = p / dp;
      xi -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double p, dp;
    legendre(n, xi, p, dp);
    x[i] = (xi + 1.0) * 0.5;
    w[i] = 1.0 / ((1.0 - xi * xi) * dp * dp);
  }
}

void eqr(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.assign(n, 1.0 / (n - 1));
  for (int i = 0; i < n; ++i) x[i] = (double)i / (n - 1);
  w[0] = w[n - 1] = 0.5 / (n - 1);
}

double lag(const std::vector<double>& xi, int j, double x) {
  double v = 1.0;
  for (size_t m = 0; m < xi.size(); ++m)
    if ((int)m != j) v *= (x - xi[m]) / (xi[j] - xi[m]);
  return v;
}

double dlag(const std::vector<double>& xi, int j, double x) {
  double s = 0.0;
  for (size_t k = 0; k < xi.size(); ++k) {
    if ((int)k == j) continue;
    double v = 1.0 / (xi[j] - xi[k]);
    for (size_t m = 0; m < xi.size(); ++m)
      if ((int)m != j && m != k) v *= (x - xi[m]) / (xi[j] - xi[m]);
    s += v;
  }
  return s;
}

// In-place inverse of an SPD matrix via Cholesky (n <= 16).
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return false;
    L[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  std::vector<double> inv(n * n, 0.0), e(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * e[k];
      e[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = e[i];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * e[k];
      e[i] = s / L[i * n + i];
    }
    for (int i = 0; i < n; ++i) inv[i * n + c] = e[i];
  }
  A = inv;
  return true;
}

struct LevelH {
  int L = 0, S = 0, P = 0;
  double dx = 0, w1 = 0;
  int cell0 = 0, ncell = 0;
  size_t off = 0;          // offset of this level's samples in the node arrays
  int face0 = 0, nface = 0;  // all faces whose fine (or equal) side is on this level
  size_t zfoff = 0;          // offset of this level's faces in the face-sample array
  // face classes: direction (x: W/E, y: S/N) x (conforming or boundary, sub-face 0,
  // sub-face 1); the faces of one class touch disjoint (cell, dof) sets
  int cface0[6]{}, cnface[6]{}, cfblk0[6]{}, cfnblk[6]{};
  int nblk = 0;              // element-kernel blocks
  std::vector<double> xh, wh;
  double* d_tab = nullptr;
  LevelTabs tabs{};
};

}  // namespace

struct sw_ctx {
  int dev = 0;
  hipStream_t s = nullptr;
  sw_params p{};
  int r = 1, N1 = 2, NP = 4, K = 0, F = 0, ns = 3;
  int64_t nvol = 0;
  int nx0 = 0, ny0 = 0;
  double x0 = 0, y0 = 0, dx0 = 0;
  std::vector<int> lev, ci, cj;
  std::vector<LevelH> lv;
  double A[4][4]{}, b[4]{}, c[4]{};
  int *d_fA = nullptr, *d_fB = nullptr, *d_meta = nullptr, *d_err = nullptr;
  double *d_zb = nullptr, *d_braw = nullptr, *d_db = nullptr, *d_bvec = nullptr, *d_zmax = nullptr;
  double *d_nman = nullptr, *d_cdx = nullptr, *d_cw1 = nullptr, *d_zf = nullptr;
  double *d_sn[4]{}, *d_ss[4]{};
  double *d_hn = nullptr, *d_cn = nullptr, *d_res = nullptr;
  double *d_scal = nullptr, *d_cdiag = nullptr, *d_bpart = nullptr, *d_red = nullptr, *d_diag = nullptr;
  int8_t *d_flag = nullptr, *d_allwet = nullptr, *d_need = nullptr;
  int fblk_total = 0;
  bool start_ready = false;   // H^n, stage-1 volume terms and degrees of the current state are in place
  bool fixed_dt = false;
  bool bathy_set = false;
  int stage_done = 0;      // stages completed in the current step (0: no step open)
  int64_t nstep = 0;
  std::vector<void*> allocs;
  // kernel timing (sw_profile): events recorded around each launch group
  bool prof = false;
  struct Ev { int kind; int nlaunch; hipEvent_t a, b; };
  std::vector<Ev> ev;
  double prof_ms[8]{};
  int64_t prof_n[8]{};

  template <class T>
  sw_status alloc(T** p, size_t n) {
    void* q = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&q, n * sizeof(T));
    if (e != hipSuccess) return fail(SW_ENOMEM, "hipMalloc failed for " + std::to_string(n * sizeof(T)) + " bytes");
    allocs.push_back(q);
    *p = (T*)q;
    return SW_OK;
  }
  ~sw_ctx() {
    for (auto& e : ev) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (void* q : allocs) (void)hipFree(q);
  }
  // bracket a group of launches of one kernel class with events when profiling
  struct Scope {
    sw_ctx* c;
    int kind, n;
    hipEvent_t a{}, b{};
    bool on = false;
    Scope(sw_ctx* c_, int k, int n_) : c(c_), kind(k), n(n_) {
      if (!c->prof) return;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
      on = hipEventRecord(a, c->s) == hipSuccess;
    }
    ~Scope() {
      if (!on) return;
      (void)hipEventRecord(b, c->s);
      c->ev.push_back({kind, n, a, b});
    }
  };
};

namespace {

constexpr int kNSlot = 5;   // residual slots: up to 4 stages + one for sw_apply_operator
constexpr int kApplySlot = 4;

void tableau(int rk, int& s, double A[4][4], double b[4], double c[4]) {
  for (int i = 0; i < 4; ++i) {
    b[i] = c[i] = 0.0;
    for (int j = 0; j < 4; ++j) A[i][j] = 0.0;
  }
  if (rk == SW_RK_FE) {
    s = 1;
    b[0] = 1.0;
  } else if (rk == SW_RK_SSP3) {
    s = 3;
    A[1][0] = 1.0;
    A[2][0] = 0.25;
    A[2][1] = 0.25;
    b[0] = 1.0 / 6.0;
    b[1] = 1.0 / 6.0;
    b[2] = 2.0 / 3.0;
    c[1] = 1.0;
    c[2] = 0.5;
  } else if (rk == SW_RK_RK32) {
    s = 3;
    const double chi = 1.0 - std::sqrt(2.0) / 2.0, a32 = 0.5;
    A[1][0] = 2.0 * chi;
    A[2][0] = 1.0 - a32;
    A[2][1] = a32;
    const double b2 = (1.0 - 2.0 * chi) / (4.0 * chi);
    b[0] = 1.0 - b2 - chi;
    b[1] = b2;
    b[2] = chi;
    c[1] = 2.0 * chi;
    c[2] = 1.0;
  } else {
    s = 4;
    A[1][0] = 0.5;
    A[2][1] = 0.5;
    A[3][2] = 1.0;
    b[0] = 1.0 / 6.0;
    b[1] = 2.0 / 6.0;
    b[2] = 2.0 / 6.0;
    b[3] = 1.0 / 6.0;
    c[1] = 0.5;
    c[2] = 0.5;
    c[3] = 1.0;
  }
}

int64_t key(int L, int i, int j) { return ((int64_t)L << 52) | ((int64_t)i << 26) | (int64_t)j; }

sw_status build_tables(sw_ctx* c, LevelH& L) {
  const int S = L.S, N1 = c->N1, NP = c->NP;
  if (c->p.rule == SW_RULE_EQ) eqr(S, L.xh, L.wh);
  else gll(S, L.xh, L.wh);
  std::vector<double> wb, xi;
  gll(N1, xi, wb);          // support points
  std::vector<double> tab;
  const size_t o_w = 0, o_l = o_w + S, o_d = o_l + (size_t)S * N1, o_m0 = o_d + (size_t)S * N1,
               o_mq = o_m0 + (size_t)NP * NP, o_mean = o_mq + (size_t)NP * NP, o_fl = o_mean + NP,
               o_dp = o_fl + (size_t)3 * S * N1, o_wl = o_dp + (size_t)S * N1, o_wdp = o_wl + (size_t)S * N1,
               total = o_wdp + (size_t)S * N1;
  tab.assign(total, 0.0);
  for (int a = 0; a < S; ++a) {
    tab[o_w + a] = L.wh[a];
    for (int k = 0; k < N1; ++k) {
      tab[o_l + a * N1 + k] = lag(xi, k, L.xh[a]);
      tab[o_d + a * N1 + k] = dlag(xi, k, L.xh[a]);
      tab[o_fl + (0 * S + a) * N1 + k] = lag(xi, k, L.xh[a]);
      tab[o_fl + (1 * S + a) * N1 + k] = lag(xi, k, 0.5 * L.xh[a]);
      tab[o_fl + (2 * S + a) * N1 + k] = lag(xi, k, 0.5 * (1.0 + L.xh[a]));
      tab[o_dp + a * N1 + k] = dlag(xi, k, L.xh[a]) / L.dx;
      tab[o_wl + a * N1 + k] = L.wh[a] * lag(xi, k, L.xh[a]);
      tab[o_wdp + a * N1 + k] = L.wh[a] * dlag(xi, k, L.xh[a]) / L.dx;
    }
  }
  // all-wet mass matrix of the sample rule on the unit square, and its inverse
  std::vector<double> M0(NP * NP, 0.0), Mq(NP * NP, 0.0);
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j < NP; ++j) {
      double s = 0.0;
      for (int b = 0; b < S; ++b)
        for (int a = 0; a < S; ++a)
          s += L.wh[a] * L.wh[b] * tab[o_l + a * N1 + i % N1] * tab[o_l + b * N1 + i / N1] *
               tab[o_l + a * N1 + j % N1] * tab[o_l + b * N1 + j / N1];
      M0[i * NP + j] = s;
    }
  // exact mass matrix (Gauss-Legendre with r+1 points per direction, Table 1)
  std::vector<double> xg, wg;
  gl(N1, xg, wg);
  std::vector<double> mean(NP, 0.0);
  for (int i = 0; i < NP; ++i)
    for (int j = 0; j < NP; ++j) {
      double s = 0.0;
      for (int b = 0; b < N1; ++b)
        for (int a = 0; a < N1; ++a)
          s += wg[a] * wg[b] * lag(xi, i % N1, xg[a]) * lag(xi, i / N1, xg[b]) * lag(xi, j % N1, xg[a]) *
               lag(xi, j / N1, xg[b]);
      Mq[i * NP + j] = s;
    }
  for (int j = 0; j < NP; ++j) {
    double s = 0.0;
    for (int b = 0; b < N1; ++b)
      for (int a = 0; a < N1; ++a) s += wg[a] * wg[b] * lag(xi, j % N1, xg[a]) * lag(xi, j / N1, xg[b]);
    mean[j] = s;
  }
  if (!spd_inverse(M0, NP) || !spd_inverse(Mq, NP)) return fail(SW_EINVAL, "reference mass matrix not SPD");
  for (int i = 0; i < NP * NP; ++i) {
    tab[o_m0 + i] = M0[i];
    tab[o_mq + i] = Mq[i];
  }
  for (int j = 0; j < NP; ++j) tab[o_mean + j] = mean[j];
  sw_status st = c->alloc(&L.d_tab, total);
  if (st != SW_OK) return st;
  HIPCHK(hipMemcpy(L.d_tab, tab.data(), total * sizeof(double), hipMemcpyHostToDevice));
  L.tabs.w = L.d_tab + o_w;
  L.tabs.l = L.d_tab + o_l;
  L.tabs.d = L.d_tab + o_d;
  L.tabs.m0inv = L.d_tab + o_m0;
  L.tabs.mqinv = L.d_tab + o_mq;
  L.tabs.meanw = L.d_tab + o_mean;
  L.tabs.fl = L.d_tab + o_fl;
  L.tabs.dp = L.d_tab + o_dp;
  L.tabs.wl = L.d_tab + o_wl;
  L.tabs.wdp = L.d_tab + o_wdp;
  L.tabs.S = S;
  L.tabs.dx = L.dx;
  L.w1 = L.wh[0];
  return SW_OK;
}

sw_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(SW_EINVAL, std::string(name) + " is NULL");
  return SW_OK;
}

StageArgs stage_args(sw_ctx* c, const LevelH& L) {
  StageArgs a{};
  a.t = L.tabs;
  a.cell0 = L.cell0;
  a.ncell = L.ncell;
  a.K = c->K;
  a.zb = c->d_zb + L.off;
  a.bvec = c->d_bvec;
  a.zmax = c->d_zmax;
  a.nman = c->d_nman;
  for (int f = 0; f < 4; ++f) {
    a.sn[f] = c->d_sn[f];
    a.ss[f] = c->d_ss[f];
    a.in[f] = nullptr;
    a.out[f] = nullptr;
  }
  a.hn = c->d_hn;
  a.cn = c->d_cn;
  a.res = c->d_res;
  a.flag = c->d_flag;
  a.need = nullptr;
  a.cdiag = c->d_cdiag;
  a.diag_init = 0;
  a.allwet = c->d_allwet;
  a.scal = c->d_scal;
  a.err = c->d_err;
  a.slot = 0;
  a.nterm = 0;
  a.g = c->p.g;
  a.eps = c->p.eps;
  a.hlim = c->p.h_lim;
  a.eps0 = c->p.eps0;
  a.newton_max = c->p.newton_max;
  a.tracer = c->p.tracer ? 1 : 0;
  a.fric = 1;
  a.adapt = c->p.adapt_degree ? 1 : 0;
  return a;
}

FaceArgs face_args(sw_ctx* c, const LevelH& L, int cls, const double* const* st, double cstage, int slot) {
  FaceArgs a{};
  a.face0 = L.cface0[cls];
  a.nface = L.cnface[cls];
  a.K = c->K;
  a.S = L.S;
  a.fA = c->d_fA;
  a.fB = c->d_fB;
  a.meta = c->d_meta;
  a.zf = c->d_zf + L.zfoff + (size_t)(L.cface0[cls] - L.face0) * 2 * L.S;
  for (int f = 0; f < 4; ++f) a.st[f] = st[f];
  a.res = c->d_res;
  a.slot = slot;
  a.cdx = c->d_cdx;
  a.cw1 = c->d_cw1;
  a.fl = L.tabs.fl;
  a.w = L.tabs.w;
  a.scal = c->d_scal;
  a.cstage = cstage;
  a.bpart = c->d_bpart;
  a.bpart0 = L.cfblk0[cls];
  a.err = c->d_err;
  a.g = c->p.g;
  a.eps = c->p.eps;
  a.tracer = c->p.tracer ? 1 : 0;
  a.tide_amp = c->p.tide_amp;
  a.tide_period = c->p.tide_period;
  a.tide_phase = c->p.tide_phase;
  a.tide_cin = c->p.tide_c_in;
  return a;
}

// all face classes of all levels, adding into residual slot `slot`
sw_status faces(sw_ctx* c, const double* const* st, double cstage, int slot, const double* scal_override = nullptr) {
  int n = 0;
  for (auto& L : c->lv)
    for (int k = 0; k < 6; ++k) n += L.cnface[k] > 0;
  sw_ctx::Scope sc(c, 3, n);
  for (auto& L : c->lv)
    for (int k = 0; k < 6; ++k) {
      if (L.cnface[k] == 0) continue;
      FaceArgs fa = face_args(c, L, k, st, cstage, slot);
      if (scal_override) fa.scal = scal_override;
      HIPCHK(launch_face(c->r, L.P, fa, L.cfnblk[k], c->s));
    }
  return SW_OK;
}

// dt = cfl * min of the face kernels' block bounds (two-level reduction)
sw_status reduce_dt(sw_ctx* c, double cfl, double* dst) {
  if (c->fblk_total == 0) return SW_OK;
  const int n1 = (c->fblk_total + 1023) / 1024;
  hipLaunchKernelGGL(k_minred, dim3(n1), dim3(256), 0, c->s, c->d_bpart, c->fblk_total, c->d_red);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, c->s, c->d_red, n1, cfl, 0.0, dst);
  HIPCHK(hipGetLastError());
  return SW_OK;
}

// element work of one phase on every level: the fast kernel where it applies,
// then the general kernel on the cells it left (or on all cells)
sw_status elements(sw_ctx* c, int fmode, int gmode, int gmode2, int slot, int nterm, const double* coef, int diag_init,
                   int kind) {
  const bool fast_ok = !c->p.tracer;
  for (auto& L : c->lv) {
    StageArgs a = stage_args(c, L);
    a.slot = slot;
    a.nterm = nterm;
    for (int m = 0; m < 4; ++m) a.a[m] = coef ? coef[m] : 0.0;
    a.diag_init = diag_init;
    if (fast_ok) {
      sw_ctx::Scope sc(c, kind, 1);
      a.need = c->d_need;
      HIPCHK(launch_elem(c->r, L.P, fmode, a, L.nblk, c->s));
    }
    StageArgs g = a;
    g.need = fast_ok ? c->d_need : nullptr;
    if (gmode >= 0) {
      sw_ctx::Scope sc(c, 4, 1);
      HIPCHK(launch_stage(c->r, L.P, gmode, g, L.nblk, c->s));
    }
    if (gmode2 >= 0) {
      sw_ctx::Scope sc(c, 4, 1);
      g.slot = 0;
      HIPCHK(launch_stage(c->r, L.P, gmode2, g, L.nblk, c->s));
    }
  }
  return SW_OK;
}

sw_status rebake(sw_ctx* c) {
  c->start_ready = false;
  for (auto& L : c->lv) {
    const size_t n = (size_t)L.ncell * L.S * L.S;
    if (n == 0) continue;
    hipLaunchKernelGGL(k_bathy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->s, c->d_braw, c->d_db, c->d_zb,
                       L.cell0, L.ncell, L.S, L.off);
    HIPCHK(hipGetLastError());
  }
  for (auto& L : c->lv) {
    if (L.nface > 0) {
      const int n = L.nface * L.S;   // all classes of the level: one contiguous range
      hipLaunchKernelGGL(k_facez, dim3((n + 255) / 256), dim3(256), 0, c->s, c->d_fA, c->d_fB, c->d_meta, L.face0,
                         L.nface, L.S, L.cell0, L.ncell, L.off, c->d_zb, c->d_braw, c->d_db, c->d_zf + L.zfoff,
                         c->d_err, c->K);
      HIPCHK(hipGetLastError());
    }
    if (L.ncell > 0) {
      const int n = L.ncell * c->NP;
      hipLaunchKernelGGL(k_cellinit, dim3((n + 127) / 128), dim3(128), 0, c->s, L.tabs, L.cell0, L.ncell, L.off,
                         c->N1, c->d_zb, c->d_bvec, c->d_zmax);
      HIPCHK(hipGetLastError());
    }
  }
  return SW_OK;
}

sw_status need_bathy(const sw_ctx* c) {
  if (!c->bathy_set) return fail(SW_EINVAL, "sw_set_bathymetry has not been called");
  return SW_OK;
}

}  // namespace

extern "C" {

const char* sw_last_error(void) { return g_err.c_str(); }

sw_status sw_create(sw_ctx** out, const sw_mesh_desc* m, const sw_params* p, void* stream) {
  if (!out || !m || !p) return fail(SW_EINVAL, "NULL argument to sw_create");
  *out = nullptr;
  if (p->r < 1 || p->r > 3) return fail(SW_EINVAL, "r must be 1, 2 or 3");
  if (p->rule != SW_RULE_EQ && p->rule != SW_RULE_GLL) return fail(SW_EINVAL, "unknown rule");
  if (p->rk < SW_RK_FE || p->rk > SW_RK_RK44) return fail(SW_EINVAL, "unknown RK scheme");
  if (!(p->eps > 0.0)) return fail(SW_EINVAL, "eps must be > 0");
  if (p->newton_max < 1 || p->newton_max > 1000) return fail(SW_EINVAL, "newton_max out of range");
  if (p->tide_period == 0.0 && (m->bc[0] == SW_BC_ELEV || m->bc[1] == SW_BC_ELEV || m->bc[2] == SW_BC_ELEV ||
                                m->bc[3] == SW_BC_ELEV))
    return fail(SW_EINVAL, "tide_period must be non-zero with an elevation boundary");
  if (m->n_cells < 1 || !m->level || !m->i || !m->j) return fail(SW_EINVAL, "empty mesh");
  if (m->nx0 < 1 || m->ny0 < 1 || !(m->dx0 > 0.0)) return fail(SW_EINVAL, "bad coarse grid");
  for (int s = 0; s < 4; ++s)
    if (m->bc[s] < 0 || m->bc[s] > 3) return fail(SW_EINVAL, "bad boundary kind");
  if ((m->bc[0] == SW_BC_PERIODIC) != (m->bc[1] == SW_BC_PERIODIC) ||
      (m->bc[2] == SW_BC_PERIODIC) != (m->bc[3] == SW_BC_PERIODIC))
    return fail(SW_EINVAL, "periodic boundaries must come in pairs");
  auto* c = new sw_ctx();
  c->s = (hipStream_t)stream;
  HIPCHK(hipGetDevice(&c->dev));
  c->p = *p;
  c->r = p->r;
  c->N1 = p->r + 1;
  c->NP = c->N1 * c->N1;
  c->K = m->n_cells;
  c->nx0 = m->nx0;
  c->ny0 = m->ny0;
  c->x0 = m->x0;
  c->y0 = m->y0;
  c->dx0 = m->dx0;
  tableau(p->rk, c->ns, c->A, c->b, c->c);
  const int K = c->K;
  c->lev.assign(m->level, m->level + K);
  c->ci.assign(m->i, m->i + K);
  c->cj.assign(m->j, m->j + K);
  int maxL = 0;
  for (int k = 0; k < K; ++k) {
    const int L = c->lev[k];
    if (L < 0 || L >= 8 || L >= p->n_levels) {
      delete c;
      return fail(SW_EINVAL, "cell level out of range (n_levels)");
    }
    if (k > 0 && L < c->lev[k - 1]) {
      delete c;
      return fail(SW_EINVAL, "cells must be sorted by level");
    }
    if (c->ci[k] < 0 || c->cj[k] < 0 || c->ci[k] >= (m->nx0 << L) || c->cj[k] >= (m->ny0 << L)) {
      delete c;
      return fail(SW_EINVAL, "cell outside the domain");
    }
    maxL = std::max(maxL, L);
  }
  // tiling check: sum of areas (in finest units) equals the domain
  {
    long double area = 0.0L;
    for (int k = 0; k < K; ++k) area += std::ldexp(1.0L, -2 * c->lev[k]);
    if (std::fabs((double)(area - (long double)m->nx0 * m->ny0)) > 1e-9) {
      delete c;
      return fail(SW_EINVAL, "cells do not tile the domain");
    }
  }
  std::unordered_map<int64_t, int> leaf;
  leaf.reserve(K * 2);
  for (int k = 0; k < K; ++k) {
    if (!leaf.emplace(key(c->lev[k], c->ci[k], c->cj[k]), k).second) {
      delete c;
      return fail(SW_EINVAL, "duplicate cell");
    }
  }
  // levels
  for (int L = 0; L <= maxL; ++L) {
    LevelH h;
    h.L = L;
    h.S = p->S[L];
    if (h.S < p->r + 2 || h.S > 32) {
      delete c;
      return fail(SW_EINVAL, "S must satisfy r+2 <= S <= 32 on every level");
    }
    h.P = lanes_for(h.S);
    h.dx = m->dx0 / std::ldexp(1.0, L);
    c->lv.push_back(h);
  }
  {
    int k = 0;
    int64_t off = 0;
    for (auto& L : c->lv) {
      L.cell0 = k;
      while (k < K && c->lev[k] == L.L) ++k;
      L.ncell = k - L.cell0;
      L.off = (size_t)off;
      off += (int64_t)L.ncell * L.S * L.S;
    }
    c->nvol = off;
  }
  // faces: conforming (recorded from the W/S cell), hanging (from the fine cell),
  // boundary; A is the fine or equal side
  struct FaceH { int a, b, sa, sb, sub, bnd, bc, lvl; };
  std::vector<FaceH> fh;
  const bool perx = m->bc[0] == SW_BC_PERIODIC, pery = m->bc[2] == SW_BC_PERIODIC;
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1}, opp[4] = {1, 0, 3, 2};
  for (int k = 0; k < K; ++k) {
    const int L = c->lev[k], i = c->ci[k], j = c->cj[k];
    const int nxL = m->nx0 << L, nyL = m->ny0 << L;
    for (int s = 0; s < 4; ++s) {
      int ni = i + di[s], nj = j + dj[s];
      bool outside = false;
      if (ni < 0 || ni >= nxL) {
        if (perx) ni = (ni + nxL) % nxL;
        else outside = true;
      }
      if (nj < 0 || nj >= nyL) {
        if (pery) nj = (nj + nyL) % nyL;
        else outside = true;
      }
      if (outside) {
        fh.push_back({k, -1, s, 0, -1, 1, m->bc[s], L});
        continue;
      }
      auto it = leaf.find(key(L, ni, nj));
      if (it != leaf.end()) {
        if (s == 1 || s == 3) fh.push_back({k, it->second, s, opp[s], -1, 0, 0, L});
        continue;
      }
      if (L > 0) {
        auto ic = leaf.find(key(L - 1, ni >> 1, nj >> 1));
        if (ic != leaf.end()) {
          const int sub = (s < 2) ? (j & 1) : (i & 1);
          fh.push_back({k, ic->second, s, opp[s], sub, 0, 0, L});
          continue;
        }
      }
      // finer neighbour: both children along this side must be leaves
      bool ok = true;
      for (int t = 0; t < 2; ++t) {
        int ki, kj;
        if (s < 2) {
          ki = 2 * ni + (s == 0 ? 1 : 0);
          kj = 2 * nj + t;
        } else {
          ki = 2 * ni + t;
          kj = 2 * nj + (s == 2 ? 1 : 0);
        }
        if (leaf.find(key(L + 1, ki, kj)) == leaf.end()) ok = false;
      }
      if (!ok) {
        delete c;
        return fail(SW_EINVAL, "mesh is not 2:1 balanced at cell " + std::to_string(k));
      }
    }
  }
  // class of a face: x or y direction times (conforming/boundary, sub-face 0, sub-face 1)
  auto cls = [](const FaceH& h) { return (h.sa < 2 ? 0 : 3) + (h.sub + 1); };
  std::stable_sort(fh.begin(), fh.end(), [&](const FaceH& x, const FaceH& y) {
    return x.lvl != y.lvl ? x.lvl < y.lvl : cls(x) < cls(y);
  });
  c->F = (int)fh.size();
  std::vector<int> fA(c->F), fB(c->F), meta(c->F), used((size_t)K * 8, 0);
  for (int f = 0; f < c->F; ++f) {
    const FaceH& h = fh[f];
    fA[f] = h.a;
    fB[f] = h.b;
    meta[f] = h.sa | (h.sb << 2) | ((h.sub + 1) << 4) | (h.bnd << 6) | (h.bc << 8);
    // every cell side carries one face, or two sub-faces on a coarse side
    if (used[(size_t)h.a * 8 + h.sa * 2]++) {
      delete c;
      return fail(SW_EINVAL, "two faces on one cell side");
    }
    if (!h.bnd && used[(size_t)h.b * 8 + h.sb * 2 + (h.sub < 0 ? 0 : h.sub)]++) {
      delete c;
      return fail(SW_EINVAL, "two faces on one cell side");
    }
  }
  {
    int f = 0;
    size_t zo = 0;
    int fblk = 0;
    for (auto& L : c->lv) {
      L.face0 = f;
      const int cpb = kWave / L.P;
      for (int k = 0; k < 6; ++k) {
        L.cface0[k] = f;
        while (f < c->F && fh[f].lvl == L.L && cls(fh[f]) == k) ++f;
        L.cnface[k] = f - L.cface0[k];
        L.cfnblk[k] = (L.cnface[k] + kWave / kFaceLanes - 1) / (kWave / kFaceLanes);
        L.cfblk0[k] = fblk;
        fblk += L.cfnblk[k];
      }
      L.nface = f - L.face0;
      L.zfoff = zo;
      zo += (size_t)L.nface * 2 * L.S;
      L.nblk = (L.ncell + cpb - 1) / cpb;
    }
    if (f != c->F) {
      delete c;
      return fail(SW_EINVAL, "internal: face classes do not cover the face list");
    }
    c->fblk_total = fblk;
    sw_status st = SW_OK;
    const size_t KN = (size_t)K * c->NP;
#define ALLOC(ptr, n)                \
  if ((st = c->alloc(&ptr, n)) != SW_OK) { \
    delete c;                        \
    return st;                       \
  }
    ALLOC(c->d_fA, c->F);
    ALLOC(c->d_fB, c->F);
    ALLOC(c->d_meta, c->F);
    ALLOC(c->d_err, 1);
    ALLOC(c->d_zb, (size_t)c->nvol);
    ALLOC(c->d_braw, (size_t)c->nvol);
    ALLOC(c->d_db, K);
    ALLOC(c->d_bvec, KN);
    ALLOC(c->d_zmax, K);
    ALLOC(c->d_nman, K);
    ALLOC(c->d_cdx, K);
    ALLOC(c->d_cw1, K);
    ALLOC(c->d_zf, zo);
    for (int q = 0; q < 4; ++q) {
      ALLOC(c->d_sn[q], KN);
      ALLOC(c->d_ss[q], KN);
    }
    ALLOC(c->d_hn, KN);
    ALLOC(c->d_cn, KN);
    ALLOC(c->d_res, (size_t)kNSlot * 4 * KN);
    ALLOC(c->d_scal, 8);
    ALLOC(c->d_cdiag, (size_t)K * D_NSLOT);
    ALLOC(c->d_bpart, (size_t)std::max(c->fblk_total, 1));
    ALLOC(c->d_red, (size_t)std::max((c->fblk_total + 1023) / 1024, (K + 255) / 256) * D_NSLOT);
    ALLOC(c->d_need, K);
    ALLOC(c->d_diag, 16);
    ALLOC(c->d_flag, K);
    ALLOC(c->d_allwet, K);
#undef ALLOC
  }
  for (auto& L : c->lv) {
    sw_status st = build_tables(c, L);
    if (st != SW_OK) {
      delete c;
      return st;
    }
  }
  std::vector<double> cdx(K), cw1(K);
  for (int k = 0; k < K; ++k) {
    const LevelH& L = c->lv[c->lev[k]];
    cdx[k] = L.dx;
    cw1[k] = p->cfl_mode == 1 ? L.w1 : 1.0;
  }
  HIPCHK(hipMemcpy(c->d_fA, fA.data(), sizeof(int) * c->F, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->d_fB, fB.data(), sizeof(int) * c->F, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->d_meta, meta.data(), sizeof(int) * c->F, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->d_cdx, cdx.data(), sizeof(double) * K, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->d_cw1, cw1.data(), sizeof(double) * K, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(c->d_err, 0, sizeof(int)));
  HIPCHK(hipMemset(c->d_db, 0, sizeof(double) * K));
  HIPCHK(hipMemset(c->d_nman, 0, sizeof(double) * K));
  HIPCHK(hipMemset(c->d_scal, 0, sizeof(double) * 8));
  HIPCHK(hipMemset(c->d_diag, 0, sizeof(double) * 16));
  HIPCHK(hipMemset(c->d_cdiag, 0, sizeof(double) * (size_t)K * D_NSLOT));
  HIPCHK(hipMemset(c->d_need, 0, K));
  HIPCHK(hipMemset(c->d_res, 0, sizeof(double) * (size_t)kNSlot * 4 * K * c->NP));
  HIPCHK(hipMemset(c->d_flag, c->r, K));
  HIPCHK(hipMemset(c->d_allwet, 0, K));
  for (int q = 0; q < 4; ++q) {
    HIPCHK(hipMemset(c->d_sn[q], 0, sizeof(double) * K * c->NP));
    HIPCHK(hipMemset(c->d_ss[q], 0, sizeof(double) * K * c->NP));
  }
  HIPCHK(hipMemset(c->d_hn, 0, sizeof(double) * K * c->NP));
  HIPCHK(hipMemset(c->d_cn, 0, sizeof(double) * K * c->NP));
  HIPCHK(hipDeviceSynchronize());
  *out = c;
  return SW_OK;
}

void sw_destroy(sw_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->s);
  delete c;
}

sw_status sw_counts(const sw_ctx* c, int64_t* n_cells, int64_t* n_vol, int64_t* n_dofs) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (n_cells) *n_cells = c->K;
  if (n_vol) *n_vol = c->nvol;
  if (n_dofs) *n_dofs = (int64_t)c->K * c->NP;
  return SW_OK;
}

sw_status sw_node_coords(const sw_ctx* c, double* xy) {
  if (!c || !xy) return fail(SW_EINVAL, "NULL argument");
  for (const auto& L : c->lv) {
    for (int cl = 0; cl < L.ncell; ++cl) {
      const int k = L.cell0 + cl;
      double* o = xy + 2 * (L.off + (size_t)cl * L.S * L.S);
      for (int b = 0; b < L.S; ++b)
        for (int a = 0; a < L.S; ++a) {
          o[2 * (b * L.S + a) + 0] = c->x0 + (c->ci[k] + L.xh[a]) * L.dx;
          o[2 * (b * L.S + a) + 1] = c->y0 + (c->cj[k] + L.xh[b]) * L.dx;
        }
    }
  }
  return SW_OK;
}

sw_status sw_dof_coords(const sw_ctx* c, double* xy) {
  if (!c || !xy) return fail(SW_EINVAL, "NULL argument");
  std::vector<double> xi, wb;
  gll(c->N1, xi, wb);
  for (int k = 0; k < c->K; ++k) {
    const double dx = c->lv[c->lev[k]].dx;
    for (int jy = 0; jy < c->N1; ++jy)
      for (int jx = 0; jx < c->N1; ++jx) {
        const size_t q = (size_t)k * c->NP + jy * c->N1 + jx;
        xy[2 * q + 0] = c->x0 + (c->ci[k] + xi[jx]) * dx;
        xy[2 * q + 1] = c->y0 + (c->cj[k] + xi[jy]) * dx;
      }
  }
  return SW_OK;
}

sw_status sw_set_bathymetry(sw_ctx* c, const double* b) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = check_ptr(b, "b");
  if (st != SW_OK) return st;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((c->nvol + 255) / 256)), dim3(256), 0, c->s, b, c->d_braw,
                     (size_t)c->nvol);
  HIPCHK(hipGetLastError());
  c->bathy_set = true;
  return rebake(c);
}

sw_status sw_set_bed_offset(sw_ctx* c, const double* db) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = check_ptr(db, "db");
  if (st != SW_OK) return st;
  hipLaunchKernelGGL(k_copy, dim3((c->K + 255) / 256), dim3(256), 0, c->s, db, c->d_db, (size_t)c->K);
  HIPCHK(hipGetLastError());
  if (!c->bathy_set) return SW_OK;
  return rebake(c);
}

sw_status sw_set_manning(sw_ctx* c, const double* n) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = check_ptr(n, "n");
  if (st != SW_OK) return st;
  hipLaunchKernelGGL(k_copy, dim3((c->K + 255) / 256), dim3(256), 0, c->s, n, c->d_nman, (size_t)c->K);
  HIPCHK(hipGetLastError());
  c->start_ready = false;
  return SW_OK;
}

sw_status sw_set_state(sw_ctx* c, const double* eta, const double* qx, const double* qy, const double* tr) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!eta || !qx || !qy) return fail(SW_EINVAL, "eta, qx, qy must be non-NULL");
  const size_t n = (size_t)c->K * c->NP;
  const unsigned nb = (unsigned)((n + 255) / 256);
  const double* src[4] = {eta, qx, qy, tr};
  for (int q = 0; q < 4; ++q) {
    if (src[q]) hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, c->s, src[q], c->d_sn[q], n);
    else hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, c->s, c->d_sn[q], n, 0.0);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_fill8, dim3((c->K + 255) / 256), dim3(256), 0, c->s, c->d_flag, (size_t)c->K,
                     (int8_t)c->r);
  HIPCHK(hipGetLastError());
  c->stage_done = 0;
  c->start_ready = false;
  return SW_OK;
}

sw_status sw_get_state(const sw_ctx* c, double* eta, double* qx, double* qy, double* tr) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  const size_t n = (size_t)c->K * c->NP;
  const unsigned nb = (unsigned)((n + 255) / 256);
  double* dst[4] = {eta, qx, qy, tr};
  for (int q = 0; q < 4; ++q) {
    if (!dst[q]) continue;
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, c->s, c->d_sn[q], dst[q], n);
    HIPCHK(hipGetLastError());
  }
  return SW_OK;
}

sw_status sw_init_lake_at_rest(sw_ctx* c, const double* eta) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = check_ptr(eta, "eta");
  if (st != SW_OK) return st;
  if ((st = need_bathy(c)) != SW_OK) return st;
  for (auto& L : c->lv) {
    if (L.ncell == 0) continue;
    hipLaunchKernelGGL(k_lake, dim3((L.ncell + 127) / 128), dim3(128), 0, c->s, L.tabs, L.cell0, L.ncell, L.off,
                       c->N1, c->d_zb, c->d_zmax, eta, c->d_sn[0], c->d_sn[1], c->d_sn[2]);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_fill8, dim3((c->K + 255) / 256), dim3(256), 0, c->s, c->d_flag, (size_t)c->K,
                     (int8_t)c->r);
  HIPCHK(hipGetLastError());
  c->stage_done = 0;
  c->start_ready = false;
  return SW_OK;
}

sw_status sw_set_time(sw_ctx* c, double t) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, c->s, c->d_scal, 1, t);
  HIPCHK(hipGetLastError());
  return SW_OK;
}

sw_status sw_apply_operator(sw_ctx* c, const double* eta, const double* qx, const double* qy, const double* tr,
                            double t, double* F, double* Gx, double* Gy, double* R, double* dtb) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (!eta || !qx || !qy || !F || !Gx || !Gy) return fail(SW_EINVAL, "state and residual pointers must be non-NULL");
  if (c->p.tracer && (!tr || !R)) return fail(SW_EINVAL, "tracer and R are required with a tracer");
  sw_status st = need_bathy(c);
  if (st != SW_OK) return st;
  if (c->stage_done != 0) return fail(SW_EINVAL, "sw_apply_operator cannot run inside an open step");
  // the elevation boundary reads the time from scal[1]: evaluate at t with dt = 0
  hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, c->s, c->d_scal, 3, t);
  for (auto& L : c->lv) {
    StageArgs a = stage_args(c, L);
    a.in[0] = eta;
    a.in[1] = qx;
    a.in[2] = qy;
    a.in[3] = c->p.tracer ? tr : nullptr;
    a.slot = kApplySlot;
    HIPCHK(launch_stage(c->r, L.P, M_APPLY, a, L.nblk, c->s));
  }
  const double* st4[4] = {eta, qx, qy, c->p.tracer ? tr : eta};
  // the face kernel reads t from scal[1] = d_scal[3] (cstage = 0)
  if ((st = faces(c, st4, 0.0, kApplySlot, c->d_scal + 2)) != SW_OK) return st;
  for (auto& L : c->lv) {
    StageArgs a = stage_args(c, L);
    a.slot = kApplySlot;
    a.out[0] = F;
    a.out[1] = Gx;
    a.out[2] = Gy;
    a.out[3] = c->p.tracer ? R : nullptr;
    HIPCHK(launch_stage(c->r, L.P, M_FOLD, a, L.nblk, c->s));
  }
  if (dtb) {
    if (c->fblk_total > 0) {
      if ((st = reduce_dt(c, 1.0, dtb)) != SW_OK) return st;
    } else {
      hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, c->s, dtb, 0, 1e300);
    }
  }
  c->start_ready = false;   // the apply slot does not disturb the step's data, but stay safe
  return SW_OK;
}

sw_status sw_step_begin(sw_ctx* c, double dt) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  sw_status st = need_bathy(c);
  if (st != SW_OK) return st;
  if (c->stage_done != 0) return fail(SW_EINVAL, "a step is already open (call sw_rk_stage / sw_step_end)");
  c->fixed_dt = dt > 0.0;
  if (c->fixed_dt) hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, c->s, c->d_scal, 0, dt);
  // degree adaptation, H(zeta^n) and stage-1 volume terms (already in place after
  // a previous step's final kernel)
  if (!c->start_ready)
    if ((st = elements(c, F_START, M_START, -1, 0, 0, nullptr, 0, 0)) != SW_OK) return st;
  const double* stn[4] = {c->d_sn[0], c->d_sn[1], c->d_sn[2], c->d_sn[3]};
  if ((st = faces(c, stn, c->c[0], 0)) != SW_OK) return st;
  if (!c->fixed_dt)
    if ((st = reduce_dt(c, c->p.cfl, c->d_scal)) != SW_OK) return st;
  c->start_ready = false;
  c->stage_done = 1;
  return SW_OK;
}

sw_status sw_rk_stage(sw_ctx* c, int32_t l) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (l < 2 || l > c->ns) return fail(SW_EINVAL, "stage index out of range");
  if (c->stage_done != l - 1) return fail(SW_EINVAL, "stages must be taken in order after sw_step_begin");
  double coef[4];
  for (int m = 0; m < 4; ++m) coef[m] = m < l - 1 ? c->A[l - 1][m] : 0.0;
  sw_status st = elements(c, F_STAGE, M_STAGE, -1, l - 1, l - 1, coef, l == 2 ? 1 : 0, 1);
  if (st != SW_OK) return st;
  const double* sts[4] = {c->d_ss[0], c->d_ss[1], c->d_ss[2], c->d_ss[3]};
  if ((st = faces(c, sts, c->c[l - 1], l - 1)) != SW_OK) return st;
  c->stage_done = l;
  return SW_OK;
}

sw_status sw_step_end(sw_ctx* c) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  if (c->stage_done != c->ns) return fail(SW_EINVAL, "all stages must be taken before sw_step_end");
  // final combination; the same pass prepares the next step's start (slot 0)
  sw_status st = elements(c, F_FINAL, M_FINAL, M_START, 0, c->ns, c->b, c->ns == 1 ? 1 : 0, 2);
  if (st != SW_OK) return st;
  const int nb = (c->K + 255) / 256;
  hipLaunchKernelGGL(k_diag_part, dim3(nb), dim3(256), 0, c->s, c->d_cdiag, c->d_flag, c->K, c->d_red);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_diag, dim3(1), dim3(256), 0, c->s, c->d_red, nb, c->d_diag, c->d_scal);
  HIPCHK(hipGetLastError());
  c->stage_done = 0;
  c->start_ready = true;
  ++c->nstep;
  return SW_OK;
}

sw_status sw_step(sw_ctx* c, double dt) {
  sw_status st = sw_step_begin(c, dt);
  if (st != SW_OK) return st;
  for (int l = 2; l <= c->ns; ++l)
    if ((st = sw_rk_stage(c, l)) != SW_OK) return st;
  return sw_step_end(c);
}

sw_status sw_run(sw_ctx* c, int32_t n, double dt) {
  for (int i = 0; i < n; ++i) {
    sw_status st = sw_step(c, dt);
    if (st != SW_OK) return st;
  }
  return SW_OK;
}

sw_status sw_sync(sw_ctx* c) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  HIPCHK(hipStreamSynchronize(c->s));
  int err = 0;
  HIPCHK(hipMemcpy(&err, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (err) return fail(SW_EDEVICE, "a kernel reported an invalid index (code " + std::to_string(err) + ")");
  return SW_OK;
}

sw_status sw_profile(sw_ctx* c, int32_t on) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  c->prof = on != 0;
  return SW_OK;
}

sw_status sw_kernel_time(sw_ctx* c, int32_t kind, double* ms_total, int64_t* launches) {
  if (!c || !ms_total || !launches) return fail(SW_EINVAL, "NULL argument");
  if (kind < 0 || kind > 4) return fail(SW_EINVAL, "kind must be 0..4");
  for (auto& e : c->ev) {
    HIPCHK(hipEventSynchronize(e.b));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    c->prof_ms[e.kind] += ms;
    c->prof_n[e.kind] += e.nlaunch;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->ev.clear();
  *ms_total = c->prof_ms[kind];
  *launches = c->prof_n[kind];
  return SW_OK;
}

sw_status sw_kernel_time_reset(sw_ctx* c) {
  if (!c) return fail(SW_EINVAL, "NULL context");
  double ms;
  int64_t n;
  sw_status st = sw_kernel_time(c, 0, &ms, &n);
  if (st != SW_OK) return st;
  for (int k = 0; k < 8; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return SW_OK;
}

sw_status sw_diagnostics(const sw_ctx* c, sw_diag* out) {
  if (!c || !out) return fail(SW_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(c->s));
  double d[16], s[8];
  HIPCHK(hipMemcpy(d, c->d_diag, sizeof(d), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(s, c->d_scal, sizeof(s), hipMemcpyDeviceToHost));
  out->min_target_mass = d[0];
  out->n_pos_viol = (int64_t)d[1];
  out->max_newton_it = (int32_t)d[2];
  out->n_fallback = (int64_t)d[3];
  out->total_mass = d[4];
  out->n_r0_cells = (int64_t)d[5];
  out->nonfinite = d[6] != 0.0;
  out->dt = s[0];
  out->t = s[1];
  out->step = c->nstep;
  if (out->nonfinite) return fail(SW_ENONFINITE, "non-finite value in the state");
  return SW_OK;
}

}  // extern "C"
