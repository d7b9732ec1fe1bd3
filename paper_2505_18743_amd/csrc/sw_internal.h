// Internal declarations shared by the host side and the gfx950 kernels of the
// sub-grid DG shallow-water library (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swk {

constexpr int kWave = 64;
constexpr int kFaceLanes = 4;   // lanes per face of the face VJP kernel (default of the face kernel)

// ---- stage-kernel modes ---------------------------------------------------
enum Mode : int {
  M_APPLY = 0,  // volume residual of a given state
  M_FOLD = 1,   // residual slot + face contributions -> output arrays
  M_START = 2,  // degree adaptation, remap, H^n, C~^n, stage-1 volume residual
  M_STAGE = 3,  // stage-l solves from stored residuals + volume residual
  M_FINAL = 4,  // final combination + solves + mass diagnostics
};
// fast element kernel modes (see k_elem)
enum FastMode : int { F_START = 0, F_STAGE = 1, F_FINAL = 2 };

// per-level reference tables on the device
struct LevelTabs {
  const double* w;      // [S]          1-D rule weights on [0,1]
  const double* l;      // [S][N1]      l_k(xhat_a)
  const double* d;      // [S][N1]      l_k'(xhat_a)
  const double* m0inv;  // [NP][NP]     inverse all-wet rule mass matrix, unit square
  const double* mqinv;  // [NP][NP]     inverse exact mass matrix, unit square
  const double* mq;     // [NP][NP]     exact mass matrix, unit square
  const double* meanw;  // [NP]         int psi_j over the unit square
  const double* fl;     // [3][S][N1]   l_k at face nodes: s, s/2, (1+s)/2
  const double* wl;     // [S][N1]      w_a l_k(xhat_a)
  const double* wd;     // [S][N1]      w_a l_k'(xhat_a)
  int S;
};

// diagnostics partial slots per stage-kernel block
enum { D_MINT = 0, D_VIOL, D_NEWT, D_FALLB, D_MASS, D_NR0, D_NONF, D_NSLOT };

struct StageArgs {
  LevelTabs t;
  int cell0, ncell, K;
  const double* zb;      // level block of internal depth samples [ncell][S(a)][S(b)]
  // volume terms on a rule of their own (Table 1's Gauss-Legendre rule): its
  // tables and depth samples [ncell][nv(a)][nv(b)]; vol = 0: the sample rule
  int vol;
  LevelTabs tv;
  const double* zbv;
  const double* bvec;    // [K][NP] all-wet B_i = sum W psi_i zb
  const double* zmax;    // [K]     max depth sample
  const double* nman;    // [K]
  const double* cdx;     // [K]     cell size
  const int* cmem;       // [K]     member of the cell
  const double* mdt;     // [M]     time step of each member
  double* sn[4];         // persistent state (zeta, qx, qy, c) [K][NP]
  double* ss[4];         // stage state
  const double* in[4];   // M_APPLY / M_TRACER inputs
  double* out[4];        // M_FOLD outputs
  double* hn;            // [K][NP] H(zeta^n)
  double* cn;            // [K][NP] C~^n
  double* res;           // [NS][4][K][NP] residual slots (volume + face terms)
  int8_t* flag;          // [K] current degree (r or 0)
  int8_t* need;          // [K] cells left to the general kernel (fast kernel writes,
                         //     general kernel reads: only flagged cells are processed)
  int8_t* wflag;         // [nwave] per wavefront of the level (64/P cells): 1 if a cell is flagged
  int nwave;
  const int8_t* oflag;       // [K] degree flags of the step (the final kernel updates flag)
  // IMEX (friction with the implicit companion): implicit-part residuals L of
  // each stage [slot][2][K][NP]; the friction matrix Gam_ij = int gamma psi_i
  // psi_j at the state of the last volume pass [K][NP(NP+1)/2] (packed lower
  // triangle; written by every volume pass, read by the next stage's solve);
  // the implicit weights of the combination and its diagonal weight
  int imex;
  double* lres;
  double* gam;
  double at[4];
  double att;
  const double* replay[3];   // tracer replay: recorded zeta, qx, qy of this stage (else NULL)
  double* rec_end[3];        // final combination: copy of the new zeta, qx, qy before any
                             // degree change of the next step (else NULL)
  double* cdiag;         // [K][D_NSLOT] per-cell diagnostics of the current step
  int diag_init;         // 1: first solve of the step initialises cdiag
  int8_t* allwet;        // [K] zeta^n wet at every sample node
  int* err;
  int slot;              // residual slot written (volume terms) or copied (M_FOLD)
  int nterm;             // number of stored residuals combined
  double a[4];           // combination weights a_{l,m} or b_m
  double g, eps, hlim, eps0;
  double tnu;            // tracer numerical diffusion nu_K / |K| = C S / r^2 (eq:numdiff), 0: off
  double tkap;           // tracer decay rate kappa (source -kappa h c), 0: off
  int newton_max, tracer, fric, adapt;
  int xmap;              // 1: fast kernels give each XCD one contiguous range of cells
};

// One face launch covers a conflict-free group of faces (no two of them touch
// the same (cell, dof)) over several levels: segment s is a level's run of
// faces [sface0[s], sface0[s] + snface[s]) with that level's S, rule tables
// and face samples, handled by workgroups [sblk[s], sblk[s + 1]).
constexpr int kMaxSeg = 8;
struct FaceArgs {
  int K;
  int nseg;
  int sblk[kMaxSeg + 1];
  int sface0[kMaxSeg], snface[kMaxSeg], sS[kMaxSeg];
  const double* sfl[kMaxSeg];   // [3][S][N1] l_k at face nodes: s, s/2, (1+s)/2
  const double* sw[kMaxSeg];    // [S] rule weights
  const double* szf[kMaxSeg];   // [snface][2][S] face samples of the segment
  const int* fA;
  const int* fB;
  const int* meta;       // sideA | sideB<<2 | (sub+1)<<4 | boundary<<6 | bc<<8 (3 bits)
  const double* st[4];
  double* res;           // [NS][4][K][NP] residual slots
  int slot;              // slot receiving the face terms
  const double* cdx;     // [K]
  const double* cw1;     // [K]
  const int* cmem;       // [K] member of each cell
  const double* mt;      // [M] time of each member at the start of the step
  const double* mdt;     // [M] time step of each member (unused when cstage = 0)
  const double* mtide;   // [M][4] tide amplitude, period, phase, inflow tracer
  double cstage;         // c_l of the stage
  double* fdt;           // [F] positivity bound of each face
  const int* gof;        // [F] node offset of the face's given boundary data, -1: none
  const double* ghost;   // [4][ng] given zeta, qx, qy, c at those nodes
  int64_t ng;
  int* err;
  double g, eps;
  int tracer;
  int tonly;             // 1: the tracer's face terms only (a tracer replay: the flow is given)
  int xmap;              // 1: each XCD takes one contiguous range of the class's faces
};

// ---- adjoint (vector-Jacobian products) ----------------------------------
enum VjpMode : int {
  V_OP = 0,     // adjoint residual coefficients given
  V_STEP = 1,   // adjoint residual = dt M^-1 y, y combined from stage adjoints
};

struct VjpArgs {
  LevelTabs t;
  int cell0, ncell, K;
  const double* zb;      // level block of depth samples [ncell][S(a)][S(b)]
  const double* nman;    // [K]
  const double* cdx;     // [K]
  const double* u[3];    // state at which the residual is linearised [K][NP]
  const double* rin[3];  // V_OP: adjoint residual coefficients
  const double* yb[4][3];  // V_STEP: y = sum_{m < ny} yc[m] yb[m]
  double yc[4];
  int ny;
  double dt;             // V_STEP: R_bar = dt M^-1 y
  double* rbar[3];       // V_STEP: R_bar written for the face kernel
  double* ub[3];         // volume part of the state adjoint (written)
  double* nbar;          // [K] Manning adjoint (accumulated)
  double* dbbar;         // [K] bed-offset adjoint (accumulated)
  int* err;
  double g, eps, hlim;
  int check;             // 0: none, 1: every node wet, 2: also min depth >= hlim
};

struct VjpFaceArgs {
  int face0, nface, K, S;
  const int* fA;
  const int* fB;
  const int* meta;
  const double* zf;      // group block [nface][2][S]
  const double* u[3];    // state (traces)
  const double* rb[3];   // adjoint residual coefficients
  double* ub[3];         // state adjoint: face rows added
  double* fdb;           // [F][2] bed-offset adjoint parts of each face (A side, B side)
  const double* cdx;     // [K]
  const int* cmem;       // [K]
  const double* fl;      // [3][S][N1]
  const double* w;       // [S]
  const double* mtide;   // [M][4]
  const int* gof;        // [F] as in FaceArgs
  const double* ghost;   // [4][ng]
  int64_t ng;
  double tt;             // time of the stage (elevation boundary)
  int* err;
  double g, eps;
};

hipError_t launch_vjp_vol(int r, int P, int mode, const VjpArgs& a, int nblk, hipStream_t s);
hipError_t launch_vjp_face(int r, const VjpFaceArgs& a, int nblk, hipStream_t s);

// ---- dynamic h-adaptivity ------------------------------------------------
struct AmrEtaArgs {
  const double* l;       // [n][N1] basis values at the volume rule's nodes
  const double* d;       // [n][N1] their derivatives
  int n, N1, cell0, ncell;
  const double* zb;      // level block of depth samples at those nodes [ncell][n(a)][n(b)]
  const double* cdx;     // [K]
  const double *z, *qx, *qy, *c;   // state [K][NP] (c may be NULL)
  double eps;
  int kind;              // 0: vorticity, 1: tracer gradient
  double* eta;           // [K] out
};
struct AmrXferArgs {
  int Kn, NP;
  const int* type;       // [Kn] 0: same cell, 1: child of an old cell, 2: parent of four old cells
  const int* src;        // [Kn][4] 0: old cell; 1: old parent, sub-cell 2 sy + sx; 2: old children by sub-cell
  const double* tchild;  // [4][NP][NP] parent basis at each child's support points
  const double* tproj;   // [4][NP][NP] exact-mass L2 projection, part of each child
  const double* in[4];   // old state fields [K_old][NP]
  double* out[4];        // new state fields [Kn][NP]
  const double *nman_in, *db_in;
  double *nman_out, *db_out;
};
struct RasterArgs {
  const double* g;       // raster [gny][gnx]
  int gnx, gny;
  double gx0, gy0, gdx, gdy;
  int cell0, ncell, n;   // level block and nodes per direction
  size_t off;            // offset of the block's nodes in braw
  const double* xh;      // [n] node positions on [0, 1]
  const int *ci, *cj;    // [K] integer cell positions
  const double* cdx;     // [K]
  const int* cmem;       // [K] member of each cell
  const double* mxy;     // [2][M] member origins (x0 of every member, then y0)
  int M;
  double* braw;          // bed elevation at the nodes (out)
};
struct AmrMassArgs {
  const double* l;       // [S][N1] basis values at the sample nodes
  const double* w;       // [S] rule weights
  int S, N1, cell0, ncell;
  const double* zb;      // level block [ncell][S(a)][S(b)]
  const double* cdx;
  const double* z;       // free surface [K][NP]
  double* out;           // [K][2]: int h, int z_b l
};
hipError_t launch_amr_eta(const AmrEtaArgs& a, hipStream_t s);
// linear reactions coupling tracers: R_k += sum_j B_kj int h c_j psi_i on the
// volume rule, for the stage state of every tracer context (the contexts
// share the flow, so the depth comes from the first one)
constexpr int kMaxReact = 8;
constexpr int kReactMaxRule = 32;   // volume-rule nodes per direction
struct ReactArgs {
  const double* l;       // [n][N1] basis values at the volume rule's nodes
  const double* w;       // [n] the rule's weights on [0, 1]
  int n, N1, cell0, ncell, M;
  const double* cdx;     // [K]
  const double* z;       // zeta of the stage state [K][NP]
  const double* zb;      // level block of depth samples [ncell][n(a)][n(b)]
  const double* c[kMaxReact];    // tracer context j: concentration of the stage state [K][NP]
  double* res[kMaxReact];        // tracer context k: the stage's residual R [K][NP] (added to)
  double B[kMaxReact * kMaxReact];   // B_kj at [k * M + j]
};
hipError_t launch_react(int r, const ReactArgs& a, hipStream_t s);
// the tracer contexts of one replayed stage, stepped by one launch: the
// first context's arrays are those of the StageArgs; all share the flow, the
// mesh and the degree flags
struct TrcSet {
  int M;
  double* res[kMaxReact];          // residual slots [NS][4][K][NP]
  double* cn[kMaxReact];           // C~^n [K][NP]; the final combination writes the next start's
  const double* c0[kMaxReact];     // c^n, the step start's tracer [K][NP]
  double* ss[kMaxReact][4];        // stage state
  double* cdiag[kMaxReact];        // per-cell diagnostics
  double tnu[kMaxReact], tkap[kMaxReact];   // diffusion (C S / r^2) and decay
};
hipError_t launch_trc_multi(int r, int P, int mode, const StageArgs& a, const TrcSet& ts, int nblk, hipStream_t s);
hipError_t launch_amr_transfer(const AmrXferArgs& a, hipStream_t s);
hipError_t launch_amr_raster(const RasterArgs& a, hipStream_t s);
hipError_t launch_amr_mass(const AmrMassArgs& a, hipStream_t s);
hipError_t launch_amr_sum2(const double* v, int K, double* out, hipStream_t s);

// launchers (return hipError_t of the launch)
hipError_t launch_stage(int r, int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_stage_scan(int r, int P, int mode, int mode2, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_elem(int r, int P, int mode, int wpb, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_trc(int r, int P, int mode, const StageArgs& a, int nblk, hipStream_t s);
hipError_t launch_face(int r, int q, const FaceArgs& a, int nblk, hipStream_t s);

// context hooks used by the ensemble driver
}  // namespace swk
struct sw_ctx;
namespace swk {
bool ctx_graph_ready(const sw_ctx* c);   // a step may be captured/replayed now
int64_t ctx_steps(const sw_ctx* c);
void ctx_set_steps(sw_ctx* c, int64_t n);
bool ctx_set_prof(sw_ctx* c, bool on);   // returns the previous setting
hipStream_t ctx_swap_stream(sw_ctx* c, hipStream_t s);   // returns the previous stream
hipStream_t ctx_stream(const sw_ctx* c);
int ctx_cells(const sw_ctx* c);
void ctx_class(const sw_ctx* c, int* r, int* S0);   // degree and level-0 sample count
int api_fail(int status, const char* msg);   // records msg for sw_last_error, returns status

inline int lanes_for(int S) {
  int P = 4;
  while (P < S) P <<= 1;
  return P;
}

}  // namespace swk
