// C-ABI of the semi-implicit BTE step: handle lifetime, operator upload, and the
// orchestration of the kernels of one step on the caller's stream.
#include "bte.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "assemble.h"
#include "hessenberg.h"
#include "internal.h"

static_assert(bte::kIonScratchDoubles == BTE_ION_SCRATCH_DOUBLES, "ion scratch size");

namespace {

using bte::DevOps;

struct HipError : std::runtime_error {
  hipError_t code;
  HipError(hipError_t c, const char* what) : std::runtime_error(what), code(c) {}
};

#define HIP_OK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) throw HipError(e_, #expr);   \
  } while (0)

}  // namespace

// Workspace of the fully implicit step (allocated at its first call).
struct ImplicitWs {
  int m = 0;                    // Krylov vectors per cycle the basis holds
  size_t N = 0;                 // unknowns (sum Nx * n)
  double *Fn = nullptr, *R = nullptr, *Rt = nullptr, *dlt = nullptr, *tmp = nullptr, *z = nullptr, *u = nullptr;
  double *V = nullptr;          // [m + 1][N]
  double *Pa = nullptr, *Pb = nullptr, *Pc = nullptr;   // padded rows
  double *El = nullptr, *zeros = nullptr;               // [sum Nx]
  double *partial = nullptr, *coef = nullptr;
  double* hcol = nullptr;       // [m + 1] the Hessenberg column of the current Arnoldi step
  std::vector<double> hpart, hcoef;
  double* Qx = nullptr;         // inverses of the x systems over the full step (layout of DevOps::Qt)
};

struct bte_handle {
  int device = 0;
  bte_config cfg{};
  bte::HostOps host;
  DevOps d;
  std::vector<int> nx_per, x_off;
  std::vector<double> n0_host, E0_host;   // per discharge
  std::vector<void*> allocs;
  hipStream_t last_stream = nullptr;
  int refine_max_iter = 10;
  double refine_rtol = 1e-14;
  double bytes = 0.0;
  int timing = 0;   // 1: phases and LU launch groups, 2: phases only
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // timing 2: the phase events of up to kWallRing steps, read (one wait) when
  // the ring is full or the sums are asked for, so that the timed steps run
  // back to back as untimed ones do
  static constexpr int kWallRing = 64;
  std::vector<hipEvent_t> wall_ev;   // 4 per step
  int wall_n = 0;                    // steps recorded and not yet read
  void wall_flush() {
    if (wall_n == 0) return;
    HIP_OK(hipEventSynchronize(wall_ev[4 * (wall_n - 1) + 3]));
    for (int i = 0; i < wall_n; ++i) {
      float a = 0, b = 0, c = 0;
      HIP_OK(hipEventElapsedTime(&a, wall_ev[4 * i], wall_ev[4 * i + 1]));
      HIP_OK(hipEventElapsedTime(&b, wall_ev[4 * i + 1], wall_ev[4 * i + 2]));
      HIP_OK(hipEventElapsedTime(&c, wall_ev[4 * i + 2], wall_ev[4 * i + 3]));
      ms_acc[2] += b;
      ms_acc[4] += a + c;
      ms_acc[5] += 1.0;
    }
    wall_n = 0;
  }
  // the factorization runs as lu_streams groups of points on side streams
  // (fork/join by events) so that one group's latency-bound panels overlap
  // another group's MFMA updates
  static constexpr int kMaxLuStreams = 4;
  int lu_streams = 1;
  hipStream_t gs[kMaxLuStreams] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kMaxLuStreams] = {};
  std::vector<hipEvent_t> lu_ev;   // kMaxLuStreams * 8 * max_panels
  std::vector<hipEvent_t> la_ev;   // 2 kMaxPanels: the factorization's look-ahead (side stream gs[0])
  int look_ahead = 0;              // BTE_TUNE_LOOK_AHEAD
  int form_overlap = 0;            // BTE_TUNE_FORM_OVERLAP
  hipEvent_t form_ev[2] = {nullptr, nullptr};
  bte::LuTimer lu_timer[kMaxLuStreams];
  double ms_acc[6] = {0, 0, 0, 0, 0, 0};
  // Krylov V solver (bte_set_vsolver): factors of the field-binned
  // preconditioner (a DevOps over nd * nbins matrices) and the GMRES workspace
  bool krylov = false;
  bool banded = false;         // V solves in the harmonic basis, banded LU
  bool hess = false;           // V solves in the harmonic basis, Hessenberg form
  int hess_n = 0, hess_ld = 0;
  double *d_hW = nullptr, *d_hQ = nullptr;   // [nd][n][hess_ld] each (rows zero beyond n)
  double* d_hH = nullptr;                     // [nd][n][hess_col_stride(n)], the solve's layout
  size_t* d_hoff = nullptr;                   // [nd] offsets of the H of discharge d
  std::vector<size_t> hoff_host;              // [nd] offsets d n hess_ld of its W and Q
  ImplicitWs iw;               // fully implicit step
  DevOps bd;                   // its factors (FP64) and harmonic operators
  double* d_TO = nullptr;
  double* d_TS = nullptr;
  int krylov_cycles = 2;
  int krylov_prec = 0;         // precision of the bin factors (0 FP64, 1 FP32)
  DevOps kf;
  bte::GmresOps kq;
  std::vector<void*> kallocs;
  void drop_krylov() {
    for (void* p : kallocs) (void)hipFree(p);
    kallocs.clear();
    krylov = false;
    banded = false;
    hess = false;
  }
  template <typename T>
  T* kalloc(size_t count) {
    void* p = nullptr;
    const size_t b = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) throw HipError(e, "hipMalloc");
    kallocs.push_back(p);
    e = hipMemset(p, 0, b);
    if (e != hipSuccess) throw HipError(e, "hipMemset");
    return static_cast<T*>(p);
  }
  // captured run of steps (bte_graph_capture / bte_graph_launch)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_steps = 0;
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
    graph_steps = 0;
  }
  double* d_coeff = nullptr;   // [nr] Maxwellian coefficients
  double* d_gE = nullptr;      // [nx_total] adjoint field-gradient scratch
  double* d_tmpF = nullptr;    // [nx_total*n]

  template <typename T>
  T* alloc(size_t count) {
    void* p = nullptr;
    const size_t bytes_req = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes_req);
    if (e != hipSuccess) throw HipError(e, "hipMalloc");
    allocs.push_back(p);
    bytes += static_cast<double>(bytes_req);
    return static_cast<T*>(p);
  }
  template <typename T>
  T* upload(const std::vector<T>& v) {
    T* p = alloc<T>(v.size());
    HIP_OK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  ~bte_handle() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : wall_ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : lu_ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : la_ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : form_ev)
      if (e) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (auto& e : join_ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& q : gs)
      if (q) (void)hipStreamDestroy(q);
    drop_graph();
    drop_krylov();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

bte_status map_exc(const std::exception& e) {
  if (auto* h = dynamic_cast<const HipError*>(&e)) return h->code == hipErrorOutOfMemory ? BTE_ENOMEM : BTE_EHIP;
  if (dynamic_cast<const std::bad_alloc*>(&e)) return BTE_ENOMEM;
  return BTE_EINVAL;
}

bte::AssemblyInput make_input(const bte_config* c) {
  if (!c) throw std::invalid_argument("null config");
  bte::AssemblyInput in;
  in.nr = c->nr;
  in.ntheta = c->ntheta;
  in.nl = c->nl;
  in.v_bc = c->v_bc;
  in.eps_max_eV = c->eps_max_eV;
  in.T0_K = c->T0_K;
  in.dt = c->dt_s;
  in.L = c->L_m;
  if (c->n_proc < 1 || !c->proc) throw std::invalid_argument("no processes");
  if (!(c->eps_max_eV > 0) || !(c->L_m > 0) || !(c->dt_s > 0) || c->T0_K < 0) throw std::invalid_argument("bad scalars");
  for (int s = 0; s < c->n_proc; ++s) {
    const bte_process& p = c->proc[s];
    if (p.n_tab < 2 || !p.eps_eV || !p.sigma_m2 || p.kind < 0 || p.kind > 2) throw std::invalid_argument("bad process");
    bte::Process q;
    q.kind = p.kind;
    q.threshold_eV = p.threshold_eV;
    q.mass_ratio = p.mass_ratio;
    q.eps_eV.assign(p.eps_eV, p.eps_eV + p.n_tab);
    q.sigma_m2.assign(p.sigma_m2, p.sigma_m2 + p.n_tab);
    for (int i = 1; i < p.n_tab; ++i)
      if (!(q.eps_eV[i] > q.eps_eV[i - 1])) throw std::invalid_argument("table energies must increase");
    if (p.kind == 0 && !(p.mass_ratio > 0 && p.mass_ratio < 0.5)) throw std::invalid_argument("bad mass ratio");
    in.proc.push_back(q);
  }
  const int nb = std::max(1, c->n_bins);
  if (c->bin_edges_eV) in.bin_edges_eV.assign(c->bin_edges_eV, c->bin_edges_eV + nb + 1);
  else {
    for (int b = 0; b <= nb; ++b) in.bin_edges_eV.push_back(c->eps_max_eV * b / nb);
  }
  in.scal.assign(static_cast<size_t>(c->n_proc) * nb, 1.0);
  if (c->scal) in.scal.assign(c->scal, c->scal + static_cast<size_t>(c->n_proc) * nb);
  const int nd = std::max(1, c->n_discharges);
  if (nd == 1) in.nx_per.push_back(c->nx_per ? c->nx_per[0] : c->nx);
  else {
    if (!c->nx_per) throw std::invalid_argument("nx_per required for ensembles");
    in.nx_per.assign(c->nx_per, c->nx_per + nd);
  }
  for (int nx : in.nx_per)
    if (nx < 3 || nx > 1024) throw std::invalid_argument("nx must be in [3, 1024]");
  if (!c->n0_per || !c->E0_per) throw std::invalid_argument("n0_per and E0_per required");
  if (c->precision < 0 || c->precision > 3) throw std::invalid_argument("bad precision");
  if (c->field_mode < 0 || c->field_mode > 3) throw std::invalid_argument("bad field mode");
  return in;
}

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

void fill_devops(bte_handle* h) {
  const bte_config& c = h->cfg;
  bte::HostOps& H = h->host;
  DevOps& d = h->d;
  const int nd = static_cast<int>(H.xops.size());
  d.nr = H.nr;
  d.nth = H.nth;
  d.n = H.n;
  d.nh = H.nth / 2;
  d.npad = ((H.n + bte::kNB - 1) / bte::kNB) * bte::kNB;
  d.nd = nd;
  d.n_params = H.n_params;
  d.n_bins = H.n_bins;
  d.precision = c.precision;
  // FP32 factors are refined to the FP64 backward error: static pivoting by default
  d.static_piv = c.precision != BTE_FP64 ? 1 : 0;
  d.dt = c.dt_s;
  h->x_off.assign(nd + 1, 0);
  h->nx_per.resize(nd);
  std::vector<size_t> qoff(nd), poff(nd);
  size_t qtot = 0, ptot = 0;
  int maxnx = 0;
  for (int i = 0; i < nd; ++i) {
    const int nx = H.xops[i].nx;
    h->nx_per[i] = nx;
    h->x_off[i + 1] = h->x_off[i] + nx;
    qoff[i] = qtot;
    poff[i] = ptot;
    qtot += H.xops[i].Qt.size();
    ptot += H.xops[i].poisson.size();
    maxnx = std::max(maxnx, nx);
  }
  d.nx_total = h->x_off[nd];
  d.max_nx = maxnx;
  if (d.npad > bte::kMaxRows) throw std::invalid_argument("Nr*Ntheta must be <= 2048");
  std::vector<int> x_disc(d.nx_total);
  std::vector<double> xhat(d.nx_total), n0x(d.nx_total);
  std::vector<double> n0(c.n0_per, c.n0_per + nd), E0(c.E0_per, c.E0_per + nd);
  h->n0_host = n0;
  h->E0_host = E0;
  for (int i = 0; i < nd; ++i)
    for (int j = 0; j < h->nx_per[i]; ++j) {
      const int x = h->x_off[i] + j;
      x_disc[x] = i;
      xhat[x] = H.xops[i].xhat[j];
      n0x[x] = n0[i];
    }
  d.x_off = h->upload(h->x_off);
  d.nx_of = h->upload(h->nx_per);
  d.q_off = h->upload(qoff);
  d.p_off = h->upload(poff);
  d.n0_of = h->upload(n0);
  d.E0_of = h->upload(E0);
  d.x_disc = h->upload(x_disc);
  d.xhat = h->upload(xhat);
  d.n0x = h->upload(n0x);
  d.U = h->upload(H.U);
  d.Uinv = h->upload(H.Uinv);
  d.Cord = h->upload(H.Cord);
  d.Aord = h->upload(H.Aord);
  {
    std::vector<double> T1((size_t)H.n * H.n), T2((size_t)H.n * H.n);
    for (int r = 0; r < H.n; ++r)
      for (int c = 0; c < H.n; ++c) {
        T1[(size_t)c * H.n + r] = H.Cord[(size_t)r * H.n + c];
        T2[(size_t)c * H.n + r] = H.Aord[(size_t)r * H.n + c];
      }
    d.CordT = h->upload(T1);
    d.AordT = h->upload(T2);
  }
  d.Csb = h->upload(H.Csb);
  d.mom = h->upload(H.mom);
  {
    std::vector<double> Q;
    Q.reserve(qtot);
    std::vector<double> P;
    P.reserve(ptot);
    for (auto& X : H.xops) {
      Q.insert(Q.end(), X.Qt.begin(), X.Qt.end());
      P.insert(P.end(), X.poisson.begin(), X.poisson.end());
    }
    d.Qt = h->upload(Q);
    d.poisson = h->upload(P);
    if (c.precision != BTE_FP64 && c.x_fp32) {
      std::vector<float> Q32(Q.begin(), Q.end());
      d.Qt32 = h->upload(Q32);
    }
  }
  const size_t nxt = d.nx_total;
  {
    // D_x per discharge, column-major (entry (r, c) at c nx + r): the forward
    // spatial operator of the fully implicit step and the heavies' update
    std::vector<double> DT;
    DT.reserve(ptot);
    for (auto& X : H.xops)
      for (int cc = 0; cc < X.nx; ++cc)
        for (int r = 0; r < X.nx; ++r) DT.push_back(X.Dx[(size_t)r * X.nx + cc]);
    d.dxT = h->upload(DT);
    d.lam = h->upload(H.lam);
    d.mu_th = h->upload(H.mu);
  }
  if (c.field_mode == BTE_FIELD_POISSON) {
    // the heavies' update of the hybrid step: D_x (d.dxT above) and D_x^2 per
    // discharge, column-major (entry (r, c) at c nx + r)
    std::vector<double> D2;
    D2.reserve(ptot);
    for (auto& X : H.xops) {
      const int nx = X.nx;
      for (int cc = 0; cc < nx; ++cc)
        for (int r = 0; r < nx; ++r) {
          double acc = 0.0;
          for (int k = 0; k < nx; ++k) acc += X.Dx[(size_t)r * nx + k] * X.Dx[(size_t)k * nx + cc];
          D2.push_back(acc);
        }
    }
    d.dx2 = h->upload(D2);
    d.ion_M = h->alloc<double>(ptot);
    d.ion_b = h->alloc<double>(nxt);
    d.ion_E = h->alloc<double>(nxt);
    d.ni1 = h->alloc<double>(nxt);
  }
  d.Y = h->alloc<double>(nxt * d.n);
  const size_t elt = (c.precision == BTE_FP64) ? sizeof(double) : sizeof(float);
  d.lu = h->alloc<char>(nxt * d.npad * d.npad * elt);
  d.xscr = h->alloc<char>(nxt * d.npad * bte::kNB * elt);
  d.linv = h->alloc<char>(nxt * bte::kLinvElems * elt);
  d.piv = h->alloc<int>(nxt * d.npad);
  d.perm = h->alloc<int>(nxt * bte::kMaxPanels * bte::kPermStride);
  d.mirror = h->alloc<int>(nxt);
  d.E = h->alloc<double>(nxt);
  d.field_rhs = h->alloc<double>(nxt);
  d.B = h->alloc<double>(nxt * d.npad);
  d.X = h->alloc<double>(nxt * d.npad);
  d.R = h->alloc<double>(nxt * d.npad);
  d.Fs = h->alloc<double>(nxt * d.n);
  d.mu = h->alloc<double>(nxt * d.n);
  {
    const size_t gx = (d.n + 63) / 64, gy = (nxt + 31) / 32;
    d.adj_part = h->alloc<double>(static_cast<size_t>(d.n_params) * gx * gy + nxt * gx);
  }
  d.rmax = h->alloc<unsigned long long>(nxt);
  d.bmax = h->alloc<unsigned long long>(nxt);
  d.xmax = h->alloc<unsigned long long>(nxt);
  {
    const int n = d.n;
    std::vector<double> rc(n, 0.0), ra(n, 0.0), cc(n, 0.0), ca(n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double c = std::fabs(H.Cord[(size_t)i * n + j]), a = std::fabs(H.Aord[(size_t)i * n + j]);
        rc[i] += c;
        ra[i] += a;
        cc[j] += c;
        ca[j] += a;
      }
    d.c_inf = *std::max_element(rc.begin(), rc.end());
    d.a_inf = *std::max_element(ra.begin(), ra.end());
    d.c_one = *std::max_element(cc.begin(), cc.end());
    d.a_one = *std::max_element(ca.begin(), ca.end());
  }
  d.status = h->alloc<int>(4);
  d.resid = h->alloc<double>(1);
  d.scratch3 = h->alloc<double>(3 * nxt);
  h->d_coeff = h->alloc<double>(d.nr);
  h->d_gE = h->alloc<double>(nxt);
  h->d_tmpF = h->alloc<double>(nxt * d.n);
  HIP_OK(hipMemset(d.status, 0, 4 * sizeof(int)));
  HIP_OK(hipMemset(d.resid, 0, sizeof(double)));
  HIP_OK(hipMemset(d.piv, 0, nxt * d.npad * sizeof(int)));
}

// X(dt/2) in place on F.
void x_half(bte_handle* h, double* F, bool transpose, hipStream_t s) {
  const bool fp32 = (h->cfg.precision != BTE_FP64) && h->cfg.x_fp32;
  if (!transpose) {
    bte::launch_x_to_modes(h->d, F, s);
    bte::launch_advect(h->d, fp32, false, s);
    bte::launch_modes_to_x(h->d, F, s);
  } else {
    bte::launch_x_to_modes_T(h->d, F, s);
    bte::launch_advect(h->d, fp32, true, s);
    bte::launch_modes_to_x_T(h->d, F, s);
  }
}

// Form and factor every point's matrix (field already in d.E), in lu_streams
// groups of consecutive points on the side streams, joined back into s.
void factor_all(bte_handle* h, hipStream_t s) {
  DevOps& d = h->d;
  const int prec = h->cfg.precision;
  const int G = std::max(1, std::min(h->lu_streams, d.nx_total));
  if (G == 1) {
    // the side stream of the first group is free: the look-ahead takes it
    bte::LuLookAhead la;
    la.side = h->gs[0];
    la.ev = h->la_ev.data();
    la.look_ahead = h->look_ahead;
    la.form_overlap = h->form_overlap;
    la.form_ev[0] = h->form_ev[0];
    la.form_ev[1] = h->form_ev[1];
    bte::launch_lu_factor(d, prec, s, h->timing == 1 ? &h->lu_timer[0] : nullptr, 0, -1, &la);
    return;
  }
  HIP_OK(hipEventRecord(h->fork_ev, s));
  for (int g = 0; g < G; ++g) {
    const int m0 = static_cast<int>((static_cast<long long>(g) * d.nx_total) / G);
    const int m1 = static_cast<int>((static_cast<long long>(g + 1) * d.nx_total) / G);
    HIP_OK(hipStreamWaitEvent(h->gs[g], h->fork_ev, 0));
    bte::launch_lu_factor(d, prec, h->gs[g], h->timing == 1 ? &h->lu_timer[g] : nullptr, m0, m1 - m0);
    HIP_OK(hipEventRecord(h->join_ev[g], h->gs[g]));
    HIP_OK(hipStreamWaitEvent(s, h->join_ev[g], 0));
  }
}

// V(dt) by the batched restarted GMRES with the field-binned preconditioner.
void v_solve_krylov(bte_handle* h, double* F, hipStream_t s) {
  DevOps& d = h->d;
  const bte::GmresOps& q = h->kq;
  const int nxt = d.nx_total;
  const size_t vs = static_cast<size_t>(nxt) * d.npad;
  bte::launch_pad_rows(d, F, d.B, s);
  bte::launch_bin_map(d, q, s);
  // initial guess x0 = H b
  bte::launch_lu_solve_mapped(h->kf, h->krylov_prec, false, q.mat_of, nullptr, nxt, d.B, d.X, false, false, s);
  for (int cyc = 0; cyc < h->krylov_cycles; ++cyc) {
    bte::launch_apply(d, 1, d.B, d.X, q.R, cyc == 0 ? nullptr : q.conv, s);   // R = B - M X
    bte::launch_gmres_init(d, q, cyc == 0, s);
    for (int j = 0; j < q.m; ++j) {
      bte::launch_lu_solve_mapped(h->kf, h->krylov_prec, false, q.mat_of, q.conv, nxt, q.V + j * vs, q.Z, false,
                                  false, s);                      // z = H v_j
      bte::launch_apply(d, 2, nullptr, q.Z, q.W, q.conv, s);     // w = M z
      bte::launch_gmres_arnoldi(d, q, j, s);
    }
    bte::launch_gmres_combine(d, q, s);                          // Z = V y
    bte::launch_lu_solve_mapped(h->kf, h->krylov_prec, false, q.mat_of, q.inact, nxt, q.Z, d.X, true, false, s);
  }
  bte::launch_gmres_status(d, q, s);
  bte::launch_unpad_rows(d, d.X, F, s);
}

// V(dt) in the harmonic basis: Fh = P_S F, (I - dt (n0 C_h + E A_h)) Fh* = Fh by
// the batched LU restricted to the band of the l-major ordering, F* = P_O Fh*.
void v_solve_banded(bte_handle* h, double* F, hipStream_t s) {
  DevOps& d = h->d;
  DevOps& b = h->bd;
  b.E = d.E;   // the field of this step
  const int nl = h->cfg.nl;
  bte::launch_to_harm(d, nl, b.npad, F, h->d_TS, d.B, s);
  bte::launch_lu_factor(b, 0, s, h->timing == 1 ? &h->lu_timer[0] : nullptr);
  bte::launch_lu_solve_mapped(b, 0, false, nullptr, nullptr, d.nx_total, d.B, d.X, false, false, s);
  bte::launch_from_harm(d, nl, b.npad, d.X, d.B, h->d_TO, F, s);
}

// V(dt) in the harmonic basis by the Hessenberg form of every discharge:
// Fh = P_S F, u = Q_d (I - dt E H_d)^-1 W_d Fh, back to ordinates.
void v_solve_hess(bte_handle* h, double* F, hipStream_t s) {
  DevOps& d = h->d;
  const int nl = h->cfg.nl, n = h->hess_n, ld = h->hess_ld;
  bte::launch_to_harm(d, nl, ld, F, h->d_TS, d.B, s);
  for (int q = 0; q < d.nd; ++q)
    bte::launch_mat_apply(h->d_hW + h->hoff_host[q], d.B, d.X, n, ld, h->x_off[q], h->nx_per[q], s);
  bte::launch_hess_solve(d, h->d_hH, h->d_hoff, n, ld, d.X, d.R, s);
  for (int q = 0; q < d.nd; ++q)
    bte::launch_mat_apply(h->d_hQ + h->hoff_host[q], d.R, d.X, n, ld, h->x_off[q], h->nx_per[q], s);
  bte::launch_from_harm(d, nl, ld, d.X, d.B, h->d_TO, F, s);
}

// V(dt) in place on F (field already in d.E).  transpose: solve with A^T.
// The forward step takes the Krylov solver when one is configured; the
// adjoint (transpose, and its forward recomputation) always factors.
void v_solve(bte_handle* h, double* F, bool transpose, hipStream_t s, bool allow_krylov = false) {
  DevOps& d = h->d;
  const int prec = h->cfg.precision;
  if (allow_krylov && h->krylov && !transpose) {
    v_solve_krylov(h, F, s);
    return;
  }
  if (allow_krylov && h->banded && !transpose) {
    v_solve_banded(h, F, s);
    return;
  }
  if (allow_krylov && h->hess && !transpose) {
    v_solve_hess(h, F, s);
    return;
  }
  bte::launch_pad_rows(d, F, d.B, s);
  factor_all(h, s);
  bte::launch_lu_solve(d, prec, transpose, d.B, d.X, false, false, s);
  if (prec != BTE_FP64) {
    bte::launch_reset_refine(d, s);
    for (int it = 1; it <= h->refine_max_iter; ++it) {
      bte::launch_residual(d, transpose, s);
      bte::launch_refine_check(d, transpose, h->refine_rtol, it - 1, false, s);
      bte::launch_lu_solve(d, prec, transpose, d.R, d.X, true, true, s);
    }
    bte::launch_residual(d, transpose, s);
    bte::launch_refine_check(d, transpose, h->refine_rtol, h->refine_max_iter, true, s);
  }
  bte::launch_unpad_rows(d, d.X, F, s);
}

// Solve with existing factors (no refactorization), used by the adjoint.
// refine = false: one solve with the stored (possibly FP32) factors, no
// refinement -- a fixed linear map, as a preconditioner needs, accurate to the
// factors' precision.
void v_solve_again(bte_handle* h, double* F, bool transpose, hipStream_t s, bool refine = true) {
  DevOps& d = h->d;
  const int prec = h->cfg.precision;
  bte::launch_pad_rows(d, F, d.B, s);
  bte::launch_lu_solve(d, prec, transpose, d.B, d.X, false, false, s);
  if (prec != BTE_FP64 && refine) {
    bte::launch_reset_refine(d, s);
    for (int it = 1; it <= h->refine_max_iter; ++it) {
      bte::launch_residual(d, transpose, s);
      bte::launch_refine_check(d, transpose, h->refine_rtol, it - 1, false, s);
      bte::launch_lu_solve(d, prec, transpose, d.R, d.X, true, true, s);
    }
    bte::launch_residual(d, transpose, s);
    bte::launch_refine_check(d, transpose, h->refine_rtol, h->refine_max_iter, true, s);
  }
  bte::launch_unpad_rows(d, d.X, F, s);
}

bool field_ok(const bte_handle* h, const bte_field& f) {
  if (h->cfg.field_mode == BTE_FIELD_GIVEN && !f.E_half) return false;
  if (h->cfg.field_mode == BTE_FIELD_POISSON && !f.ni) return false;
  return true;
}

void eval_field(bte_handle* h, const double* Fh, double t_s, const bte_field& f, hipStream_t s) {
  const bte_config& c = h->cfg;
  bte::launch_field(h->d, c.field_mode, t_s + 0.5 * c.dt_s, c.field_freq_hz, c.field_a1, c.poisson_V0, Fh, f.E_half,
                    f.ni, h->d.E, s);
}


// ---- fully implicit step (eq. bte_fully_implicit) ------------------------------
void implicit_alloc(bte_handle* h, int m, int precond) {
  ImplicitWs& w = h->iw;
  const DevOps& d = h->d;
  const size_t N = (size_t)d.nx_total * d.n, P = (size_t)d.nx_total * d.npad;
  if (w.N == 0) {
    w.N = N;
    w.Fn = h->alloc<double>(N);
    w.R = h->alloc<double>(N);
    w.Rt = h->alloc<double>(N);
    w.dlt = h->alloc<double>(N);
    w.tmp = h->alloc<double>(N);
    w.z = h->alloc<double>(N);
    w.u = h->alloc<double>(N);
    w.Pa = h->alloc<double>(P);
    w.Pb = h->alloc<double>(P);
    w.Pc = h->alloc<double>(P);
    HIP_OK(hipMemset(w.Pa, 0, P * sizeof(double)));
    HIP_OK(hipMemset(w.Pb, 0, P * sizeof(double)));
    HIP_OK(hipMemset(w.Pc, 0, P * sizeof(double)));
    w.El = h->alloc<double>(d.nx_total);
    w.zeros = h->alloc<double>(d.nx_total);
    HIP_OK(hipMemset(w.zeros, 0, d.nx_total * sizeof(double)));
  }
  if (precond == BTE_PRECOND_SPLIT && !w.Qx) {
    // the backward-Euler x solve over dt of the split preconditioner, per
    // discharge in the layout (and at the offsets) of the half-step inverses
    std::vector<double> Q, Qd;
    for (const auto& X : h->host.xops) {
      bte::advection_inverses(h->host, X, d.dt, &Qd);
      Q.insert(Q.end(), Qd.begin(), Qd.end());
    }
    w.Qx = h->upload(Q);
  }
  if (w.m < m) {
    w.m = m;
    w.V = h->alloc<double>((size_t)(m + 1) * N);
    w.partial = h->alloc<double>((size_t)bte::dot_blocks() * (m + 1));
    w.coef = h->alloc<double>((size_t)m + 1);
    w.hcol = h->alloc<double>((size_t)m + 1);
    w.hpart.assign((size_t)bte::dot_blocks() * (m + 1), 0.0);
    w.hcoef.assign((size_t)m + 1, 0.0);
  }
}

// out[v] = w . V_v (v < nvec), partial sums added in a fixed order
void imp_dots(bte_handle* h, const double* w, const double* V, int nvec, double* out, hipStream_t s) {
  ImplicitWs& iw = h->iw;
  const int nb = bte::dot_blocks();
  bte::launch_dots(w, V, nvec, iw.N, iw.N, iw.partial, s);
  HIP_OK(hipMemcpyAsync(iw.hpart.data(), iw.partial, sizeof(double) * nb * nvec, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  for (int v = 0; v < nvec; ++v) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += iw.hpart[(size_t)b * nvec + v];
    out[v] = t;
  }
}

double imp_norm(bte_handle* h, const double* x, hipStream_t s) {
  double v = 0.0;
  imp_dots(h, x, x, 1, &v, s);
  return std::sqrt(v);
}

// y = beta y + sum_v c[v] V_v
void imp_comb(bte_handle* h, double* y, double beta, const double* V, const double* c, int nvec, hipStream_t s) {
  ImplicitWs& iw = h->iw;
  for (int v = 0; v < nvec; ++v) iw.hcoef[v] = c[v];
  HIP_OK(hipMemcpyAsync(iw.coef, iw.hcoef.data(), sizeof(double) * nvec, hipMemcpyHostToDevice, s));
  bte::launch_comb(y, beta, V, iw.coef, nvec, iw.N, iw.N, s);
  HIP_OK(hipStreamSynchronize(s));
}

// E(F) at t1 (specified field, or the Poisson field of n_i - u^T F)
void imp_field(bte_handle* h, const double* F, double t1, const double* ni, double* E, hipStream_t s) {
  const bte_config& c = h->cfg;
  bte::launch_field(h->d, c.field_mode, t1, c.field_freq_hz, c.field_a1, c.poisson_V0, F, nullptr, ni, E, s);
}

// out = A_x X D_x^T
void imp_xop(bte_handle* h, const double* X, double* out, hipStream_t s) {
  bte::launch_x_to_modes(h->d, X, s);
  bte::launch_x_forward(h->d, s);
  bte::launch_modes_to_x(h->d, out, s);
}

// R = F - F^n + dt A_x F D_x^T - dt (n0 C + E(F) A) F, R = F at the inflow entries; d.E <- E(F)
void imp_residual(bte_handle* h, const double* F, const double* ni, double t1, double* R, hipStream_t s) {
  DevOps& d = h->d;
  ImplicitWs& iw = h->iw;
  imp_field(h, F, t1, ni, d.E, s);
  bte::launch_pad_rows(d, F, iw.Pa, s);
  bte::launch_apply_field(d, 2, nullptr, iw.Pa, iw.Pb, d.E, s);
  bte::launch_unpad_rows(d, iw.Pb, R, s);
  imp_xop(h, F, iw.tmp, s);
  bte::launch_axpby(R, iw.tmp, 1.0, d.dt, iw.N, s);
  bte::launch_axpby(R, iw.Fn, 1.0, -1.0, iw.N, s);
  bte::launch_wall_rows(d, R, F, s);
}

// out = J_F X (eq. 1dbte_jac_action in residual form), with d.E = E(F); without
// the field-coupling term (the Poisson field's E(X) . F) when !coupling: the
// Jacobian of the residual with the field frozen at E(F)
void imp_jac(bte_handle* h, const double* F, const double* X, double* out, bool coupling, hipStream_t s) {
  DevOps& d = h->d;
  ImplicitWs& iw = h->iw;
  const bte_config& c = h->cfg;
  bte::launch_pad_rows(d, X, iw.Pa, s);
  bte::launch_apply_field(d, 2, nullptr, iw.Pa, iw.Pb, d.E, s);
  if (coupling && c.field_mode == BTE_FIELD_POISSON) {
    // E_lin(X) = L (0 - u^T X): the derivative of the affine field map
    bte::launch_field(d, BTE_FIELD_POISSON, 0.0, c.field_freq_hz, c.field_a1, 0.0, X, nullptr, iw.zeros, iw.El, s);
    bte::launch_pad_rows(d, F, iw.Pc, s);
    bte::launch_apply_field(d, 3, iw.Pb, iw.Pc, iw.Pb, iw.El, s);
  }
  bte::launch_unpad_rows(d, iw.Pb, out, s);
  imp_xop(h, X, iw.tmp, s);
  bte::launch_axpby(out, iw.tmp, 1.0, d.dt, iw.N, s);
  bte::launch_wall_rows(d, out, X, s);
}

// z = S v with the field frozen (factors of d.E).  BTE_PRECOND_SPLIT:
// S = (I + dt A_x (.) D_x^T)^-1 (I - dt V)^-1, the V solve then the backward-Euler
// x solve over the whole step, so that S^-1 = J - dt^2 V X (X the x operator) and
// the stiff x modes, which the splitting leaves exact, do not enter the error.
// BTE_PRECOND_SEMI_IMPLICIT: the semi-implicit step X(dt/2) V(dt) X(dt/2), whose
// inverse differs from J by dt^2 X^2 / 4 + ..., large on the stiff x modes.
void imp_precond(bte_handle* h, const double* v, double* z, int kind, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(z, v, sizeof(double) * h->iw.N, hipMemcpyDeviceToDevice, s));
  if (kind == BTE_PRECOND_SEMI_IMPLICIT) {
    x_half(h, z, false, s);
    v_solve_again(h, z, false, s, false);
    x_half(h, z, false, s);
    return;
  }
  v_solve_again(h, z, false, s, false);
  bte::launch_x_to_modes(h->d, z, s);
  bte::launch_advect(h->d, false, false, s, h->iw.Qx);
  bte::launch_modes_to_x(h->d, z, s);
}

// Right-preconditioned restarted GMRES for J_F dlt = b (b in iw.Rt); classical
// Gram-Schmidt twice; returns the iterations.  An Arnoldi step runs on the device
// (both Gram-Schmidt passes, the norm and the normalization, with sums in a fixed
// order) and reads back only its Hessenberg column; the Givens rotations and the
// small triangular solve run on the host.
int imp_gmres(bte_handle* h, const double* F, double rtol, int m, int maxit, int pk, bool coupling, hipStream_t s) {
  ImplicitWs& iw = h->iw;
  const size_t N = iw.N;
  double* V = iw.V;
  bte::launch_comb(iw.dlt, 0.0, V, iw.coef, 0, N, N, s);   // dlt = 0
  HIP_OK(hipMemcpyAsync(V, iw.Rt, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  const double beta0 = imp_norm(h, iw.Rt, s);
  if (!(beta0 > 0.0)) return 0;
  int total = 0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hc(m + 1), y(m);
  while (total < maxit) {
    const double beta = imp_norm(h, V, s);
    if (!(beta > rtol * beta0)) break;
    bte::launch_axpby(V, V, 1.0 / beta, 0.0, N, s);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (size_t)j * N;
      double* w = V + (size_t)(j + 1) * N;
      imp_precond(h, vj, iw.z, pk, s);
      imp_jac(h, F, iw.z, w, coupling, s);
      for (int pass = 0; pass < 2; ++pass) {
        bte::launch_dots(w, V, j + 1, N, N, iw.partial, s);
        bte::launch_gs_reduce(iw.partial, j + 1, pass, iw.hcol, iw.coef, s);
        bte::launch_comb(w, 1.0, V, iw.coef, j + 1, N, N, s);
      }
      bte::launch_dots(w, w, 1, N, N, iw.partial, s);
      bte::launch_norm_reduce(iw.partial, iw.hcol + j + 1, s);
      bte::launch_scale_inv(w, iw.hcol + j + 1, N, s);
      HIP_OK(hipMemcpyAsync(hc.data(), iw.hcol, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      const double hn = hc[j + 1];
      // Givens rotations on column j
      for (int i = 0; i < j; ++i) {
        const double a = cs[i] * hc[i] + sn[i] * hc[i + 1];
        hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
        hc[i] = a;
      }
      const double r = std::hypot(hc[j], hn);
      cs[j] = (r > 0.0) ? hc[j] / r : 1.0;
      sn[j] = (r > 0.0) ? hn / r : 0.0;
      hc[j] = r;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hc[i];
      ++total;
      k = j + 1;
      if (std::fabs(g[j + 1]) <= rtol * beta0 || !(hn > 0.0) || total >= maxit) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int c = i + 1; c < k; ++c) t -= H[(size_t)i * m + c] * y[c];
      y[i] = t / H[(size_t)i * m + i];
    }
    imp_comb(h, iw.u, 0.0, V, y.data(), k, s);
    imp_precond(h, iw.u, iw.z, pk, s);
    bte::launch_axpby(iw.dlt, iw.z, 1.0, 1.0, N, s);
    // true residual of the accumulated correction into V_0
    imp_jac(h, F, iw.dlt, iw.u, coupling, s);
    HIP_OK(hipMemcpyAsync(V, iw.Rt, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    bte::launch_axpby(V, iw.u, 1.0, -1.0, N, s);
  }
  return total;
}

// Heavies' update (eq. fluid_step) with E^n = L (n_i^n - u^T F^n) at t_s.
void ion_update(bte_handle* h, const double* F, const double* ni_in, double* ni_out, double t_s, hipStream_t s) {
  const bte_config& c = h->cfg;
  bte::launch_field(h->d, BTE_FIELD_POISSON, t_s, c.field_freq_hz, c.field_a1, c.poisson_V0, F, nullptr, ni_in,
                    h->d.ion_E, s);
  bte::launch_ion_update(h->d, F, ni_in, ni_out, s);
}

}  // namespace

extern "C" {

const char* bte_status_string(bte_status s) {
  switch (s) {
    case BTE_OK: return "ok";
    case BTE_EINVAL: return "invalid argument";
    case BTE_EHIP: return "HIP runtime error";
    case BTE_ESINGULAR: return "zero pivot in a velocity-space factorization";
    case BTE_ENOCONV: return "iterative refinement did not converge";
    case BTE_ENOMEM: return "out of device memory";
    case BTE_ENONFINITE: return "non-finite value in the state";
    case BTE_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

bte_status bte_setup_operators(const bte_config* cfg, int hip_device, bte_handle** out) {
  if (!out) return BTE_EINVAL;
  *out = nullptr;
  bte_handle* h = nullptr;
  try {
    bte::AssemblyInput in = make_input(cfg);
    h = new bte_handle();
    h->cfg = *cfg;
    h->device = hip_device;
    h->refine_max_iter = cfg->refine_max_iter > 0 ? cfg->refine_max_iter : 10;
    h->refine_rtol = cfg->refine_rtol > 0 ? cfg->refine_rtol : 1e-14;
    HIP_OK(hipSetDevice(hip_device));
    bte::assemble(in, &h->host);
    fill_devops(h);
    if (cfg->field_mode == BTE_FIELD_POISSON) {   // this GPU's copy of the ion step's fixed scratch
      double* ws = nullptr;
      HIP_OK(bte::ion_scratch(&ws));
    }
    for (auto& e : h->ev) HIP_OK(hipEventCreate(&e));
    const int P = h->d.npad / bte::kNB;
    h->lu_ev.assign(static_cast<size_t>(bte_handle::kMaxLuStreams) * 8 * P, nullptr);
    for (auto& e : h->lu_ev) HIP_OK(hipEventCreate(&e));
    for (int g = 0; g < bte_handle::kMaxLuStreams; ++g) {
      h->lu_timer[g].max_panels = P;
      h->lu_timer[g].ev = h->lu_ev.data() + static_cast<size_t>(g) * 8 * P;
      HIP_OK(hipStreamCreateWithFlags(&h->gs[g], hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&h->join_ev[g], hipEventDisableTiming));
    }
    HIP_OK(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
    h->la_ev.assign(2 * bte::kMaxPanels, nullptr);
    for (auto& e : h->la_ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : h->form_ev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_OK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    // pointers inside cfg are not retained
    h->cfg.proc = nullptr;
    h->cfg.bin_edges_eV = nullptr;
    h->cfg.scal = nullptr;
    h->cfg.nx_per = nullptr;
    h->cfg.n0_per = nullptr;
    h->cfg.E0_per = nullptr;
    *out = h;
    return BTE_OK;
  } catch (const std::exception& e) {
    delete h;
    return map_exc(e);
  }
}

void bte_destroy(bte_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  delete h;
}

bte_status bte_get_info(bte_handle* h, bte_info* out) {
  if (!h || !out) return BTE_EINVAL;
  out->nx_total = h->d.nx_total;
  out->n = h->d.n;
  out->n_params = h->d.n_params;
  out->n_discharges = h->d.nd;
  out->vmax = h->host.vmax;
  out->bytes_device = h->bytes;
  out->lu_flops_per_step = (2.0 / 3.0) * std::pow(static_cast<double>(h->d.n), 3) * h->d.nx_total;
  double qb = 0.0;
  const double el = (h->cfg.precision != BTE_FP64 && h->cfg.x_fp32) ? 4.0 : 8.0;
  for (int nx : h->nx_per) qb += static_cast<double>(h->d.nr) * h->d.nh * nx * nx * el;
  out->q_bytes_per_half_step = qb;
  return BTE_OK;
}

bte_status bte_step(bte_handle* h, double* F, double t_s, bte_field field, void* stream) {
  if (!h || !F || !field_ok(h, field)) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    if (h->timing == 2) {
      hipEvent_t* we = h->wall_ev.data() + 4 * h->wall_n;
      HIP_OK(hipEventRecord(we[0], s));
      x_half(h, F, false, s);
      eval_field(h, F, t_s, field, s);
      HIP_OK(hipEventRecord(we[1], s));
      v_solve(h, F, false, s, true);
      HIP_OK(hipEventRecord(we[2], s));
      x_half(h, F, false, s);
      HIP_OK(hipEventRecord(we[3], s));
      if (++h->wall_n == bte_handle::kWallRing) h->wall_flush();
      HIP_OK(hipGetLastError());
      return BTE_OK;
    }
    if (h->timing) HIP_OK(hipEventRecord(h->ev[0], s));
    x_half(h, F, false, s);
    eval_field(h, F, t_s, field, s);
    if (h->timing) HIP_OK(hipEventRecord(h->ev[1], s));
    v_solve(h, F, false, s, true);
    if (h->timing) HIP_OK(hipEventRecord(h->ev[2], s));
    x_half(h, F, false, s);
    if (h->timing) {
      HIP_OK(hipEventRecord(h->ev[3], s));
      HIP_OK(hipEventSynchronize(h->ev[3]));
      float a = 0, b = 0, c = 0;
      HIP_OK(hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
      HIP_OK(hipEventElapsedTime(&b, h->ev[1], h->ev[2]));
      HIP_OK(hipEventElapsedTime(&c, h->ev[2], h->ev[3]));
      float upd = 0.f, pan = 0.f;
      int n_upd = 0;
      for (const auto& tm : h->lu_timer) {
        const int P = tm.max_panels;
        for (int p = 0; p < tm.used; ++p) {
          float t[4] = {0.f, 0.f, 0.f, 0.f};
          for (int slot = 0; slot < 4; ++slot)
            HIP_OK(hipEventElapsedTime(&t[slot], tm.ev[2 * P * slot + 2 * p], tm.ev[2 * P * slot + 2 * p + 1]));
          upd += t[0] + t[2];
          pan += t[1] + t[3];
        }
        if (tm.used > 0) n_upd += tm.launches;
      }
      for (auto& tm : h->lu_timer) {
        tm.used = 0;
        tm.launches = 0;
      }
      h->ms_acc[0] += upd;        // LU trailing-update launches (summed over streams)
      h->ms_acc[1] += pan;        // LU panel + U12 launches (summed over streams)
      h->ms_acc[2] += b;          // V step, wall
      h->ms_acc[3] += n_upd;      // trailing-update launches timed
      h->ms_acc[4] += a + c;      // X half-steps (+ field)
      h->ms_acc[5] += 1.0;
    }
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_graph_capture(bte_handle* h, double* F, double t0_s, int32_t n_steps, bte_field field) {
  if (!h || !F || n_steps < 1 || !field_ok(h, field) || h->timing) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    h->drop_graph();
    hipStream_t c = h->cap_stream;
    HIP_OK(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
    try {
      for (int k = 0; k < n_steps; ++k) {
        const double t = t0_s + k * h->cfg.dt_s;
        x_half(h, F, false, c);
        eval_field(h, F, t, field, c);
        v_solve(h, F, false, c, true);
        x_half(h, F, false, c);
      }
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(c, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIP_OK(hipStreamEndCapture(c, &h->graph));
    HIP_OK(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
    h->graph_steps = n_steps;
    return BTE_OK;
  } catch (const std::exception& e) {
    h->drop_graph();
    return map_exc(e);
  }
}

bte_status bte_graph_launch(bte_handle* h, void* stream) {
  if (!h || !h->graph_exec) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    HIP_OK(hipGraphLaunch(h->graph_exec, s));
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_xstep(bte_handle* h, double* F, void* stream) {
  if (!h || !F) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    h->last_stream = S(stream);
    x_half(h, F, false, S(stream));
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_xstep_T(bte_handle* h, double* F, void* stream) {
  if (!h || !F) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    h->last_stream = S(stream);
    x_half(h, F, true, S(stream));
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_implicit_step(bte_handle* h, double* F, const double* ni, double t_s, bte_implicit_opts opts,
                             bte_implicit_stats* stats, void* stream) {
  if (!h || !F) return BTE_EINVAL;
  const int fm = h->cfg.field_mode;
  if (fm == BTE_FIELD_GIVEN) return BTE_EUNSUPPORTED;
  if (fm == BTE_FIELD_POISSON && !ni) return BTE_EINVAL;
  const double nrtol = opts.newton_rtol > 0.0 ? opts.newton_rtol : 1e-12;
  const int max_newton = opts.max_newton > 0 ? opts.max_newton : 20;
  const double grtol = opts.gmres_rtol > 0.0 ? opts.gmres_rtol : 1e-6;
  const int m = opts.restart > 0 ? std::min(opts.restart, 200) : 30;
  const int max_gmres = opts.max_gmres > 0 ? opts.max_gmres : 200;
  const int pk = opts.precond;
  if (pk != BTE_PRECOND_SPLIT && pk != BTE_PRECOND_SEMI_IMPLICIT) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    implicit_alloc(h, m, pk);
    ImplicitWs& iw = h->iw;
    const size_t N = iw.N;
    const double t1 = t_s + h->cfg.dt_s;
    HIP_OK(hipMemcpyAsync(iw.Fn, F, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    imp_residual(h, F, ni, t1, iw.R, s);
    double rn = imp_norm(h, iw.R, s);
    const double r0 = rn;
    const double tol = nrtol * std::max(imp_norm(h, iw.Fn, s), 1e-300);
    int it = 0, gits = 0;
    bool ok = rn <= tol;
    // the V factors of the preconditioner: E(F) of the iterate with the Poisson
    // field; a specified field does not depend on F, so one factorization serves
    // every Newton step
    const bool refactor = fm == BTE_FIELD_POISSON;
    for (; it < max_newton && !ok; ++it) {
      if (it == 0 || refactor) factor_all(h, s);      // d.E = E(F) from the last residual
      HIP_OK(hipMemcpyAsync(iw.Rt, iw.R, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
      bte::launch_axpby(iw.Rt, iw.Rt, -1.0, 0.0, N, s);
      // the first step linearizes with the field frozen at E(F^n) (a Picard step;
      // the Newton step itself for a specified field), the later ones with the
      // field coupling of eq. 1dbte_jac_action
      gits += imp_gmres(h, F, grtol, m, max_gmres, pk, it > 0, s);
      // line search on ||R||: full step first, then halvings
      double alpha = 1.0;
      bool acc = false;
      for (int ls = 0; ls < 10 && !acc; ++ls) {
        HIP_OK(hipMemcpyAsync(iw.z, F, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        bte::launch_axpby(iw.z, iw.dlt, 1.0, alpha, N, s);
        imp_residual(h, iw.z, ni, t1, iw.Rt, s);
        const double rt = imp_norm(h, iw.Rt, s);
        if (rt <= (1.0 - 1e-4 * alpha) * rn) {
          HIP_OK(hipMemcpyAsync(F, iw.z, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
          HIP_OK(hipMemcpyAsync(iw.R, iw.Rt, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
          rn = rt;
          acc = true;
        } else {
          alpha *= 0.5;
        }
      }
      if (!acc) break;
      ok = rn <= tol;
    }
    HIP_OK(hipStreamSynchronize(s));
    if (stats) {
      stats->newton_iters = it;
      stats->gmres_iters = gits;
      stats->residual = rn;
      stats->residual0 = r0;
    }
    return ok ? BTE_OK : BTE_ENOCONV;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_ion_step(bte_handle* h, const double* F, const double* ni_in, double* ni_out, double t_s,
                        void* stream) {
  if (!h || !F || !ni_in || !ni_out) return BTE_EINVAL;
  if (h->cfg.field_mode != BTE_FIELD_POISSON) return BTE_EUNSUPPORTED;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    ion_update(h, F, ni_in, ni_out, t_s, s);
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_ion_step_noalloc(bte_handle* h, const double* F, const double* ni_in, double* ni_out, double t_s,
                                void* stream) {
  if (!h || !F || !ni_in || !ni_out) return BTE_EINVAL;
  if (h->cfg.field_mode != BTE_FIELD_POISSON) return BTE_EUNSUPPORTED;
  const size_t nxt = static_cast<size_t>(h->d.nx_total);
  size_t m = 0;
  for (int nx : h->nx_per) m += static_cast<size_t>(nx) * nx;
  if (m + 3 * nxt > bte::kIonScratchDoubles) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    double* ws = nullptr;
    HIP_OK(bte::ion_scratch(&ws));
    double* M = ws;            // [sum Nx_d^2] the formed systems
    double* b = M + m;         // [sum Nx] right-hand sides
    double* E = b + nxt;       // [sum Nx] E^n
    double* rhs = E + nxt;     // [sum Nx] Poisson right-hand side
    hipStream_t s = S(stream);
    h->last_stream = s;
    const bte_config& c = h->cfg;
    bte::launch_field(h->d, BTE_FIELD_POISSON, t_s, c.field_freq_hz, c.field_a1, c.poisson_V0, F, nullptr, ni_in, E,
                      s, rhs);
    bte::launch_ion_update_ws(h->d, F, ni_in, ni_out, M, b, E, s);
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_hybrid_step(bte_handle* h, double* F, double* ni, double t_s, void* stream) {
  if (!h || !F || !ni) return BTE_EINVAL;
  if (h->cfg.field_mode != BTE_FIELD_POISSON) return BTE_EUNSUPPORTED;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    ion_update(h, F, ni, h->d.ni1, t_s, s);
    bte_field f{nullptr, h->d.ni1};
    const bte_status st = bte_step(h, F, t_s, f, stream);
    if (st != BTE_OK) return st;
    HIP_OK(hipMemcpyAsync(ni, h->d.ni1, sizeof(double) * h->d.nx_total, hipMemcpyDeviceToDevice, s));
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_vstep(bte_handle* h, double* F, const double* E, void* stream) {
  if (!h || !F || !E) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    HIP_OK(hipMemcpyAsync(h->d.E, E, sizeof(double) * h->d.nx_total, hipMemcpyDeviceToDevice, s));
    v_solve(h, F, false, s, true);
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_field_eval(bte_handle* h, const double* F_half, double t_s, bte_field field, double* E_out,
                          void* stream) {
  if (!h || !E_out || !field_ok(h, field)) return BTE_EINVAL;
  if (h->cfg.field_mode == BTE_FIELD_POISSON && !F_half) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    eval_field(h, F_half, t_s, field, s);
    HIP_OK(hipMemcpyAsync(E_out, h->d.E, sizeof(double) * h->d.nx_total, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_moments(bte_handle* h, const double* F, double* out, void* stream) {
  if (!h || !F || !out) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    h->last_stream = S(stream);
    bte::launch_moments(h->d, F, out, S(stream));
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_moments_vjp(bte_handle* h, const double* F, const double* gbar, double* lam, void* stream) {
  if (!h || !F || !gbar || !lam) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    h->last_stream = S(stream);
    bte::launch_moments_vjp(h->d, F, gbar, lam, S(stream));
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_initial_maxwellian(bte_handle* h, const double* ne, double Te_eV, double* F, void* stream) {
  if (!h || !ne || !F || !(Te_eV > 0)) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    std::vector<double> c = bte::maxwellian_coeffs(h->host, Te_eV);
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(h->d_coeff, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice));
    bte::launch_maxwellian(h->d, ne, h->d_coeff, F, s);
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_adjoint_step(bte_handle* h, const double* F_n, double t_s, bte_field field, double* lam,
                            double* grad_scal, double* grad_E0, double* grad_E, void* stream) {
  if (!h || !F_n || !lam || !grad_scal || !field_ok(h, field)) return BTE_EINVAL;
  if (h->cfg.field_mode == BTE_FIELD_POISSON) return BTE_EUNSUPPORTED;
  try {
    HIP_OK(hipSetDevice(h->device));
    hipStream_t s = S(stream);
    h->last_stream = s;
    DevOps& d = h->d;
    const size_t nb = sizeof(double) * d.nx_total * d.n;
    // forward recompute: F* = A^-1 X F_n (factors stay in the workspace)
    HIP_OK(hipMemcpyAsync(d.Fs, F_n, nb, hipMemcpyDeviceToDevice, s));
    x_half(h, d.Fs, false, s);
    eval_field(h, d.Fs, t_s, field, s);
    v_solve(h, d.Fs, false, s);
    // mu = A^-T X^T lam
    HIP_OK(hipMemcpyAsync(d.mu, lam, nb, hipMemcpyDeviceToDevice, s));
    x_half(h, d.mu, true, s);
    v_solve_again(h, d.mu, true, s);
    // gradients
    bte::launch_adjoint_grads(d, grad_scal, h->d_gE, s);
    if (grad_E) HIP_OK(hipMemcpyAsync(grad_E, h->d_gE, sizeof(double) * d.nx_total, hipMemcpyDeviceToDevice, s));
    if (grad_E0 && h->cfg.field_mode != BTE_FIELD_GIVEN)
      bte::launch_field_dE0(d, h->cfg.field_mode, t_s + 0.5 * h->cfg.dt_s, h->cfg.field_freq_hz, h->cfg.field_a1,
                            h->d_gE, grad_E0, s);
    // lam^n = X^T mu
    HIP_OK(hipMemcpyAsync(lam, d.mu, nb, hipMemcpyDeviceToDevice, s));
    x_half(h, lam, true, s);
    HIP_OK(hipGetLastError());
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_get_status(bte_handle* h, int32_t* refine_iters, double* final_resid) {
  if (!h) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    HIP_OK(hipStreamSynchronize(h->last_stream));
    int st[4];
    double r = 0.0;
    HIP_OK(hipMemcpy(st, h->d.status, sizeof(st), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&r, h->d.resid, sizeof(double), hipMemcpyDeviceToHost));
    if (refine_iters) *refine_iters = st[2];
    if (final_resid) *final_resid = r;
    const int zero = 0;
    HIP_OK(hipMemcpy(h->d.status, &zero, sizeof(int), hipMemcpyHostToDevice));
    if (st[0] & bte::kStNonFinite) return BTE_ENONFINITE;
    if (st[0] & bte::kStSingular) return BTE_ESINGULAR;
    if (st[0] & bte::kStNoConv) return BTE_ENOCONV;
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

bte_status bte_set_refine(bte_handle* h, int32_t max_iter, double rtol) {
  if (!h || max_iter > 100 || !std::isfinite(rtol)) return BTE_EINVAL;
  h->refine_max_iter = max_iter > 0 ? max_iter : 10;
  h->refine_rtol = rtol > 0 ? rtol : 1e-14;
  return BTE_OK;
}

bte_status bte_set_timing(bte_handle* h, int32_t enable) {
  if (!h) return BTE_EINVAL;
  if (enable < 0 || enable > 2) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    h->wall_flush();   // pending records of an earlier walls-only run are dropped with the sums
    if (enable == 2 && h->wall_ev.empty()) {
      h->wall_ev.assign(4 * bte_handle::kWallRing, nullptr);
      for (auto& e : h->wall_ev) HIP_OK(hipEventCreate(&e));
    }
  } catch (const std::exception& e) {
    return map_exc(e);
  }
  h->timing = enable;
  std::fill(std::begin(h->ms_acc), std::end(h->ms_acc), 0.0);
  return BTE_OK;
}

bte_status bte_set_vsolver(bte_handle* h, int32_t kind, int32_t n_bins, double E_bound, double bin_scale,
                           int32_t restart, int32_t cycles, double rtol, int32_t factor_precision) {
  if (!h) return BTE_EINVAL;
  if (kind == BTE_VSOLVER_LU) {
    h->drop_krylov();
    return BTE_OK;
  }
  if (kind == BTE_VSOLVER_HESSENBERG) {
    // the transforms stage one point and the nl x ntheta transform in LDS
    if (h->cfg.ntheta > 64) return BTE_EUNSUPPORTED;
    try {
      HIP_OK(hipSetDevice(h->device));
      HIP_OK(hipDeviceSynchronize());
      h->drop_krylov();
      const DevOps& d = h->d;
      const bte::HostOps& H = h->host;
      const int n = H.nh, nd = d.nd;
      const int nthreads = static_cast<int>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
      // W and Q with rows of length ld (zero beyond n); H in the solve's layout:
      // column c holds row n-1-j at entry j, zero-padded
      const int ld = ((n + bte::kNB - 1) / bte::kNB) * bte::kNB;
      const size_t nw = (size_t)n * ld;
      const int ldh = bte::hess_col_stride(n);
      const size_t nh = (size_t)n * ldh;
      h->d_hW = h->kalloc<double>(nw * nd);
      h->d_hQ = h->kalloc<double>(nw * nd);
      h->d_hH = h->kalloc<double>(nh * nd);
      h->hoff_host.assign(nd, 0);
      std::vector<size_t> h_off(nd);
      std::vector<double> hr(nh), wq(nw, 0.0);
      for (int q = 0; q < nd; ++q) {
        bte::HessForm f;
        bte::hessenberg_setup(H, h->n0_host[q], h->cfg.dt_s, nthreads, &f);
        h->hoff_host[q] = nw * q;
        h_off[q] = nh * q;
        std::fill(hr.begin(), hr.end(), 0.0);
        for (int c = 0; c < n; ++c)
          for (int j = 0; j < n; ++j) hr[(size_t)c * ldh + j] = f.Hc[(size_t)c * n + (n - 1 - j)];
        for (int i = 0; i < n; ++i) std::copy(f.W.begin() + (size_t)i * n, f.W.begin() + (size_t)(i + 1) * n, wq.begin() + (size_t)i * ld);
        HIP_OK(hipMemcpy(h->d_hW + nw * q, wq.data(), nw * sizeof(double), hipMemcpyHostToDevice));
        for (int i = 0; i < n; ++i) std::copy(f.Q.begin() + (size_t)i * n, f.Q.begin() + (size_t)(i + 1) * n, wq.begin() + (size_t)i * ld);
        HIP_OK(hipMemcpy(h->d_hQ + nw * q, wq.data(), nw * sizeof(double), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(h->d_hH + nh * q, hr.data(), nh * sizeof(double), hipMemcpyHostToDevice));
      }
      h->d_hoff = h->kalloc<size_t>(nd);
      HIP_OK(hipMemcpy(h->d_hoff, h_off.data(), nd * sizeof(size_t), hipMemcpyHostToDevice));
      h->d_TO = h->kalloc<double>(H.TO.size());
      h->d_TS = h->kalloc<double>(H.TS.size());
      HIP_OK(hipMemcpy(h->d_TO, H.TO.data(), H.TO.size() * sizeof(double), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(h->d_TS, H.TS.data(), H.TS.size() * sizeof(double), hipMemcpyHostToDevice));
      h->hess_n = n;
      h->hess_ld = ld;
      h->hess = true;
      return BTE_OK;
    } catch (const std::exception& e) {
      h->drop_krylov();
      return map_exc(e);
    }
  }
  if (kind == BTE_VSOLVER_BANDED) {
    // the transforms stage one point and the nl x ntheta transform in LDS
    if (h->cfg.ntheta > 64) return BTE_EUNSUPPORTED;
    try {
      HIP_OK(hipSetDevice(h->device));
      HIP_OK(hipDeviceSynchronize());
      h->drop_krylov();
      const DevOps& d = h->d;
      const bte::HostOps& H = h->host;
      const int n = H.nh, nxt = d.nx_total;   // harmonic unknowns nr * nl
      const int np = ((n + bte::kNB - 1) / bte::kNB) * bte::kNB;
      DevOps b = d;
      b.n = n;
      b.npad = np;
      // operators by columns (the formation kernel reads columns contiguously)
      std::vector<double> T1((size_t)n * n), T2((size_t)n * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          T1[(size_t)j * n + i] = H.Ch[(size_t)i * n + j];
          T2[(size_t)j * n + i] = H.Ah[(size_t)i * n + j];
        }
      b.CordT = h->kalloc<double>((size_t)n * n);
      b.AordT = h->kalloc<double>((size_t)n * n);
      HIP_OK(hipMemcpy(b.CordT, T1.data(), T1.size() * sizeof(double), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(b.AordT, T2.data(), T2.size() * sizeof(double), hipMemcpyHostToDevice));
      h->d_TO = h->kalloc<double>(H.TO.size());
      h->d_TS = h->kalloc<double>(H.TS.size());
      HIP_OK(hipMemcpy(h->d_TO, H.TO.data(), H.TO.size() * sizeof(double), hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(h->d_TS, H.TS.data(), H.TS.size() * sizeof(double), hipMemcpyHostToDevice));
      b.lu = h->kalloc<char>((size_t)nxt * np * np * sizeof(double));
      b.xscr = h->kalloc<char>((size_t)nxt * np * bte::kNB * sizeof(double));
      b.linv = h->kalloc<char>((size_t)nxt * bte::kLinvElems * sizeof(double));
      b.piv = h->kalloc<int>((size_t)nxt * np);
      b.perm = h->kalloc<int>((size_t)nxt * bte::kMaxPanels * bte::kPermStride);
      b.precision = 0;
      b.update_kc = 0;
      b.form_xpb = 0;
      b.static_piv = 0;
      b.mirror = nullptr;
      b.band_kl = 2 * d.nr - 1;
      b.band_ku = 2 * d.nr - 1;
      h->bd = b;
      h->banded = true;
      return BTE_OK;
    } catch (const std::exception& e) {
      h->drop_krylov();
      return map_exc(e);
    }
  }
  if (kind != BTE_VSOLVER_GMRES || n_bins < 1 || n_bins > 4096 || restart < 1 || restart > 63 || cycles < 1 ||
      cycles > 100 || !(rtol > 0.0) || bin_scale < 0.0 ||
      (factor_precision != BTE_FP64 && factor_precision != BTE_MIXED_FP32 && factor_precision != BTE_FACTORS_FP16))
    return BTE_EINVAL;
  const bool fp16 = factor_precision == BTE_FACTORS_FP16;
  const int lu_prec = fp16 ? BTE_MIXED_FP32 : factor_precision;   // the factorization itself
  const bte_config& c = h->cfg;
  double bound = E_bound;
  if (!(bound > 0.0)) {
    if (c.field_mode != BTE_FIELD_CONST && c.field_mode != BTE_FIELD_RF) return BTE_EINVAL;
    bound = 0.0;
    for (double e0 : h->E0_host) bound = std::max(bound, std::fabs(e0) * (1.0 + std::fabs(c.field_a1)));
    if (!(bound > 0.0)) bound = 1.0;
  }
  try {
    HIP_OK(hipSetDevice(h->device));
    HIP_OK(hipDeviceSynchronize());
    h->drop_krylov();
    const DevOps& d = h->d;
    const int nd = d.nd, nb = n_bins, nmat = nd * nb;
    const size_t elt = (lu_prec == BTE_FP64) ? sizeof(double) : sizeof(float);
    // bin matrices: I - dt (n0_d C + s_p A), s_p the centre of bin p
    DevOps f = d;
    f.nx_total = nmat;
    // bins uniform in u = E, or in u = asinh(E / bin_scale); centres mapped back
    std::vector<double> Eb(nmat), n0b(nmat);
    const double ub = bin_scale > 0.0 ? std::asinh(bound / bin_scale) : bound;
    const double width = 2.0 * ub / nb;
    for (int di = 0; di < nd; ++di)
      for (int p = 0; p < nb; ++p) {
        const double uc = -ub + (p + 0.5) * width;
        Eb[di * nb + p] = bin_scale > 0.0 ? bin_scale * std::sinh(uc) : uc;
        n0b[di * nb + p] = h->n0_host[di];
      }
    f.E = h->kalloc<double>(nmat);
    f.n0x = h->kalloc<double>(nmat);
    HIP_OK(hipMemcpy(f.E, Eb.data(), nmat * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(f.n0x, n0b.data(), nmat * sizeof(double), hipMemcpyHostToDevice));
    f.lu = h->kalloc<char>(static_cast<size_t>(nmat) * d.npad * d.npad * elt);
    f.xscr = h->kalloc<char>(static_cast<size_t>(nmat) * d.npad * bte::kNB * elt);
    f.linv = h->kalloc<char>(static_cast<size_t>(nmat) * bte::kLinvElems * elt);
    f.piv = h->kalloc<int>(static_cast<size_t>(nmat) * d.npad);
    f.perm = h->kalloc<int>(static_cast<size_t>(nmat) * bte::kMaxPanels * bte::kPermStride);
    f.precision = lu_prec;
    f.update_kc = 0;
    f.form_xpb = 0;
    f.static_piv = 0;   // the bins keep partially pivoted factors
    f.mirror = nullptr;
    bte::launch_lu_factor(f, lu_prec, nullptr);
    HIP_OK(hipDeviceSynchronize());
    if (fp16) {  // keep the factors in FP16 only: half the bytes per preconditioner solve
      const size_t cnt = static_cast<size_t>(nmat) * d.npad * d.npad;
      void* h16 = h->kalloc<char>(cnt * 2);
      bte::launch_to_half(static_cast<const float*>(f.lu), h16, cnt, nullptr);
      HIP_OK(hipDeviceSynchronize());
      auto it = std::find(h->kallocs.begin(), h->kallocs.end(), f.lu);
      if (it != h->kallocs.end()) h->kallocs.erase(it);
      HIP_OK(hipFree(f.lu));
      f.lu = h16;
    }
    int st = 0;
    HIP_OK(hipMemcpy(&st, d.status, sizeof(int), hipMemcpyDeviceToHost));
    if (st & bte::kStSingular) {
      const int zero = 0;
      HIP_OK(hipMemcpy(d.status, &zero, sizeof(int), hipMemcpyHostToDevice));
      h->drop_krylov();
      return BTE_ESINGULAR;
    }
    bte::GmresOps q;
    q.m = restart;
    q.nbins = nb;
    q.S0 = -ub;
    q.width = width;
    q.scale = bin_scale;
    q.rtol = rtol;
    const size_t nxt = d.nx_total, np = d.npad;
    q.mat_of = h->kalloc<int>(nxt);
    q.V = h->kalloc<double>((restart + 1) * nxt * np);
    q.W = h->kalloc<double>(nxt * np);
    q.Z = h->kalloc<double>(nxt * np);
    q.R = h->kalloc<double>(nxt * np);
    q.H = h->kalloc<double>(nxt * restart * (restart + 1));
    q.cs = h->kalloc<double>(nxt * restart);
    q.sn = h->kalloc<double>(nxt * restart);
    q.g = h->kalloc<double>(nxt * (restart + 1));
    q.bnorm = h->kalloc<double>(nxt);
    q.conv = h->kalloc<int>(nxt);
    q.inact = h->kalloc<int>(nxt);
    q.kcount = h->kalloc<int>(nxt);
    q.ktot = h->kalloc<int>(nxt);
    q.rest = h->kalloc<double>(nxt);
    h->kf = f;
    h->kq = q;
    h->krylov_prec = fp16 ? bte::kFactorsFp16 : (factor_precision == BTE_FP64 ? 0 : 1);
    h->krylov_cycles = cycles;
    h->krylov = true;
    return BTE_OK;
  } catch (const std::exception& e) {
    h->drop_krylov();
    return map_exc(e);
  }
}

bte_status bte_set_tuning(bte_handle* h, int32_t key, int32_t value) {
  if (!h) return BTE_EINVAL;
  const bool fp64 = h->cfg.precision == BTE_FP64;
  switch (key) {
    case BTE_TUNE_LU_STREAMS:
      if (value < 1 || value > bte_handle::kMaxLuStreams) return BTE_EINVAL;
      h->lu_streams = value;
      return BTE_OK;
    case BTE_TUNE_UPDATE_KC:
      if (value != 0 && value != (fp64 ? 8 : 16) && value != (fp64 ? 16 : 32)) return BTE_EINVAL;
      h->d.update_kc = value;
      return BTE_OK;
    case BTE_TUNE_FORM_XPB:
      if (value < 0 || value > 64) return BTE_EINVAL;
      h->d.form_xpb = value;
      return BTE_OK;
    case BTE_TUNE_PANEL_PAIRS:
      if (value < 0 || value > 2) return BTE_EINVAL;
      h->d.lu_pairs = value;
      return BTE_OK;
    case BTE_TUNE_STATIC_PIVOTING:
      if (value != 0 && value != 1) return BTE_EINVAL;
      if (fp64 && value == 1) return BTE_EINVAL;
      h->d.static_piv = value;
      return BTE_OK;
    case BTE_TUNE_LOOK_AHEAD:
      if (value != 0 && value != 1) return BTE_EINVAL;
      h->look_ahead = value;
      return BTE_OK;
    case BTE_TUNE_FORM_OVERLAP:
      if (value != 0 && value != 1) return BTE_EINVAL;
      h->form_overlap = value;
      return BTE_OK;
    default:
      return BTE_EINVAL;
  }
}

bte_status bte_get_tuning(bte_handle* h, int32_t key, int32_t* value) {
  if (!h || !value) return BTE_EINVAL;
  const bool fp64 = h->cfg.precision == BTE_FP64;
  switch (key) {
    case BTE_TUNE_LU_STREAMS: *value = h->lu_streams; return BTE_OK;
    case BTE_TUNE_UPDATE_KC: {
      const bool bf16 = h->cfg.precision == BTE_MIXED_BF16 || h->cfg.precision == BTE_MIXED_BF16X3;
      *value = bf16 ? 32 : (h->d.update_kc ? h->d.update_kc : 16);
      return BTE_OK;
    }
    case BTE_TUNE_FORM_XPB: *value = h->d.form_xpb ? h->d.form_xpb : (fp64 ? 16 : 8); return BTE_OK;
    case BTE_TUNE_PANEL_PAIRS: *value = h->d.lu_pairs; return BTE_OK;
    case BTE_TUNE_STATIC_PIVOTING: *value = h->d.static_piv; return BTE_OK;
    case BTE_TUNE_LOOK_AHEAD: *value = h->look_ahead; return BTE_OK;
    case BTE_TUNE_FORM_OVERLAP: *value = h->form_overlap; return BTE_OK;
    default: return BTE_EINVAL;
  }
}

bte_status bte_get_timing(bte_handle* h, double* ms_out) {
  if (!h || !ms_out) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    h->wall_flush();
  } catch (const std::exception& e) {
    return map_exc(e);
  }
  for (int i = 0; i < 6; ++i) ms_out[i] = h->ms_acc[i];
  return BTE_OK;
}

bte_status bte_get_operator(bte_handle* h, int32_t which, double* host_out) {
  if (!h || !host_out) return BTE_EINVAL;
  const bte::HostOps& H = h->host;
  auto put = [&](const std::vector<double>& v) { std::memcpy(host_out, v.data(), v.size() * sizeof(double)); };
  switch (which) {
    case 0: put(H.Cord); break;
    case 1: put(H.Aord); break;
    case 2: put(H.M); break;
    case 3: put(H.G); break;
    case 4: put(H.lam); break;
    case 5: put(H.U); break;
    case 6: {
      size_t o = 0;
      for (auto& X : H.xops) {
        std::memcpy(host_out + o, X.xhat.data(), X.xhat.size() * sizeof(double));
        o += X.xhat.size();
      }
      break;
    }
    case 7: put(H.mom); break;
    case 8: put(H.Csb); break;
    case 10: put(H.Ch); break;
    case 11: put(H.Ah); break;
    case 12: put(H.TO); break;
    case 13: put(H.TS); break;
    case 9: {
      // expand Q of discharge 0 to [nr][ntheta][nx][nx] row-major Q_ia
      const bte::XOps& X = H.xops[0];
      const int nx = X.nx, nr = H.nr, nth = H.nth, nh = nth / 2;
      for (int i = 0; i < nr; ++i)
        for (int a = 0; a < nth; ++a) {
          double* Q = host_out + ((size_t)i * nth + a) * nx * nx;
          const bool pos = a >= nh;
          const int hh = pos ? a - nh : nh - 1 - a;
          const double* Qt = X.Qt.data() + ((size_t)i * nh + hh) * nx * nx;
          for (int r = 0; r < nx; ++r)
            for (int c = 0; c < nx; ++c) {
              // Q_pos[r][c] = Qt[c][r]; Q_neg = J Q_pos J
              const int rr = pos ? r : nx - 1 - r, cc = pos ? c : nx - 1 - c;
              Q[(size_t)r * nx + c] = Qt[(size_t)cc * nx + rr];
            }
        }
      break;
    }
    default: return BTE_EINVAL;
  }
  return BTE_OK;
}

bte_status bte_factor_export(bte_handle* h, const double* E, int32_t x, double* lu_host, int32_t* piv_host) {
  if (!h || !E || !lu_host || !piv_host || x < 0 || x >= h->d.nx_total) return BTE_EINVAL;
  try {
    HIP_OK(hipSetDevice(h->device));
    DevOps& d = h->d;
    HIP_OK(hipMemcpy(d.E, E, sizeof(double) * d.nx_total, hipMemcpyDeviceToDevice));
    bte::launch_lu_factor(d, h->cfg.precision, nullptr);
    HIP_OK(hipDeviceSynchronize());
    const size_t nn = (size_t)d.npad * d.npad;
    if (h->cfg.precision == BTE_FP64) {
      HIP_OK(hipMemcpy(lu_host, static_cast<double*>(d.lu) + x * nn, nn * sizeof(double), hipMemcpyDeviceToHost));
    } else {
      std::vector<float> tmp(nn);
      HIP_OK(hipMemcpy(tmp.data(), static_cast<float*>(d.lu) + x * nn, nn * sizeof(float), hipMemcpyDeviceToHost));
      for (size_t i = 0; i < nn; ++i) lu_host[i] = tmp[i];
    }
    HIP_OK(hipMemcpy(piv_host, d.piv + (size_t)x * d.npad, d.npad * sizeof(int32_t), hipMemcpyDeviceToHost));
    return BTE_OK;
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

// Host-only assembly (no device needed): the same operators as bte_get_operator
// for which = 0..8 (and 9 with nx of the first discharge), for verification.
bte_status bte_host_operator(const bte_config* cfg, int32_t which, double* host_out) {
  if (!host_out) return BTE_EINVAL;
  try {
    bte::AssemblyInput in = make_input(cfg);
    bte_handle tmp;
    bte::assemble(in, &tmp.host);
    if (which >= 14 && which <= 16) {
      bte::HessForm f;
      const int nthreads = static_cast<int>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
      bte::hessenberg_setup(tmp.host, cfg->n0_per[0], cfg->dt_s, nthreads, &f);
      const int n = f.n;
      if (which == 14) std::memcpy(host_out, f.W.data(), f.W.size() * sizeof(double));
      if (which == 15) std::memcpy(host_out, f.Q.data(), f.Q.size() * sizeof(double));
      if (which == 16)
        for (int r = 0; r < n; ++r)
          for (int c = 0; c < n; ++c) host_out[(size_t)r * n + c] = f.Hc[(size_t)c * n + r];
      return BTE_OK;
    }
    return bte_get_operator(&tmp, which, host_out);
  } catch (const std::exception& e) {
    return map_exc(e);
  }
}

}  // extern "C"
