/*
 * bte.h -- C-ABI of the MI355X (gfx950) semi-implicit 1D-space electron BTE step.
 *
 * The library advances the electron distribution f(x, v, theta) of the
 * 1D3V Boltzmann transport equation (eq. bte-1d of the paper, "The electron
 * Boltzmann transport equation" section) by the semi-implicit split step of
 * eq. (bte_semi_implicit), "Hybrid solver time integration" section:
 *
 *     X(dt/2) -> field E^{1/2} -> V(dt) -> X(dt/2)
 *
 * with Chebyshev collocation in x, a Galerkin cubic B-spline basis in speed
 * and Gauss-Legendre discrete ordinates in the polar angle (eqs. f_expansion,
 * proj_ops, A_x, bte_1d_discrete).  The velocity-space step solves, at every
 * collocation point x_i, the dense system of eq. (vspace_batched_system)
 *
 *     (I - dt (n0 C + E_i A)) F*_i = F_i        (n = Nr * Ntheta unknowns)
 *
 * by a batched LU factorization with partial pivoting on the GPU; the spatial
 * step applies the precomputed inverses Q_ij of the per-(eigen-speed,
 * ordinate) Chebyshev systems (Alg. bte_spatial_adv).
 *
 * State layout (all device arrays, FP64, owned by the caller):
 *   F[x][k][a]  x: collocation point (ascending xhat = -cos(pi i/(Nx-1))),
 *               k: B-spline in speed, a: ordinate (ascending cos theta_a);
 *               f(x_i, v, theta_a) = sum_k F[i][k][a] phi_k(v)  [m^-3 (m/s)^-3].
 *   With several discharges the per-discharge blocks are concatenated along x
 *   (total sum_d Nx_d rows).
 *
 * Conventions:
 *   - Every device buffer passed in is allocated and owned by the caller; the
 *     library only reads/writes it on the given stream.  The handle owns all
 *     operator and workspace memory from setup until bte_destroy.
 *   - Argument errors are returned synchronously.  Device-side failures
 *     (refinement not converged, non-finite values, zero pivot) are latched in
 *     a device status word; bte_get_status or the next synchronous query
 *     returns them.
 *   - A handle must not be used on two streams at the same time.
 *   - Units are SI, energies at this boundary are in eV.
 *   - ``stream`` is a hipStream_t (NULL = the null stream).
 */
#ifndef BTE_H
#define BTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BTE_OK = 0,
  BTE_EINVAL = -1,        /* invalid argument (sizes, null pointers, modes)            */
  BTE_EHIP = -2,          /* a HIP runtime call failed                                  */
  BTE_ESINGULAR = -3,     /* exactly zero pivot in a velocity-space factorization       */
  BTE_ENOCONV = -4,       /* mixed-precision refinement did not reach refine_rtol       */
  BTE_ENOMEM = -5,        /* device allocation failed                                   */
  BTE_ENONFINITE = -6,    /* NaN/Inf found in the state                                 */
  BTE_EUNSUPPORTED = -7   /* valid request that the library does not implement          */
} bte_status;

typedef enum {
  BTE_FP64 = 0,           /* FP64 LU (MFMA f64) and FP64 advection                       */
  BTE_MIXED_FP32 = 1,     /* FP32 LU + FP64 iterative refinement of the V-step residual  */
  BTE_MIXED_BF16 = 2,     /* as MIXED_FP32, LU trailing updates with bf16 operands
                           * (MFMA bf16, FP32 accumulation)                           */
  BTE_MIXED_BF16X3 = 3,   /* as MIXED_BF16 with operands split a = hi + lo in bf16 and
                           * the products hi*hi + hi*lo + lo*hi                       */
  BTE_FACTORS_FP16 = 4    /* bte_set_vsolver only: preconditioner factored in FP32 and
                           * stored in FP16                                           */
} bte_precision;

typedef enum { BTE_ELASTIC = 0, BTE_EXCITATION = 1, BTE_IONIZATION = 2 } bte_process_kind;

typedef enum {
  BTE_VBC_NATURAL = 0,    /* no condition at v = 0 or v = vmax (Nr clamped splines)             */
  BTE_VBC_ZERO_VMAX = 1   /* f(vmax) = 0: Nr+1 clamped splines, the one non-zero at vmax dropped */
} bte_vbc;

typedef enum {
  BTE_FIELD_CONST = 0,    /* E = E0_d everywhere                                                */
  BTE_FIELD_RF = 1,       /* E = E0_d sin(2 pi f (t + dt/2)) (1 + a1 xhat)                      */
  BTE_FIELD_GIVEN = 2,    /* E^{1/2} supplied by the caller (bte_field.E_half)                  */
  BTE_FIELD_POISSON = 3   /* eq. bte_semi_implicit_efield: Delta V = -(e/eps0)(n_i - n_e),     */
                          /* V(0) = V0 sin(2 pi f (t + dt/2)), V(L) = 0, E = -dV/dx              */
} bte_field_mode;

/* One electron-neutral collision process (Table of collisions; the hybrid
 * model's operator sum of the "Hybrid fluid-BTE solver" section).  The cross
 * section is a table interpolated linearly in energy.  Host arrays, copied. */
typedef struct {
  int32_t kind;             /* bte_process_kind                                      */
  double threshold_eV;      /* excitation / ionization threshold (ignored: elastic)  */
  double mass_ratio;        /* m_e / m0 (elastic energy loss, gas-temperature term)  */
  int32_t n_tab;            /* >= 2                                                  */
  const double* eps_eV;     /* [n_tab] ascending                                     */
  const double* sigma_m2;   /* [n_tab]                                               */
} bte_process;

typedef struct {
  int32_t nx, nr, ntheta, nl;   /* 1 <= nl <= ntheta harmonics; nx per discharge if n_discharges == 1 */
  int32_t v_bc;                 /* bte_vbc                                                      */
  double L_m;                   /* electrode gap                                                */
  double eps_max_eV;            /* speed domain [0, sqrt(2 e eps_max / m_e)]                    */
  double T0_K;                  /* gas temperature (eq. c_T0_mat_1d)                            */
  double dt_s;                  /* time step                                                    */
  int32_t n_proc;
  const bte_process* proc;      /* host [n_proc]                                                */
  int32_t n_bins;               /* energy bins of the cross-section scalings (>= 1)             */
  const double* bin_edges_eV;   /* host [n_bins+1] or NULL (= one bin [0, eps_max])             */
  const double* scal;           /* host [n_proc*n_bins] multiplicative scalings or NULL (= 1)   */
  int32_t precision;            /* bte_precision                                                */
  int32_t refine_max_iter;      /* mixed modes: max refinement sweeps (<= 0: 10)                */
  double refine_rtol;           /* mixed modes: stop when, at every point, the normwise backward
                                 * error max|r| / (||M|| max|x| + max|b|) <= rtol, with ||M|| <=
                                 * 1 + dt (n0 ||C_ord|| + |E| ||A_ord||) (<= 0: 1e-14)            */
  int32_t field_mode;           /* bte_field_mode                                               */
  double field_freq_hz;         /* RF / Poisson voltage frequency                               */
  double field_a1;              /* RF spatial profile coefficient                               */
  double poisson_V0;            /* Poisson mode: peak electrode voltage                         */
  int32_t n_discharges;         /* >= 1; >1 = uneven ensemble (batching form)                   */
  const int32_t* nx_per;        /* host [n_discharges] or NULL when n_discharges == 1           */
  const double* n0_per;         /* host [n_discharges] neutral densities [m^-3]                  */
  const double* E0_per;         /* host [n_discharges] field amplitudes [V/m] (CONST / RF)       */
  int32_t x_fp32;               /* 1: stream Q in FP32 (mixed modes only); 0: FP64 advection      */
} bte_config;

/* Per-call field data for the GIVEN and POISSON modes (device arrays, [sum Nx]). */
typedef struct {
  const double* E_half;         /* GIVEN: E^{1/2} at every collocation point */
  const double* ni;             /* POISSON: ion density                      */
} bte_field;

typedef struct bte_handle bte_handle;   /* opaque */

typedef struct {
  int32_t nx_total;             /* sum_d Nx_d                          */
  int32_t n;                    /* Nr * Ntheta                          */
  int32_t n_params;             /* n_proc * n_bins                      */
  int32_t n_discharges;
  double vmax;                  /* m/s                                  */
  double bytes_device;          /* device memory held by the handle     */
  double lu_flops_per_step;     /* (2/3) n^3 * nx_total                 */
  double q_bytes_per_half_step; /* HBM bytes of Q streamed per X(dt/2)  */
} bte_info;

/* Setup (synchronous).  Assembles every operator in FP64 on the host --
 * mass matrices, collision operator eq. (c_en_mat_1d) with the gas-temperature
 * term eq. (c_T0_mat_1d), acceleration eq. (adv_v_ws), projections
 * eq. (proj_ops), the eigen-decomposition of G_v and the inverses Q_ij of the
 * X systems (with zero-inflow rows, eq. hybrid_cnt_b_bdy) -- and uploads them to
 * device ``hip_device``.  On success *out owns the device memory.
 * Errors: BTE_EINVAL (bad sizes/modes), BTE_ENOMEM, BTE_EHIP. */
bte_status bte_setup_operators(const bte_config* cfg, int hip_device, bte_handle** out);

/* One semi-implicit step F^n -> F^{n+1} at time t_s (eq. bte_semi_implicit),
 * in place.  Asynchronous on ``stream``; no host synchronization.
 * Errors (synchronous): BTE_EINVAL.  Device errors are latched. */
bte_status bte_step(bte_handle* h, double* F, double t_s, bte_field field, void* stream);

/* Fully implicit electron step (eq. bte_fully_implicit): F^{n+1} solves
 *   F^{n+1} - F^n = dt [-A_x F^{n+1} D_x^T + P_O C P_S F^{n+1} + P_O A_v P_S (E(F^{n+1}) . F^{n+1})]
 * with E(F) = L (n_i - u^T F) at t_s + dt (POISSON mode; ni device [sum Nx])
 * or the specified field at t_s + dt (CONST, RF: the equation is then linear),
 * and F = 0 at the inflow entries of the walls (eq. hybrid_cnt_b_bdy).
 * Newton's method with a backtracking line search on ||R||_2; each Newton
 * system J_F dlt = -R (Jacobian action of eq. 1dbte_jac_action, matrix free;
 * the first step drops the Poisson field's coupling term E(dlt) . F, i.e. it
 * linearizes with the field frozen at E(F^n), which keeps a full first step
 * from overshooting) by restarted GMRES, right-preconditioned by an operator split of the same
 * equation, taken as a linear map with the field frozen at E(F): one solve with
 * the V factors of the handle's precision (without refinement) and backward-Euler
 * x solves, classical Gram-Schmidt twice.  opts.precond picks the split:
 *   BTE_PRECOND_SPLIT (0, default): the V solve over dt, then the x solve over dt
 *     (the inverses of I + dt lam_i cos(theta_a) D_x, formed on the host at the
 *     first call, sum Nx^2 Nr Ntheta / 2 doubles of device memory);
 *   BTE_PRECOND_SEMI_IMPLICIT (1): the semi-implicit step X(dt/2) V(dt) X(dt/2)
 *     (eq. bte_semi_implicit), the paper's preconditioner.
 * The V systems are factored once per call with a specified field and at every
 * Newton step with the Poisson field.  F (device [sum Nx][Nr][Ntheta]) is
 * replaced by F^{n+1}.  Synchronous on the stream (the host drives the
 * iterations).  Defaults for zero fields of opts: newton_rtol 1e-12 (relative
 * to ||F^n||_2), max_newton 20, gmres_rtol 1e-6, restart 30 (<= 200), max_gmres
 * 200 per Newton step.  stats (may be NULL) receives the counts and the final
 * and initial ||R||_2.  Errors: BTE_EINVAL (also an unknown precond),
 * BTE_EUNSUPPORTED (GIVEN field), BTE_ENOCONV (Newton did not reach
 * newton_rtol; F holds the last iterate). */
enum { BTE_PRECOND_SPLIT = 0, BTE_PRECOND_SEMI_IMPLICIT = 1 };
typedef struct {
  double newton_rtol;
  int32_t max_newton;
  double gmres_rtol;
  int32_t restart;
  int32_t max_gmres;
  int32_t precond;
} bte_implicit_opts;
typedef struct {
  int32_t newton_iters;
  int32_t gmres_iters;
  double residual;
  double residual0;
} bte_implicit_stats;
bte_status bte_implicit_step(bte_handle* h, double* F, const double* ni, double t_s, bte_implicit_opts opts,
                             bte_implicit_stats* stats, void* stream);

/* Heavies' update of the hybrid model (operator split of eq. glow_hybrid,
 * eq. fluid_step), POISSON field mode only:
 *   (n_i^{n+1} - n_i^n)/dt + D_x J_i(E^n, n_i^{n+1}) = (k_i^T F^n) n0 (u^T F^n),
 *   J_i = mu_i n_i E - D_i D_x n_i (eq. hybrid_cnt_a_flux),
 * with E^n = L (n_i^n - u^T F^n) at t_s (eq. hybrid_cnt_c with the voltage of
 * eq. voltage_bc at t_s) frozen, per discharge on its CGL points.  The walls take
 * the drift outflow condition of eq. fl_ion_bc with the outward normal,
 * J_i . n = n_i max(0, mu_i E . n) (no inflow), in place of the equation at the
 * wall nodes.  Ion coefficients from the table of modeling parameters:
 * n0 mu_i = 4.65e21 /(V m s), n0 D_i = 2.07e20 /(m s), n0 per discharge.
 * F is device [sum Nx][Nr][Ntheta] (read), ni_in / ni_out device [sum Nx]
 * (distinct).  Each discharge's Nx x Nx system is solved by Gaussian
 * elimination with partial pivoting on the device; a zero pivot latches
 * BTE_ESINGULAR, a non-finite one BTE_ENONFINITE in the status word.
 * Errors: BTE_EINVAL (null pointers), BTE_EUNSUPPORTED (other field modes). */
bte_status bte_ion_step(bte_handle* h, const double* F, const double* ni_in, double* ni_out, double t_s,
                        void* stream);
/* bte_ion_step for callers that cannot allocate device memory or call the
 * allocator (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, same kernels and the same result bit for
 * bit, but its scratch -- the formed ion systems (sum_d Nx_d^2 doubles), their
 * right-hand sides, E^n and the Poisson right-hand side (sum_d Nx_d doubles
 * each) -- lives in a fixed device array of the library of
 * BTE_ION_SCRATCH_DOUBLES doubles (16 MiB), one copy on every GPU the library
 * runs on, held until the process ends, instead of in the handle's buffers.  Calls no allocator.  Every entry of the
 * scratch is written before it is read, so nothing has to start at zero.  All
 * calls on one GPU share the array: calls that overlap on one GPU (two streams,
 * or two handles) race and must be ordered by the caller.
 * Errors: as bte_ion_step; BTE_EINVAL when sum_d Nx_d^2 + 3 sum_d Nx_d >
 * BTE_ION_SCRATCH_DOUBLES. */
#define BTE_ION_SCRATCH_DOUBLES 2097152
bte_status bte_ion_step_noalloc(bte_handle* h, const double* F, const double* ni_in, double* ni_out, double t_s,
                                void* stream);
/* One step of the hybrid model: n_i <- n_i^{n+1} by bte_ion_step, then
 * F <- bte_step(F, t_s) with the Poisson field of n_i^{n+1}.  ni is device
 * [sum Nx], updated in place.  POISSON field mode only (else BTE_EUNSUPPORTED). */
bte_status bte_hybrid_step(bte_handle* h, double* F, double* ni, double t_s, void* stream);

/* Velocity-space solver of bte_step / bte_vstep / bte_graph_capture.
 *   BTE_VSOLVER_LU (default): batched LU factorization of every point's system
 *     each step (FP64, or FP32/BF16 factors with FP64 iterative refinement).
 *   BTE_VSOLVER_GMRES: the paper's Krylov form (velocity space update of the
 *     semi-implicit scheme; Alg. vspace_action and Alg. vspace_action_precon):
 *     restarted GMRES per point in FP64, right-preconditioned by
 *     H_p = (I - dt (n0 C + s_p A))^-1 for the field bin p of the point: the
 *     n_bins bins split (-E_bound, E_bound) uniformly in u = E (bin_scale = 0)
 *     or in u = asinh(E / bin_scale) (bin_scale > 0: bins graded towards zero
 *     field, where the preconditioner no longer damps the speed-advection
 *     operator), s_p is the bin centre in u mapped back to E, and fields
 *     outside fall into the end bins.  The H_p are factored here, once, per
 *     discharge, by the batched LU in factor_precision: BTE_FP64,
 *     BTE_MIXED_FP32, or BTE_FACTORS_FP16 (FP32 factorization stored in FP16,
 *     solves accumulate in FP64).  E_bound <= 0 takes max_d |E0_d| (1 + |a1|)
 *     (CONST and RF fields only).  restart: Krylov vectors per cycle (1..63);
 *     cycles: restart cycles (1..100); a point stops when
 *     ||b - M x||_2 <= rtol ||b||_2 (GMRES estimate); points not converged after
 *     the last cycle latch BTE_ENOCONV, bte_get_status then reports the largest
 *     iteration count over the points and the largest relative residual estimate.
 *   BTE_VSOLVER_BANDED: the systems solved in the spherical-harmonic basis of
 *     eq. (f_expansion) (with nl == ntheta, P_S = P_O^-1): with the
 *     unknowns ordered l-major, the collision operator is block diagonal in l
 *     and the acceleration operator couples l to l +- 1, so
 *     I - dt (n0 C_h + E A_h) is banded with half-bandwidth 2 Nr - 1; the
 *     batched LU with partial pivoting runs restricted to that band (fill
 *     included) in FP64, between F_h = P_S F and F* = P_O F_h*.  With
 *     nl < ntheta the operator part of the ordinate system has rank Nr nl and the
 *     reduction is exact: (I - P_O K P_S)^-1 = I - P_O P_S + P_O (I - K)^-1 P_S
 *     (T_S T_O = I_nl), so F* = F + P_O (F_h* - F_h) with the Nr nl harmonic
 *     systems factored.  The other arguments are ignored.  Returns
 *     BTE_EUNSUPPORTED when ntheta > 64.
 *   BTE_VSOLVER_HESSENBERG: the same harmonic-basis systems (B - s A_h) u = F_h,
 *     B = I - dt n0 C_h (block diagonal in l), s = dt E, by their Hessenberg
 *     form: K = B^-1 A_h is reduced here, once per discharge, by Householder
 *     similarity to K = Q H Q^T (H upper Hessenberg), and each V step computes
 *     u = Q (I - s H)^-1 W F_h, W = Q^T B^-1, with one O(n^2) Givens solve per
 *     point instead of a factorization (the frequency-response form of Laub,
 *     1981), in FP64.  Setup is on the host, O(n^3) per discharge; the handle
 *     then holds W, Q and H (3 (Nr nl)^2 doubles per discharge).  A zero
 *     rotation latches BTE_ESINGULAR.  Other arguments ignored; BTE_EUNSUPPORTED
 *     when ntheta > 64.
 * The adjoint step always factors the dense ordinate-space systems (it needs
 * the transposed solves).
 * Synchronous (factors the bins).  Errors: BTE_EINVAL, BTE_ESINGULAR, BTE_ENOMEM, BTE_EHIP. */
typedef enum { BTE_VSOLVER_LU = 0, BTE_VSOLVER_GMRES = 1, BTE_VSOLVER_BANDED = 2, BTE_VSOLVER_HESSENBERG = 3 } bte_vsolver;
bte_status bte_set_vsolver(bte_handle* h, int32_t kind, int32_t n_bins, double E_bound, double bin_scale,
                           int32_t restart, int32_t cycles, double rtol, int32_t factor_precision);

/* Captures n_steps consecutive steps of F (times t0_s + k dt, k = 0..n_steps-1,
 * the same launches as bte_step) into a HIP graph owned by the handle,
 * replacing a previously captured one; nothing runs at capture.  The graph
 * holds the addresses of F and of the field buffers: they must stay valid and
 * are read and written at every bte_graph_launch.  A capture of one RF period
 * (1000 steps of dt = T/1000) replays every later period with the same field
 * phases.  Not with timing enabled.  Errors: BTE_EINVAL, BTE_EHIP. */
bte_status bte_graph_capture(bte_handle* h, double* F, double t0_s, int32_t n_steps, bte_field field);
/* Replays the captured graph on ``stream`` (asynchronous).  BTE_EINVAL if none. */
bte_status bte_graph_launch(bte_handle* h, void* stream);

/* Moments of F (eq. hybrid_discrete_c; k_i of the hybrid model): out[0][x] =
 * n_e [m^-3], out[1][x] = mean energy [eV], out[2][x] = ionization rate
 * coefficient k_i [m^3/s] (0 where n_e == 0).  out is device [3][sum Nx]. */
bte_status bte_moments(bte_handle* h, const double* F, double* out, void* stream);

/* Vector-Jacobian product of bte_moments: lam[x] += sum_q gbar[q][x] d out[q][x] / d F[x].
 * gbar: device [3][sum Nx]; lam: device like F (accumulated). */
bte_status bte_moments_vjp(bte_handle* h, const double* F, const double* gbar, double* lam, void* stream);

/* Transposed (adjoint) step for the specified-field modes (CONST, RF, GIVEN).
 * F_n is the state at t_s (the step is recomputed internally).  On entry lam
 * holds dL/dF^{n+1}; on exit dL/dF^n through this step.  With F* = A^-1 X F^n
 * and mu = A^-T X^T lam:
 *   grad_scal[s*n_bins+b] += dt n0_d sum_x mu_x^T C^(s,b) F*_x   (device [n_params], accumulated)
 *   grad_E0[d]           += sum_{x in d} (dL/dE_x) dE_x/dE0_d    (device [n_discharges], accumulated; may be NULL)
 *   grad_E[x]             = dt mu_x^T A F*_x                     (device [sum Nx], overwritten; may be NULL)
 * POISSON mode returns BTE_EUNSUPPORTED. */
bte_status bte_adjoint_step(bte_handle* h, const double* F_n, double t_s, bte_field field, double* lam,
                            double* grad_scal, double* grad_E0, double* grad_E, void* stream);

/* F = n_e(x) * (Galerkin projection of the unit-density Maxwellian at Te), the
 * same on every ordinate.  ne: device [sum Nx]; F: device like the state. */
bte_status bte_initial_maxwellian(bte_handle* h, const double* ne, double Te_eV, double* F, void* stream);

/* Sub-steps of bte_step, for tests and instrumentation (same kernels):
 *   bte_xstep:   F <- X(dt/2) F                         (Alg. bte_spatial_adv)
 *   bte_xstep_T: F <- X(dt/2)^T F
 *   bte_vstep:   F <- (I - dt(n0 C + E A))^-1 F at every x, E device [sum Nx]
 *   bte_field_eval: E_out <- E^{1/2} at t_s for state F^{n+1/2} (device [sum Nx]) */
bte_status bte_xstep(bte_handle* h, double* F, void* stream);
bte_status bte_xstep_T(bte_handle* h, double* F, void* stream);
bte_status bte_vstep(bte_handle* h, double* F, const double* E, void* stream);
bte_status bte_field_eval(bte_handle* h, const double* F_half, double t_s, bte_field field, double* E_out,
                          void* stream);

/* Host copies of the assembled operators (synchronous), for verification.
 * which: 0 C_ord [n][n] (sum_sb scal C^(s,b), per unit n0), 1 A_ord [n][n],
 *        2 M_v [Nr][Nr], 3 G_v [Nr][Nr], 4 eigenvalues Lambda [Nr], 5 U [Nr][Nr],
 *        6 xhat [sum Nx], 7 moment weights [3][n] (number, energy in eV, k_i),
 *        8 C^(s,b) [n_params][n][n], 9 Q of discharge 0 [Nr][Ntheta][Nx][Nx] (row-major Q_ia),
 *        10 C_h [Nr nl][Nr nl], 11 A_h [Nr nl][Nr nl]: the operators of C_ord and A_ord in
 *        the harmonic basis, unknowns ordered l-major (l * Nr + k), so that C_ord = P_O C_h P_S,
 *        12 T_O [Ntheta][nl] (F[k][a] = sum_l T_O[a][l] F_h[l][k]),
 *        13 T_S [nl][Ntheta] (F_h[l][k] = sum_a T_S[l][a] F[k][a]).
 * host_out must hold the documented number of doubles. */
bte_status bte_get_operator(bte_handle* h, int32_t which, double* host_out);

/* The same operators (which = 0..13) assembled on the host from a configuration,
 * without a device or handle (synchronous).  Used to verify the assembly.  Also
 * the Hessenberg form of discharge 0 (BTE_VSOLVER_HESSENBERG, n = Nr nl, n0 and
 * dt of the configuration): 14 W = Q^T B^-1 [n][n], 15 Q [n][n] (orthogonal),
 * 16 H [n][n] (upper Hessenberg, row-major), with B^-1 A_h = Q H Q^T. */
bte_status bte_host_operator(const bte_config* cfg, int32_t which, double* host_out);

/* Verification: forms and factors (I - dt (n0 C + E A)) at every point with the
 * field E (device [sum Nx]), synchronizes, and copies the factors of point x
 * (npad x npad column-major, npad = n rounded up to a multiple of 128, converted
 * to FP64) and its pivot rows (getrf-style, 0-based, applied panel by panel) to
 * host memory.  Overwrites the handle's factor workspace. */
bte_status bte_factor_export(bte_handle* h, const double* E, int32_t x, double* lu_host, int32_t* piv_host);

bte_status bte_get_info(bte_handle* h, bte_info* out);

/* Refinement of the mixed-precision V step (bte_config.refine_max_iter and
 * refine_rtol set it at setup): at most max_iter sweeps (1..100; <= 0: 10),
 * stopping once the normwise backward error of every point is <= rtol
 * (<= 0: 1e-14).  A V step that ends above rtol latches BTE_ENOCONV and leaves
 * its last iterate in F; the handle stays usable.  Applies from the next call
 * (a captured graph keeps the settings it was captured with).
 * Errors: BTE_EINVAL (max_iter > 100 or rtol not finite). */
bte_status bte_set_refine(bte_handle* h, int32_t max_iter, double rtol);

/* Synchronizes the handle's last stream and returns the latched device status
 * (then clears it), the refinement sweeps used by the last mixed V-step and the
 * final max|r|/max|b|.  Any pointer may be NULL. */
bte_status bte_get_status(bte_handle* h, int32_t* refine_iters, double* final_resid);

/* Kernel-level timing of bte_step (HIP events on the streams the kernels run
 * on).  enable: 1 = events around the phases of the step and around every LU
 * launch group, each timed step synchronizing the caller's stream; 2 = around
 * the phases only, with no wait between steps (the events of up to 64 steps
 * are read when their ring is full or by bte_get_timing), so that the walls
 * are those of steps running back to back ([0], [1] and [3] stay zero); 0 =
 * off (default).  Any call clears the sums; other values are EINVAL.  bte_get_timing fills
 * ms_out[0..5] with sums over the timed steps of: [0] the durations of the LU
 * trailing-update launches, [1] the durations of the LU panel + U12 launches
 * (both summed over the concurrent factorization streams, so they can exceed
 * the wall time), [2] the wall time of the V step, [3] the number of
 * trailing-update launches timed, [4] the wall time of the X half-steps and
 * the field, [5] the number of timed steps. */
bte_status bte_set_timing(bte_handle* h, int32_t enable);
bte_status bte_get_timing(bte_handle* h, double* ms_out);

/* Launch-shape tuning; apart from BTE_TUNE_PANEL_PAIRS, results do not depend
 * on it (every matrix is factored by the same arithmetic in the same order
 * whatever the shape).
 *   BTE_TUNE_LU_STREAMS: the points are split into this many groups of
 *     consecutive points, factored concurrently on the handle's own side
 *     streams (default priority) and joined back into the caller's stream with
 *     events, so that the latency-bound panel kernels of one group can overlap
 *     the MFMA updates of another.  1..4, default 1.
 *   BTE_TUNE_UPDATE_KC: K chunk of the trailing-update tiles staged per LDS
 *     buffer: 16 or 32 (FP32 factors), 8 or 16 (FP64); 0 = default (16).  The
 *     16-chunk FP32 form runs four blocks per CU, the 32-chunk form two.  The
 *     BF16 updates have a fixed chunk of 32 (reported as such).
 *   BTE_TUNE_FORM_XPB: matrices formed per block of the formation kernel,
 *     1..64; 0 = default (8 for FP32 factors, 16 for FP64).
 *   BTE_TUNE_PANEL_PAIRS: 2 (default), 1 or 0.  1: dense factors take the
 *     panels in pairs: a panel's update of the columns beyond the next panel is
 *     deferred and applied together with the next panel's in one update of
 *     depth 256, which reads and writes the trailing matrix half as often.  The
 *     factors then store each pair's second interchanges in the first panel's L
 *     rows as well (the solves follow).  2: statically pivoted dense factors
 *     take groups of four panels (the next panel's columns and top rows get the
 *     group's earlier panels' updates at depth 128 j, in place and in one
 *     launch, the columns beyond the group one update of depth 512; a last
 *     group that does not fit goes singly); other factors take pairs.  Measured
 *     at Nx = 256, n = 2048: 17.8 ms per FP32 step against 18.5 with pairs
 *     (BF16x3 14.45 against 15.15).  0: single panels.  Unlike the other keys this one changes the
 *     rounding of the trailing updates (not the pivots of a well-separated
 *     column); it only takes effect at the next factorization.
 *   BTE_TUNE_STATIC_PIVOTING: 0 or 1 (default 1 for the mixed precisions, 0 for
 *     FP64, where 1 is BTE_EINVAL).  1 factors the FP32 matrices without row
 *     interchanges (static pivoting: a pivot below 2^-20 of the largest entry
 *     of its 128 x 128 diagonal block is replaced by that bound, with its sign);
 *     each panel is then its diagonal block's factorization plus L21 = A21
 *     U11^-1, row-parallel, instead of 128 sequential pivot searches.  The FP64
 *     refinement works with the exact matrix, so the solution meets the same
 *     refine_rtol; a system that the perturbed factors cannot resolve latches
 *     BTE_ENOCONV (never BTE_ESINGULAR).  Changes the factors, not the result
 *     beyond rounding; takes effect at the next factorization.
 *   BTE_TUNE_LOOK_AHEAD: 0 (default) or 1.  With statically pivoted FP32
 *     factors and one factorization group, an update that reaches the next
 *     panel updates that panel's columns first; the panel's diagonal-block
 *     factorization and L21 then run on a side stream (default priority)
 *     during the rest of the update.  Same arithmetic in the same order: the
 *     results do not depend on it.  Measured at Nx = 256, n = 2048: 0.3 ms
 *     slower per FP32 step (the update fills every CU's registers, so the
 *     side kernels wait for its blocks to drain), 0.1 ms faster with the
 *     split-bf16 update; the autotuner tries both.
 *   BTE_TUNE_FORM_OVERLAP: 0 (default) or 1.  With statically pivoted FP32
 *     factors, panels in pairs, dense systems and one factorization group, the
 *     matrices' columns and rows below 256 are formed first, and the rest of
 *     each matrix (read first by the first depth-256 update) is formed on a
 *     side stream (default priority) while the first pair of panels factors.
 *     The same values are formed: the results do not depend on it.  Measured
 *     at Nx = 256, n = 2048: 0.05-0.1 ms slower per FP32 step (the formation's
 *     writes and the panels' reads share HBM and the CUs).
 * Returns BTE_EINVAL for an unknown key or a value out of range. */
typedef enum {
  BTE_TUNE_LU_STREAMS = 0,
  BTE_TUNE_UPDATE_KC = 1,
  BTE_TUNE_FORM_XPB = 2,
  BTE_TUNE_PANEL_PAIRS = 3,
  BTE_TUNE_STATIC_PIVOTING = 4,
  BTE_TUNE_LOOK_AHEAD = 5,
  BTE_TUNE_FORM_OVERLAP = 6
} bte_tune_key;
bte_status bte_set_tuning(bte_handle* h, int32_t key, int32_t value);
bte_status bte_get_tuning(bte_handle* h, int32_t key, int32_t* value);

void bte_destroy(bte_handle* h);
const char* bte_status_string(bte_status s);

#ifdef __cplusplus
}
#endif
#endif /* BTE_H */
