/*
 * libltmp2 -- Laplace-transformed MP2 (LTMP2) for periodic cells on one MI355X.
 *
 * C ABI over the hot path of the quartic-scaling plane-wave LTMP2 method of
 * Schaefer, Ramberger and Kresse ("Quartic scaling MP2 for solids",
 * arXiv:1611.06797).  Given Hartree-Fock orbitals and energies for all
 * occupied and virtual states (the inputs the paper's Implementation section
 * assumes), the library returns the direct and exchange MP2 correlation
 * energies of a cell: spin-restricted at the Gamma point (ltmp2_setup),
 * spin-unrestricted (ltmp2_setup_unrestricted) or on a k-point mesh
 * (ltmp2_setup_kpoints), optionally with the internal extrapolation of the
 * auxiliary cutoff.  For the spin-restricted Gamma-point cell:
 *
 *   E_d = -2 sum_n w_n Tr[(chi(tau_n) v)^2]                (Eq. dLTMP2Compact, q = 0)
 *   E_x =    sum_n w_n sum_{G,G'} v(G) v(G') sum_ij A^{G'}_ij(G) A^{-G'}_ji(-G)
 *                                                          (Eqs. SCHnewstate,
 *                                                           SCHtransmatrix, SCHfocklike)
 * with v(G) = 4 pi / (Omega |G|^2) on the auxiliary set (Eq. SCH2EI), the
 * Laplace transform of the energy denominator (Eq. SCHLT) and a minimax
 * quadrature (tau_n, w_n).
 *
 * Conventions (Hartree atomic units):
 *   - cubic cell of side L (bohr), Omega = L^3, FFT grid n^3, dV = Omega / n^3;
 *   - reciprocal vectors G = (2 pi / L) m with integer Miller indices m;
 *   - orbitals psi_p(r) = Omega^-1/2 sum_G c_p(G) e^{iG.r} must be real on the
 *     grid up to a phase per orbital (Gamma point, time-reversal symmetry:
 *     c_p(-G) = e^{2 i theta_p} conj c_p(G)), or span with their degenerate
 *     partners a time-reversal invariant block; setup brings them to real
 *     form (ltmp2_real_orbitals);
 *   - auxiliary set: G != 0 with |G|^2 / 2 <= eaux, |m_d| < n / 2;
 *   - real-space index used by device outputs: r = (x * n + z) * n + y
 *     for grid point (x, y, z) (z varies before y).
 *
 * Ownership: host inputs are copied during the call; device output buffers
 * are allocated by the caller and written on the context's stream; every
 * device allocation made by the library belongs to the context and is
 * released by ltmp2_destroy.  Calls return a status and never abort; a text
 * message is available from ltmp2_last_error.  After a device error the
 * context is failed and later calls return LTMP2_ESTATE.  A context must
 * not be used from two threads at once.
 */
#ifndef LTMP2_H
#define LTMP2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ltmp2_ctx ltmp2_ctx;

typedef enum {
  LTMP2_OK = 0,
  LTMP2_EINVAL = 1,   /* invalid argument or input data                    */
  LTMP2_EGAP = 2,     /* e_LUMO - e_HOMO <= 1e-8 Ha: the Laplace transform of
                         1/D needs e_i < e_F < e_a (LTMP2 subsection)        */
  LTMP2_ENOMEM = 3,   /* device memory (or the workspace cap) exhausted     */
  LTMP2_EDEVICE = 4,  /* HIP runtime error                                  */
  LTMP2_ESTATE = 5,   /* call on a failed context or out of order           */
  LTMP2_ENUMERIC = 6  /* quadrature fit failed / non-finite result          */
} ltmp2_status;

typedef enum {
  LTMP2_FP64 = 0,     /* FP64 throughout                                    */
  LTMP2_FP32 = 1,     /* FP32 storage and transforms; FP64 accumulations    */
  LTMP2_BF16X3 = 2    /* split-BF16x3 Green's-function GEMMs, FP32 otherwise */
} ltmp2_precision;

typedef enum {
  LTMP2_QUAD_PLAIN = 0,   /* library computes the minimax fit               */
  LTMP2_QUAD_LEARNED = 1, /* MLP proposal + Remez polish + certification   */
  LTMP2_QUAD_GIVEN = 2    /* caller passes tau and w                         */
} ltmp2_quad_mode;

typedef struct {
  double L;             /* cubic cell side, bohr (> 0)                          */
  int n_fft;            /* grid points per axis; one of the compiled sizes     */
  double ecut;          /* orbital cutoff, Ha: every basis G has |G|^2/2 < ecut */
  double eaux;          /* auxiliary cutoff, Ha (inclusive)                     */
  int n_pw;             /* plane-wave basis size                                */
  int n_states;         /* states passed (occupied first, then virtual);
                           0 means n_pw (all virtuals).  Passing a subset I of
                           the occupied states plus all virtuals gives the
                           energy restricted to i, j in I                       */
  int n_occ;            /* occupied states, 1 <= n_occ < n_states               */
  int n_tau;            /* Laplace points, 1..16                                */
  int quad_mode;        /* ltmp2_quad_mode                                      */
  int prec;             /* ltmp2_precision                                      */
  size_t workspace_cap; /* bytes; 0 = no cap.  Setup fails with LTMP2_ENOMEM if
                           the device footprint would exceed it                 */
  int n_extrap;         /* internal cutoff extrapolation (Implementation section,
                           "Internal cutoff extrapolation"): 0 = off, else the
                           number n_c (2..8) of nested auxiliary cutoffs
                           eaux / extrap_alpha^(n-1), n = 1..n_c, evaluated in
                           the same pass (ltmp2_get_extrapolation)              */
  double extrap_alpha;  /* ratio of consecutive cutoffs, > 1 (0: 1.05)         */
} ltmp2_params;

/* Sizes of a prepared context. */
typedef struct {
  int n_r;        /* n_grid^3: points of the internal transform grid      */
  int n_g;        /* auxiliary set size (G and -G both counted)           */
  int n_h;        /* n_g / 2: the half set, first in the library's order  */
  int n_pw, n_occ, n_vir, n_tau;
  double x_min, x_max;   /* bounds of -D = e_a + e_b - e_i - e_j          */
  double quad_delta;     /* certified max relative quadrature error       */
  size_t device_bytes;   /* device memory held by the context             */
  int quad_flags;        /* LTMP2_QUAD_LEARNED only: bit 0 the polished MLP
                            proposal was certified, bit 1 the plain fit was
                            used instead, bit 2 the weight file was unusable */
  int n_grid;            /* side of the internal transform grid: the smallest
                            compiled size <= n_fft with n_grid >= 2 k_orb +
                            k_aux + 1 (k_orb, k_aux: largest |Miller index| of
                            the orbital and auxiliary spheres), else n_fft.
                            Products of orbital-sphere functions are alias-free
                            at the auxiliary wavevectors on it, so every energy
                            equals the n_fft-grid value to rounding.  Grid rows
                            of ltmp2_green are on this grid. */
  int g_block;           /* outer G' of the half set per transformed-state
                            block (the exchange runs ceil(n_h / g_block) blocks
                            per Laplace point; set by the workspace budget) */
  int n_spin;            /* 1 (ltmp2_setup) or 2 (ltmp2_setup_unrestricted) */
  int n_occ_b;           /* occupied states of the second spin channel        */
  int n_k;               /* k-point mesh points per axis (ltmp2_setup_kpoints;
                            1 otherwise).  With n_k > 1 the sizes above are
                            those of the Born-von Karman supercell. */
} ltmp2_info;

/*
 * Prepare a cell (Implementation section, step (i)): validates all inputs on
 * the host before any device call, brings the orbitals to real form (as
 * ltmp2_real_orbitals), uploads them, synthesises the orbitals on the grid,
 * computes and stores the overlap densities <a|e^{-iG.r}|j> (Eq. SCHovrlp)
 * and fixes the Laplace quadrature.
 *   miller [n_pw][3] int32   basis Miller indices: closed under m -> -m,
 *                            without duplicates, and every (m_y, m_z)
 *                            column a run of consecutive m_x (a sphere);
 *                            LTMP2_EINVAL otherwise
 *   eps    [n_states]        orbital energies, ascending
 *   coeff  [n_states][n_pw][2]  state-major coefficients c_p(G), (re, im)
 *   tau, w [n_tau]           quadrature (only with LTMP2_QUAD_GIVEN, else NULL)
 *   mlp_weights              path of a weight file (LTMP2_QUAD_LEARNED), else NULL;
 *                            the proposal is polished by 3 Remez passes and
 *                            certified to 1e-6, else the plain fit is used
 *   hip_stream               hipStream_t to run on (NULL: default stream)
 * On success *out receives a context; on failure *out is NULL.
 */
ltmp2_status ltmp2_setup(const ltmp2_params* p, const int32_t* miller, const double* eps,
                         const double* coeff, const double* tau, const double* w,
                         const char* mlp_weights, void* hip_stream, ltmp2_ctx** out);

/*
 * Spin-unrestricted cell (Theory section, Eqs. MP2direct and MP2exchange):
 * two spin channels with their own orbitals and energies on one basis.  The
 * direct term sums over both channels of each of the two electron pairs, so
 * it is evaluated once on chi = chi_up + chi_down (the products of the two
 * channels' Green's functions added tile by tile); the exchange term couples
 * one channel only and is evaluated per channel, each at half weight.  For
 * identical channels every energy equals ltmp2_setup's.
 *   p                    as ltmp2_setup; p->n_occ is channel 1's count
 *   n_occ_b              occupied states of channel 2 (1 <= n_occ_b < n_states)
 *   miller               one basis for both channels, as ltmp2_setup
 *   eps_a, coeff_a       channel 1, laid out as ltmp2_setup's eps / coeff
 *   eps_b, coeff_b       channel 2, same layout
 *   tau, w, mlp_weights, hip_stream, out   as ltmp2_setup
 * One Laplace quadrature serves both channels: it is fitted on
 * [2 min(gap_1, gap_2), 2 max(spread_1, spread_2)] (gap: LUMO - HOMO,
 * spread: highest - lowest state of a channel), so it covers every
 * denominator of either channel; each channel keeps its own mu in its
 * Green's functions (the Laplace factors do not depend on mu).
 * On the returned context ltmp2_energy, ltmp2_chi, ltmp2_exchange and
 * ltmp2_get_extrapolation return spin-summed values: per tau the direct value
 * is 1/4 of the restricted trace formula on chi_up + chi_down (ltmp2_chi's
 * chi_GG_dev is that sum's transform) and the exchange value half the sum of
 * the two channels' restricted exchange values.  ltmp2_green returns channel
 * 1's functions; ltmp2_direct_hartree answers LTMP2_ESTATE.  ltmp2_get_info
 * reports n_spin = 2, n_occ_b and both channels' device bytes; ltmp2_destroy
 * frees both.  Device memory: the overlap densities and orbitals of each
 * channel; the chi and transformed-state scratch is shared (channel 2 runs
 * its transformed-state blocks in channel 1's buffers, with as many outer G'
 * per block as fit there, or in buffers of its own when not one fits).
 * p->workspace_cap bounds each channel's footprint separately.
 */
ltmp2_status ltmp2_setup_unrestricted(const ltmp2_params* p, int n_occ_b, const int32_t* miller,
                                      const double* eps_a, const double* coeff_a,
                                      const double* eps_b, const double* coeff_b,
                                      const double* tau, const double* w,
                                      const char* mlp_weights, void* hip_stream,
                                      ltmp2_ctx** out);

/*
 * k-point sampling (Theory section, "MP2 for periodic systems" and "LTMP2 in
 * the plane wave basis"; Eqs. BlochOrbital, 2eIPLWV, OverlapDens): the
 * Gamma-centred n_k^3 mesh k = (2 pi / L) kappa / n_k, kappa in
 * {0..n_k-1}^3, mesh index t = (kappa_x n_k + kappa_y) n_k + kappa_z.  The
 * Bloch states of the N = n_k^3 mesh points are, unchanged, the orbitals of
 * the Born-von Karman supercell of side n_k L (supercell Miller index
 * n_k m + kappa), whose Gamma-point MP2 energy is N times the energy per
 * unit cell of the mesh: the supercell's Coulomb wavevectors are the G + q of
 * Eq. 2eIPLWV, its auxiliary sphere the cutoff on |G + q|, and momentum
 * conservation is the orthogonality of its plane waves.  The context is that
 * supercell, prepared by the Gamma-point path; every energy it returns
 * (ltmp2_energy, ltmp2_chi, ltmp2_exchange, ltmp2_get_extrapolation,
 * ltmp2_direct_hartree) is per unit cell.  Cost grows as N^4 (the paper's
 * momentum-conserving loops grow as N^3).
 *   p          p->L, p->n_fft: the unit cell and its grid (the supercell uses
 *              n_k n_fft); p->n_states: bands per k (the same at every k);
 *              p->n_occ: occupied bands per k; p->n_pw: sum of n_pw_k
 *   n_k        mesh points per axis, 1..6
 *   n_pw_k     [N] basis size of each mesh point
 *   miller     [sum n_pw_k][3] int32, mesh point after mesh point: the m of
 *              the plane waves e^{i (G + k).r}, G = (2 pi / L) m
 *   eps        [N][n_states] band energies, ascending at each k
 *   coeff      per mesh point [n_states][n_pw_k][2] (re, im), concatenated;
 *              unit norm, time-reversal related (phi*_{k} = phi_{-k})
 * Errors: LTMP2_EINVAL for inconsistent sizes or a supercell basis the
 * Gamma-point rules reject (the per-k spheres of a cutoff make a supercell
 * sphere); LTMP2_EGAP when an occupied band at one k lies above a virtual
 * band at another (no common gap).  Host memory: the unfolded coefficient
 * table, N n_states x n_pw doubles x 2, during setup.
 */
ltmp2_status ltmp2_setup_kpoints(const ltmp2_params* p, int n_k, const int32_t* n_pw_k,
                                 const int32_t* miller, const double* eps, const double* coeff,
                                 const double* tau, const double* w, const char* mlp_weights,
                                 void* hip_stream, ltmp2_ctx** out);

/*
 * Occupied and virtual imaginary-time Green's functions at tau_itau
 * (the occupied and virtual sums of Eq. dLTMP2Compact), rows [row0, row0 + nrows) of the n_r x n_r matrices
 *   G_occ(r, r') = sum_i psi_i(r) exp((e_i - mu) tau) psi_i(r')
 *   G_vir(r, r') = sum_a psi_a(r) exp(-(e_a - mu) tau) psi_a(r')
 * with mu = (e_HOMO + e_LUMO) / 2, written as doubles [nrows][n_r] to the
 * caller's device buffers (either may be NULL); r runs over the internal
 * transform grid (ltmp2_info.n_grid).  The rows are computed in the
 * context's precision by the same operand forms the energy uses (FP64, FP32,
 * or split-BF16x3 operands with FP32 accumulation).  Diagnostic entry point.
 */
ltmp2_status ltmp2_green(ltmp2_ctx* ctx, int itau, int row0, int nrows, void* gocc_dev,
                         void* gvir_dev);

/*
 * Direct term at tau_itau (Eq. dLTMP2Compact at q = 0, the Laplace-transformed
 * direct energy written with the Green's functions of the same equation):
 * chi(r, r') = G_occ(r, r') G_vir(r', r) tile by tile, its double Fourier
 * transform
 *   chi(G, G') = dV^2 sum_{r, r'} e^{-iG.r} chi(r, r') e^{iG'.r'}
 * on the auxiliary set and the Coulomb trace
 *   *e_direct_tau = -2 sum_{G, G'} v(G) v(G') |chi(G, G')|^2   (unweighted).
 * chi_GG_dev (may be NULL) receives chi(G, G') as complex doubles
 * [n_g][n_g] in the library's auxiliary order (ltmp2_aux_miller).
 */
ltmp2_status ltmp2_chi(ltmp2_ctx* ctx, int itau, void* chi_GG_dev, double* e_direct_tau);

/*
 * Direct term at tau_itau by the paper's own Hartree-like step (Implementation
 * section, step (iv.a)): for every outer G', the transformed states
 * w_i^{(G')} of the exchange path (Eqs. SCHnewstate, SCHtransmatrix), their
 * sum h(r) = sum_i psi_i(r) w_i^{(G')}(r), its transform
 * X(G) = dV sum_r e^{-iG.r} h(r) (= chi(G, -G') of the Green's-function
 * route) and
 *   *e_direct_tau = -2 sum_{G, G'} v(G) v(G') |X^{(G')}(G)|^2   (unweighted).
 * Equal to ltmp2_chi's value; none of the Green's-function, chi-transform or
 * trace kernels take part, so the two routes check each other.  Uses the
 * context's chi scratch (LTMP2_ESTATE on a cell of a batch).
 */
ltmp2_status ltmp2_direct_hartree(ltmp2_ctx* ctx, int itau, double* e_direct_tau);

/*
 * Exchange term at tau_itau through the transformed states of
 * Eqs. SCHnewstate / SCHtransmatrix and the Fock-like contraction of
 * Eq. SCHfocklike (Implementation section, steps (iii) and (iv.b)):
 *   *e_exchange_tau = sum_{G'} v(G') sum_G v(G) sum_ij A^{G'}_ij(G) A^{-G'}_ji(-G)
 * (unweighted).  g_first / g_count select a range of the half set H of
 * outer G' (g_count <= 0: all); the value then covers G' and -G' of that
 * range only, so disjoint ranges add up to the full term.
 */
ltmp2_status ltmp2_exchange(ltmp2_ctx* ctx, int itau, int g_first, int g_count,
                            double* e_exchange_tau);

/*
 * Full energy: the Laplace transform of the energy denominator (Eq. SCHLT)
 * evaluated by the quadrature, E_d = sum_n w_n E_d(tau_n) and
 * E_x = sum_n w_n E_x(tau_n) (Eqs. dLTMP2Compact and xLTMP2Compact at q = 0),
 * summed in FP64 (Ha per cell).  per_tau (may be NULL) receives [2 n_tau]
 * unweighted values (E_d(tau_n), E_x(tau_n)) pairs; quad_err (may be NULL)
 * the certified max relative error of the quadrature.
 */
ltmp2_status ltmp2_energy(ltmp2_ctx* ctx, double* e_direct, double* e_exchange,
                          double* per_tau, double* quad_err);

/*
 * Internal cutoff extrapolation (Implementation section, "Internal cutoff
 * extrapolation"; Eq. CutDecay), available after ltmp2_energy on a context
 * set up with n_extrap = n_c > 0.  During the energy every Coulomb-weighted
 * (G, G') sum is also split by the nested auxiliary spheres
 * |G|^2 / 2 <= eaux / alpha^(n-1), n = 1..n_c: a term counts for sphere n iff
 * both vectors lie in it, which gives the energy of every smaller auxiliary
 * cutoff exactly (the orbitals, overlap densities and quadrature do not
 * depend on it).  The energies are then fitted by E[n] = a + b eaux[n]^(-3/2)
 * (least squares, FP64); a is the extrapolated energy.
 *   e_aux      [n_c]  the cutoffs eaux[n] (Ha)              (may be NULL)
 *   e_direct   [n_c]  E_d at each cutoff (Ha; e_direct[0] = ltmp2_energy's)
 *   e_exchange [n_c]  E_x at each cutoff                     (may be NULL)
 *   e_inf      [3]    intercepts of E_d + E_x, E_d and E_x   (may be NULL)
 * LTMP2_ESTATE if the context has no extrapolation or no energy yet.
 */
ltmp2_status ltmp2_get_extrapolation(const ltmp2_ctx* ctx, double* e_aux, double* e_direct,
                                     double* e_exchange, double* e_inf);

/* Quadrature in use: tau, w [n_tau] (host), may be NULL. */
ltmp2_status ltmp2_get_quadrature(const ltmp2_ctx* ctx, double* tau, double* w, double* delta);

/* Sizes of the context. */
ltmp2_status ltmp2_get_info(const ltmp2_ctx* ctx, ltmp2_info* info);

/* Miller indices of the auxiliary set in the library's order, [n_g][3]
 * (half set H first, then -H in the same order). */
ltmp2_status ltmp2_aux_miller(const ltmp2_ctx* ctx, int32_t* out);

/*
 * Host-only relative-error minimax Laplace quadrature for 1/x on
 * [x_min, x_max] (Eq. SCHLT evaluated by a quadrature, LTMP2 subsection):
 * minimises max |x sum_n w_n e^{-x tau_n} - 1| by Remez exchange with
 * continuation in R = x_max / x_min.  For n_tau >= 9 the fit is computed on
 * [x_min, x_min * max(R, R_floor)], R_floor = exp(0.5 (n_tau - 10) + 3.8),
 * the double-precision limit of the exchange.  tau, w [n_tau] ascending in
 * tau; delta = certified max relative error.  Touches no device.
 */
ltmp2_status ltmp2_quadrature(double x_min, double x_max, int n_tau, double* tau, double* w,
                              double* delta);

/*
 * Per-stage device timing (diagnostics for roofline accounting).  When on,
 * every kernel launch of the hot path is bracketed by HIP events on the
 * context's stream; ltmp2_get_timing synchronises the stream and returns the
 * summed milliseconds and launch count of one stage:
 *   0 chi tiles (G_occ / G_vir GEMMs + Hadamard), 1 chi row transforms,
 *   2 chi column transforms + Coulomb trace, 3 transformed-state GEMM,
 *   4 transformed-state synthesis, 5 Fock-like pair transforms, 6 reductions.
 * ltmp2_set_timing(ctx, 1) also clears the accumulated values.
 */
ltmp2_status ltmp2_set_timing(ltmp2_ctx* ctx, int on);
ltmp2_status ltmp2_get_timing(ltmp2_ctx* ctx, int stage, double* ms, long* launches);

/*
 * Learned Laplace quadrature (grown form of the quadrature step).  A small
 * network 3 -> 64 (tanh) -> 64 (tanh) -> 24 (FP32, LTMP2_MLP_NPARAM floats:
 * W1[64][3] b1[64] W2[64][64] b2[64] W3[24][64] b3[24]) maps the features
 * (log x_min, log R / log 1e4, n_tau / 12), R = x_max / x_min, to the
 * logarithms of the unit-interval exponents (outputs 0..11) and weights
 * (outputs 12..23) of the n_tau-point minimax fit.  It is trained on the GPU
 * by the library's own forward / backward / Adam kernels on fits that the
 * plain method generates.  Weight files: 8 bytes "LTMP2MLP", uint32 version
 * (1), uint32 count (LTMP2_MLP_NPARAM), then the floats, little endian.
 */
#define LTMP2_MLP_NPARAM 5976

/* Seeded Glorot-uniform initial parameters (host). */
ltmp2_status ltmp2_mlp_init(uint64_t seed, float* params);

/* Plain minimax fits for ascending ratios R[0..count) in one continuation
 * sweep (host): alpha, beta [count][n_tau] on [1, max(R, R_floor)], delta
 * [count] (may be NULL). */
ltmp2_status ltmp2_quadrature_table(int n_tau, int count, const double* R, double* alpha,
                                    double* beta, double* delta);

/* Seeded training set (host): count samples with x_min log-uniform in
 * [dmin_lo, dmin_hi], R log-uniform in [ratio_lo, ratio_hi], n_tau drawn from
 * n_taus[0..n_choices) (each in 1..12), random numbers from splitmix64(seed);
 * X [count][3] features, Y [count][24] targets, M [count][24] mask,
 * xrange [count][2] (x_min, x_max) or NULL. */
ltmp2_status ltmp2_mlp_dataset(int count, uint64_t seed, double dmin_lo, double dmin_hi,
                               double ratio_lo, double ratio_hi, const int* n_taus, int n_choices,
                               float* X, float* Y, float* M, double* xrange);

/* Network outputs for n inputs (host arrays; computed on the GPU). */
ltmp2_status ltmp2_mlp_forward(const float* params, const float* X, int n, float* Y,
                               void* hip_stream);

/*
 * Network outputs for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops): the same forward pass as
 * ltmp2_mlp_forward on caller-owned DEVICE arrays, params_dev
 * [LTMP2_MLP_NPARAM], X_dev [n][3], Y_dev [n][24] (floats), enqueued on
 * hip_stream without synchronising and without any allocation; the hidden
 * activations use a fixed 8 MiB device array of the library (at most
 * LTMP2_MLP_NOALLOC_MAX_ROWS rows per call, else LTMP2_EINVAL).  Each GPU
 * holds one such array for the life of the process: calls that overlap on
 * one GPU race.
 */
#define LTMP2_MLP_NOALLOC_MAX_ROWS 16384
ltmp2_status ltmp2_mlp_forward_noalloc(const float* params_dev, const float* X_dev, int n,
                                       float* Y_dev, void* hip_stream);

/* Gradient of the masked mean squared error (host arrays; GPU kernels):
 * grad [LTMP2_MLP_NPARAM], *loss = sum M (out - Y)^2 / sum M. */
ltmp2_status ltmp2_mlp_grad(const float* params, const float* X, const float* Y, const float* M,
                            int n, float* grad, float* loss, void* hip_stream);

/* Adam training on the GPU (cosine learning-rate decay, seeded shuffles);
 * params is updated in place; loss_hist [epochs] may be NULL. */
ltmp2_status ltmp2_mlp_train(float* params, const float* X, const float* Y, const float* M, int n,
                             int epochs, int batch, float lr, uint64_t seed, float* loss_hist,
                             void* hip_stream);

/* MLP proposal for [x_min, x_max], polish_steps Remez passes, certification
 * (2 n_tau + 1 alternating extrema equal to cert_tol relative), else the
 * plain fit.  flags: bit 0 certified, bit 1 fell back to the plain fit. */
ltmp2_status ltmp2_learned_quadrature(const float* params, double x_min, double x_max, int n_tau,
                                      int polish_steps, double cert_tol, double* tau, double* w,
                                      double* delta, int* flags, void* hip_stream);

/* Host-only Remez polish of a proposal (tau, w updated in place): `steps`
 * exchange passes on [x_min, x_max]; *certified = 1 if the 2 n_tau + 1
 * alternating extrema agree to cert_tol relative. */
ltmp2_status ltmp2_remez_polish(double x_min, double x_max, int n_tau, int steps, double cert_tol,
                                double* tau, double* w, double* delta, int* certified);

/* Message of the last failed MLP / table call on this thread. */
const char* ltmp2_mlp_last_error(void);

/*
 * Batched evaluation of many independent cells (grown form: many small cells
 * of uneven size, each with its own Laplace grid).  Cells are grouped by FFT
 * grid; per Laplace point and round of outer G', one persistent fused launch
 * evaluates the Fock-like pair transforms of every cell of a group; the large
 * scratch is pooled; a tuner picks the pair kernel's slab tile and resident
 * workgroups per CU on first use; the launch sequence is captured into a
 * hipGraph after the first (eager) evaluation and replayed afterwards.
 * Per-cell arrays are as in ltmp2_setup; tau / w may be NULL (or hold NULL
 * entries for cells without a given quadrature).  All cells must use the same
 * precision.  If hip_stream is NULL the batch creates its own stream.
 */
typedef struct ltmp2_batch ltmp2_batch;

typedef struct {
  int n_cells, n_groups;
  int graph_ready;        /* 1 once the launch sequence is captured          */
  size_t device_bytes;
} ltmp2_batch_stats;

ltmp2_status ltmp2_batch_create(int n_cells, const ltmp2_params* params,
                                const int32_t* const* miller, const double* const* eps,
                                const double* const* coeff, const double* const* tau,
                                const double* const* w, const char* mlp_weights,
                                void* hip_stream, ltmp2_batch** out);
/* e_direct, e_exchange [n_cells] (Ha per cell). */
ltmp2_status ltmp2_batch_energy(ltmp2_batch* b, double* e_direct, double* e_exchange);
ltmp2_status ltmp2_batch_info(const ltmp2_batch* b, ltmp2_batch_stats* stats);
/* Stage timing as for a single context, summed over cells; stage 5 times
 * the fused multi-cell pair launches.  While timing is on, evaluations run
 * eagerly (not from the captured graph) so that launches can be bracketed. */
ltmp2_status ltmp2_batch_set_timing(ltmp2_batch* b, int on);
ltmp2_status ltmp2_batch_get_timing(ltmp2_batch* b, int stage, double* ms, long* launches);
/* Group g: grid size, cells, rounds of outer G', tuned slab tile and
 * workgroups per CU of the fused pair launch, tuned launch time (ms). */
ltmp2_status ltmp2_batch_group(const ltmp2_batch* b, int g, int* n_fft, int* n_cells, int* rounds,
                               int* slab_tile, int* wg_per_cu, double* tuned_ms);
ltmp2_status ltmp2_batch_cell(const ltmp2_batch* b, int k, ltmp2_info* info);
void ltmp2_batch_destroy(ltmp2_batch* b);
const char* ltmp2_batch_last_error(const ltmp2_batch* b);

/*
 * Host-only: orbitals that are real on the grid up to a phase per orbital
 * (a non-degenerate Gamma-point eigenstate of a real potential, the paper's
 * time-reversal subsection) are multiplied by the phase that makes them real;
 * a block of degenerate orbitals (energies equal to 1e-9 relative) that is
 * not real orbital by orbital is replaced by a real orthonormal basis of its
 * span.  Energies of the method are unchanged by either step.
 *   miller [n_pw][3], eps [n_states] ascending, coeff_in / coeff_out
 *   [n_states][n_pw][2] (may alias); n_occ marks the occupied states.
 * Returns LTMP2_EINVAL for a state with no real form (not time-reversal
 * invariant), LTMP2_EGAP for a degenerate block across n_occ.  Touches no
 * device.
 */
ltmp2_status ltmp2_real_orbitals(int n_pw, const int32_t* miller, int n_states, const double* eps,
                                 int n_occ, const double* coeff_in, double* coeff_out);

/* Release a context and all of its device memory (NULL is ignored). */
void ltmp2_destroy(ltmp2_ctx* ctx);

/* Message of the last error on ctx (or of the last failed setup if ctx is
 * NULL).  Valid until the next call on the same context. */
const char* ltmp2_last_error(const ltmp2_ctx* ctx);

/* Compiled grid sizes: writes up to cap values to sizes, returns the count. */
int ltmp2_supported_grids(int* sizes, int cap);

#ifdef __cplusplus
}
#endif

#endif /* LTMP2_H */
