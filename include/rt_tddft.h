/*
 * rt_tddft.h -- C ABI of the MI355X real-time TDDFT time-step library.
 *
 * One time step of Kohn-Sham electron dynamics on a real-space grid, in the
 * density-matrix form of arXiv:2410.09189 (Jakowski et al.): the Hamiltonian is
 * applied to every active orbital on the grid and projected to the orbital
 * basis, the density matrix is advanced by the first-order Magnus (midpoint)
 * operator through the commutator series, and the density, Hartree and
 * exchange potentials are rebuilt, all inside the self-consistent Hamiltonian
 * loop of Algorithm 1.
 *
 * Conventions shared by every call
 *   - Atomic units (hbar = m_e = e = 1).
 *   - Grid arrays are C-order [nz][ny][nx] (x fastest); grid point (i,j,k) sits
 *     at (i h, j h, k h) in a periodic cell of side n h per axis.
 *   - Orbital arrays are orbital-major [N][nz][ny][nx]; orbitals are real
 *     (Gamma point) and orthonormal under the quadrature <f,g> = h^3 sum f g.
 *   - N x N matrices are row-major double.  The density matrix is carried as the
 *     pair (S', A') of its real symmetric and imaginary antisymmetric parts.
 *   - Host pointers are read during the call only; the library copies what it
 *     keeps.  Device pointers are caller-owned and must stay valid for the call.
 *   - All device work is enqueued on the stream given to rt_init.  rt_step with
 *     stats == NULL and rt_apply_h are asynchronous; rt_dipole and the matrix
 *     getters synchronise the stream.
 *   - Every call returns an rt_status; no exception crosses the ABI.  On any
 *     status other than RT_OK, rt_last_error(ctx) names the cause.  RT_EINVAL
 *     leaves no side effects.  One context must not be used from two threads
 *     at once.
 */
#ifndef RT_TDDFT_H
#define RT_TDDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_ctx rt_ctx; /* opaque; created by rt_init, released by rt_free */

typedef enum {
  RT_OK = 0,
  RT_EINVAL = -1,   /* inconsistent or out-of-range argument                     */
  RT_ENOMEM = -2,   /* workspace smaller than rt_workspace_size reported          */
  RT_EDEVICE = -3,  /* a HIP call failed                                          */
  RT_ENOCONV = -4,  /* self-consistent loop or commutator series hit its cap      */
  RT_ESTATE = -5    /* call not valid in the context's current state              */
} rt_status;

enum { RT_FP64 = 0, RT_MIXED = 1 };               /* arithmetic of the time step   */
/* first guess of H(t + dt): RT_PRED_LINEAR 2 H_0 - H_-1 (Algorithm 1);
   RT_PRED_MLP the linear guess plus a learned correction (below);
   RT_PRED_QUADRATIC 3 H_0 - 3 H_-1 + H_-2 (extrapolation error O(dt^3) instead of
   O(dt^2); the fixed point is the same, only the number of updates changes).
   H_-1 = H_-2 = H_0 at the first step and after rt_set_state with hm1 (H_-2 = hm1). */
enum { RT_PRED_LINEAR = 0, RT_PRED_MLP = 1, RT_PRED_QUADRATIC = 2 };
enum { RT_HUPDATE_FULL = 0, RT_HUPDATE_LOCAL = 1 };/* how H[P] is rebuilt, below    */

/*
 * One molecule: grid, synthetic electron-ion terms and the ground-state active
 * space (Algorithm 1, ground-state and active-space blocks).
 *
 * Electron-ion terms (stand-ins for the norm-conserving pseudopotentials of
 * Sec. Overview of RMG):
 *   V_ion(r) = - sum_a depth[a] sum_{images |n_q| <= n_images}
 *                exp(-|r - pos_a - n L|^2 / (2 width[a]^2))
 *   V_nl     = sum_a sum_p |beta_ap> nl_D[a*nl_rank+p] <beta_ap| (h^3 quadrature),
 *              beta_a1 ~ g(s), beta_a(1+q) ~ (s_q / nl_sigma) g(s), q = x,y,z,
 *              g(s) = exp(-s^2/(2 nl_sigma^2)) (1 - s^2/nl_rcut^2)^2 for s < nl_rcut
 *              (minimum-image displacement s), each column h^3-normalised.
 * psi0: the N = n_occ + n_virt ground-state orbitals, FP64 [N][nz][ny][nx],
 *   host memory unless psi0_on_device != 0.  If orthonormalize != 0 they are
 *   first made h^3-orthonormal by S = h^3 Psi Psi^T = L L^T, Psi <- L^-1 Psi
 *   (basis transform of the paper's non-orthogonal formulation, Appendix).
 *   If nonorthogonal != 0 (excludes orthonormalize) they are kept as a
 *   non-orthogonal basis with overlap S = h^3 Psi Psi^T = L L^T and every
 *   propagation runs the series of eq. commutator-expansion-nonort,
 *   dP^(k) = (1/k)(-i dt)(S^-1 Hbar dP^(k-1) - dP^(k-1) Hbar S^-1); the initial
 *   density matrix is L^-T diag(f) L^-1 (the occupations of the basis
 *   orthonormalised by L, written in the given basis), the kick and the field
 *   act through S^-1 M_q, and the reported electron count is Tr(P S).  Not
 *   combined with magnus_order 4 or the learned predictor (RT_EINVAL); a basis
 *   whose overlap is not positive definite gives RT_EINVAL at rt_init.
 * occ: occupations f_i (nullable: 2 for the first n_occ, 0 for the rest).
 *
 * Sawtooth field and vacuum dipole correction (Sec. Algorithm, time-dependent
 * field: the constant field is a sawtooth potential with a dipole correction in
 * the vacuum, after Bengtsson, Phys. Rev. B 59, 12301 (1999)).  The position
 * operator along axis q is the sawtooth s_q(i) = (((i - j0) mod n_q) - (n_q-1)/2) h
 * with j0 = saw_jump[q] in [0, n_q) (0: jump at the cell faces); it gives the
 * dipole matrices M_q, the kick and the field.  Put j0 in the vacuum.  If bit q
 * of dipole_correction is set, the cell's dipole written for electrons,
 * d_q = h^3 sum rho s_q - sum_a Z_a s_q(R_a) (ions as point charges Z_a at
 * their positions, s_q taken there in its continuous form), adds
 * (4 pi / Omega) d_q s_q to V_loc (Omega = cell volume) and (2 pi / Omega) d_q^2
 * to the electrostatic energy, at every Hamiltonian evaluation (time step and
 * ground state).  This cancels the uniform field that periodic images of the
 * dipole set up.  ion_charge: Z_a [n_atoms], nullable: the electron count
 * sum_i f_i shared equally between the atoms (a neutral cell).  A zeroed tail
 * is the plain sawtooth with its jump at the faces and no correction.
 * RT_EINVAL: a jump outside [0, n_q) or a mask outside [0, 7].
 */
typedef struct {
  int n[3];            /* nx, ny, nz; each in [8, 256]                           */
  double h;            /* grid spacing (bohr)                                    */
  int n_atoms;
  const double* pos;   /* [n_atoms][3] bohr                                      */
  const double* depth; /* [n_atoms] Ha                                           */
  const double* width; /* [n_atoms] bohr                                         */
  int n_images;        /* periodic images summed per axis for V_ion (0..3)       */
  int nl_rank;         /* 0 or 4                                                 */
  double nl_rcut;      /* projector radius (bohr)                                */
  double nl_sigma;     /* projector Gaussian width (bohr)                        */
  const double* nl_D;  /* [n_atoms][nl_rank] Ha (nullable when nl_rank == 0)    */
  int n_occ;
  int n_virt;
  const double* occ;   /* [N] or NULL                                            */
  const double* psi0;  /* [N][nz][ny][nx]                                        */
  int psi0_on_device;
  int orthonormalize;
  int nonorthogonal;   /* propagate in the given basis with its overlap (above)  */
  int saw_jump[3];     /* sawtooth jump plane per axis (above)                   */
  int dipole_correction; /* bit q: vacuum dipole correction along axis q (above) */
  const double* ion_charge; /* [n_atoms] point charges for the correction, or NULL */
} rt_system;

/*
 * Time loop and trajectories (Algorithm 1, parameter block).  Each trajectory
 * starts from P_0 = diag(f) of its system, receives a delta kick
 * P(0+) = exp(-i kappa M_q) P_0 exp(+i kappa M_q) along axis q (Sec. Numerical
 * Results, kick perturbation; applied through the same commutator series with
 * Omega = -i kappa M_q), and sets H_0 = H[P(0+)], H_-1 = H_0.
 *
 * hupdate selects how H[P] = h^3 Psi^T [T + V_ion + V_nl + V_H + v_x] Psi is
 * rebuilt in the self-consistent loop:
 *   RT_HUPDATE_FULL  -- the grid Hamiltonian is applied to every orbital (FD
 *                       stencil + local + nonlocal) and projected, as in the
 *                       paper's Hamiltonian update.  In FP64 with several
 *                       trajectories per system the workspace holds each
 *                       trajectory's H Psi (n_traj N Ng doubles, if at most
 *                       16 GiB) so one launch projects them all; otherwise
 *                       they take turns in one buffer.  Same results.
 *   RT_HUPDATE_LOCAL -- the orbitals are fixed during propagation, so only the
 *                       Hartree-exchange part changes: H[P] = H_gs +
 *                       h^3 Psi^T diag(V_Hx[P] - V_Hx[P_gs]) Psi, with H_gs built
 *                       once by the full apply.  Same fixed point.
 * precision RT_MIXED computes that perturbation projection and the density
 * change from the ground state in BF16x3 (split hi/lo, FP32 accumulate) and
 * keeps H_gs, rho_gs, the series, energy and dipole in FP64; it implies
 * RT_HUPDATE_LOCAL.
 */
typedef struct {
  double dt;           /* time step (a.u.)                                       */
  int n_steps_max;     /* capacity of the dipole/energy history                  */
  double h_thrs;       /* max|H_1 - H_1_old| that ends the self-consistent loop  */
  double dp_thrs;      /* max|dP^(k)| that ends the commutator series            */
  int max_scf;         /* cap on Hamiltonian updates per step (>= 1)             */
  int max_terms;       /* cap on series terms per propagation (>= 1)             */
  int precision;       /* RT_FP64 | RT_MIXED                                     */
  int predictor;       /* RT_PRED_LINEAR | RT_PRED_MLP | RT_PRED_QUADRATIC        */
  int hupdate;         /* RT_HUPDATE_FULL | RT_HUPDATE_LOCAL                     */
  int frozen_hxc;      /* test switch: V_H and v_x fixed at the ground state     */
  int n_traj;                /* at most 256 trajectories per system              */
  const int* traj_sys;       /* [n_traj] index into the system array             */
  const double* traj_kappa;  /* [n_traj] kick strength                           */
  const int* traj_axis;      /* [n_traj] 0 = x, 1 = y, 2 = z                     */
  const float* mlp_params;   /* RT_PRED_MLP: packed network (host, rt_mlp_n_params of
                                rt_mlp_dims floats, layout under "Learned predictor")   */
  /* External field (Algorithm 1 inputs E_x(t), E_y(t), E_z(t)), nullable; host
     [n_traj][7] = a, omega, tau, phase, d_x, d_y, d_z per trajectory:
       E(t) = a sin^2(pi t / tau) sin(omega t + phase) (d_x, d_y, d_z), 0 <= t <= tau,
       E(t) = 0 otherwise, t measured from the kick (t_j = j dt after j steps).
     V(t) = sum_q E_q(t) M_q enters the midpoint of step j -> j+1 as
     (V(t_j) + V(t_(j+1)))/2 (Magnus line of Algorithm 1); the self-consistency
     residual compares the Kohn-Sham part only.  Requires tau > 0.              */
  const double* traj_field;
  int magnus_order;          /* 0 or 2: Omega_1 only (the paper's midpoint);
                                4: Omega_1 + Omega_2, Omega_2 = (dt^2/12)
                                [H_0 + V(t_j), H_1 + V(t_(j+1))] (Sec. Magnus
                                expansion, H linear over the step), taken into
                                every series term; other values: RT_EINVAL      */
  int graph_capture;         /* 1: every Hamiltonian update (density, Hartree, LDA,
                                projection, residual) and every series start with
                                its first 8 terms is launched as an executable
                                hipGraph captured once per buffer arrangement
                                (at most a few per system: the buffers rotate);
                                0: eager launches.  Off while the phase timers of
                                rt_profile are on.  Results are identical.        */
  int h_block;               /* orbitals per block of the initial FP64 grid
                                Hamiltonian application; 0: all at once.  With
                                0 < h_block < N the orbital buffer beside Psi
                                holds h_block orbitals instead of N (Psi^T H Psi
                                is assembled block by block, H_gs as H_core +
                                h^3 Psi^T diag(V_H + v_x) Psi), which is what lets
                                a 192^3 x 3000-orbital system fit one device;
                                needs hupdate RT_HUPDATE_LOCAL (or RT_MIXED) and
                                no system with orthonormalize (RT_EINVAL).
                                Results agree with h_block = 0 within rounding. */
} rt_run;

/* Per-trajectory, per-step counters written by rt_step when stats != NULL. */
typedef struct {
  int32_t scf_iters;   /* Hamiltonian updates in this step                       */
  int32_t series_terms;/* commutator-series terms summed over those updates      */
  double residual;     /* final max|H_1 - H_1_old|                               */
} rt_step_stats;

/* Bytes of device workspace rt_init needs for this problem. */
rt_status rt_workspace_size(const rt_system* sys, int n_sys, const rt_run* run, size_t* bytes);

/*
 * Builds the context: uploads (and optionally orthonormalises) the orbitals,
 * builds V_ion, projector tables, H_core and the dipole matrices
 * M_q = h^3 Psi^T diag(q) Psi (q: centred sawtooth coordinate, Sec. Algorithm),
 * then applies each trajectory's kick and computes H_0.
 * workspace_dev: device memory of at least rt_workspace_size bytes, owned by
 * the caller, untouched by the caller until rt_free.  hip_stream: a
 * hipStream_t (NULL = default stream).  The library never allocates device
 * memory itself.  psi0 with NaN or infinite entries gives RT_EINVAL.
 */
rt_status rt_init(const rt_system* sys, int n_sys, const rt_run* run, void* workspace_dev,
                  size_t ws_bytes, void* hip_stream, rt_ctx** out);

/*
 * (H psi_j)(r) = -1/2 L_FD psi_j + V_loc psi_j + V_nl psi_j for j < n_orb
 * (Eq. DFT with the kinetic sign read as -1/2 Laplacian; 8th-order central
 * differences, Sec. Overview of RMG), V_loc = V_ion + V_H + v_x of the
 * system's current density (after rt_init: that of the last Hamiltonian
 * update).  psi_dev, hpsi_dev: caller-owned device arrays [n_orb][nz][ny][nx]
 * of dtype 0 = double, 1 = float; they must not overlap.
 */
rt_status rt_apply_h(rt_ctx* ctx, int sys_index, const void* psi_dev, void* hpsi_dev, int n_orb,
                     int dtype);

/*
 * Advances every trajectory by n_steps steps of Algorithm 1: predictor
 * H_1 = 2 H_0 - H_-1; repeat { Omega = -i dt (H_0 + H_1)/2; P_1 by the
 * commutator series dP^(k) = (1/k)(-i dt)[Hbar, dP^(k-1)] until
 * max|dP^(k)| <= dp_thrs (eq. commutator-expansion-ort); H_new = H[P_1] } until
 * max|H_new - H_1| <= h_thrs; then H_-1 <- H_0, H_0 <- H_1, P_0 <- P_1 and
 * record mu_q = Tr(P M_q) and E.  stats: host [n_steps][n_traj] or NULL.
 * Returns RT_ENOCONV if a cap is hit, or at once when a Hamiltonian update
 * is not finite (NaN / Inf; rt_last_error names the trajectory); the state
 * then stays at the last completed step.  RT_ESTATE once n_steps_max steps
 * have been taken.
 */
rt_status rt_step(rt_ctx* ctx, int n_steps, rt_step_stats* stats);

/*
 * Copies the history of trajectory traj, steps first_step .. first_step+count-1
 * (step 0 = just after the kick): mu_host [count][3] (dipole, mu_0 = 0) and
 * optionally energy_host [count] (E = Tr(Re P H_core) + E_H + E_x) and
 * trace_host [count] (Tr P).  Synchronises the stream.
 */
rt_status rt_dipole(rt_ctx* ctx, int traj, int first_step, int count, double* mu_host,
                    double* energy_host, double* trace_host);

/*
 * Matrix getters (synchronise the stream); out: host [N][N] double.
 * which: 0 = H_0, 1 = H_-1, 2 = Re P_0 (S'), 3 = Im P_0 (A'), 4 = H_core,
 * 5/6/7 = M_x/M_y/M_z, 8 = H_gs = H[P_gs] of the ground state (traj selects
 * the system through traj_sys for 4..8).
 */
rt_status rt_get_matrix(rt_ctx* ctx, int traj, int which, double* out);

/*
 * Overwrites the state of trajectory traj: P = S' + i A' (host [N][N] each),
 * H_0 and H_-1 (host [N][N]); NULL keeps the current value.  For checkpoint
 * restore and tests.  Non-finite entries give RT_EINVAL (nothing is copied).
 */
rt_status rt_set_state(rt_ctx* ctx, int traj, const double* p_re, const double* p_im,
                       const double* h0, const double* hm1);

/*
 * Autotuner of the launch shapes (the paper tunes nothing; these are this
 * library's own kernels).  Tunables per system:
 *   RT_TUNE_STENCIL_FP64 / _FP32: y-tile rows p1 (a divisor of ny whose tile has
 *     at most 1024 16-byte strips: one strip a thread up to 512, two above, and
 *     then only where each thread carries at most two of the 8 halo rows'
 *     strips), z chunks p2 (1..nz) and halo look-ahead
 *     p3 in {3, 4, 5, 6, 8} planes (how early the y-halo rows are requested) of
 *     the FD8 + V stencil; the tiling changes no arithmetic (results bitwise
 *     equal);
 *   RT_TUNE_PROJ_FP64: target block count p1 in {1024, 2048, 4096} of the FP64
 *     projection's K split (p2 reported: the resulting splits);
 *   RT_TUNE_PROJ_MIXED: splits p1 in {85, 128, 170, 255} of the BF16x3 projection
 *     for N <= 256 (p2 reported: the resulting splits).
 * p3 is 0 for the projections.
 * The projection splits change the order of the FP64/FP32 partial sums, so
 * results move within rounding (and a trajectory's results then depend on the
 * splits its context uses).  0 selects the built-in choice.
 * rt_autotune: for every system, each tunable it uses is timed over its
 *   candidates on the context's own buffers (device time by hipEvents on the
 *   context's stream, one warm-up and three timed launches each) and the fastest
 *   kept.  cache_path (nullable): a text file of earlier choices, one line
 *   "arch|kernel|nx x ny x nz|N|T p1 p2 p3" each; matching entries are applied
 *   without timing and new ones appended.  Call after rt_init, before rt_step;
 *   it overwrites scratch buffers only (state and history unchanged).
 * rt_tune_set / rt_tune_get: pin or read one tunable (RT_EINVAL for shapes the
 *   kernel cannot take).  rt_tune_report: the last rt_autotune's choices and
 *   timings as text, owned by the context.
 */
enum { RT_TUNE_STENCIL_FP64 = 0, RT_TUNE_STENCIL_FP32 = 1, RT_TUNE_PROJ_FP64 = 2, RT_TUNE_PROJ_MIXED = 3 };
rt_status rt_autotune(rt_ctx* ctx, const char* cache_path);
rt_status rt_tune_set(rt_ctx* ctx, int sys_index, int kernel, int p1, int p2, int p3);
rt_status rt_tune_get(rt_ctx* ctx, int sys_index, int kernel, int* p1, int* p2, int* p3);
const char* rt_tune_report(const rt_ctx* ctx);

/*
 * Checkpoint and resume of a whole context: the time loop of Algorithm 1 carries
 * from step j to j + 1 only P_j, the Hamiltonians H_j, H_j-1 (H_j-2 for the
 * quadratic first guess), the observable history and, with the learned first
 * guess, its feature rings, counters and fallback statistics; a checkpoint holds
 * exactly these, for every system and trajectory, in a host buffer the caller
 * owns.  rt_checkpoint_size: bytes needed now (grows with the step count).
 * rt_checkpoint_save: writes them (RT_ENOMEM if bytes is short; synchronises the
 * stream).  rt_checkpoint_load: into a context made by rt_init with the same
 * systems and run arguments (n_steps_max at least the saved step count); the
 * next rt_step continues exactly as the saving context would have (the same
 * arithmetic, so the same bits).  RT_EINVAL, with nothing changed, for a buffer
 * that is not a checkpoint of this library version, is truncated, or was saved
 * from a context of other shapes or modes.
 */
rt_status rt_checkpoint_size(rt_ctx* ctx, size_t* bytes);
rt_status rt_checkpoint_save(rt_ctx* ctx, void* host, size_t bytes);
rt_status rt_checkpoint_load(rt_ctx* ctx, const void* host, size_t bytes);

/*
 * Component entry points over caller-owned device buffers (for validation of
 * single stages; they run the same kernels as rt_step):
 *   rt_eval_h:    H_out = H[P] for the density matrix with real part p_re_dev
 *                 [N][N] (Algorithm 1, H_1 <- DFT(rho(P_1))), using the
 *                 context's hupdate/precision; also leaves rho, V_H, v_x of that
 *                 density in the system (rho/vh/vx getters below).
 *   rt_propagate: (p_re, p_im) <- U (p_re + i p_im) U^dagger with
 *                 U = exp(-i dt Hbar) by the commutator series
 *                 (eq. commutator-expansion-ort), thresholds dp_thrs/max_terms
 *                 of the run; *terms_out gets the number of terms (nullable).
 *   rt_get_grid:  copies the system's current grid field: 0 = rho, 1 = V_H,
 *                 2 = v_x, 3 = V_ion, 4 = V_loc (host [nz][ny][nx]).
 */
rt_status rt_eval_h(rt_ctx* ctx, int sys_index, const double* p_re_dev, double* h_out_dev);
rt_status rt_propagate(rt_ctx* ctx, int sys_index, const double* hbar_dev, double dt,
                       double* p_re_dev, double* p_im_dev, int* terms_out);
rt_status rt_get_grid(rt_ctx* ctx, int sys_index, int which, double* out_host);

/*
 * Phase timers.  rt_profile(ctx, enable, reset): from now on record a pair of
 * hipEvents around every launch of the tracked kernel classes on the context's
 * stream (enable != 0) or stop (0); reset != 0 zeroes the totals.  Synchronises.
 * rt_profile_read: accumulated device time in ms and launch count of one phase
 * (0 <= phase < 10); *name (nullable) gets its static name:
 * stencil_fd8, nonlocal, project_gemm, reduce_partials, density, poisson_dft,
 * lda_vloc, series_gemm, series_update, small_matrix.
 */
rt_status rt_profile(rt_ctx* ctx, int enable, int reset);
rt_status rt_profile_read(rt_ctx* ctx, int phase, double* total_ms, long* launches, const char** name);

/*
 * Learned predictor (the learned extension of Algorithm 1's first guess).
 * With fixed orbitals H is affine in the Hartree-exchange potential V, so the
 * linear extrapolation H_1 = 2 H_0 - H_-1 is the guess V = 2 V_j - V_(j-1) and
 * its error is D_j = V_(j+1) - 2 V_j + V_(j-1).  RT_PRED_MLP adds
 * h^3 Psi^T diag(P y) Psi to the linear guess, y = network(x_j) an estimate of
 * R D_j on a coarse 16^3 grid (R: block average, P: periodic trilinear
 * interpolation from cell centres).  x_j (8264 floats) = the 9 moments
 * (h^3 sum drho q_a, h^3 sum drho q_a q_b) of the density change drho = rho - rho_gs
 * at steps j-7..j (oldest first), then R drho_j, then R drho_(j-1).  The
 * self-consistent loop then runs as usual, so the fixed point is unchanged;
 * a trajectory falls back to the linear guess for good if its first residual
 * exceeds 10x the median first residual of its linear-guess steps.  Needs
 * grid edges divisible by 16; the first 8 steps use the linear guess.
 *
 * Network: tanh MLP n_in -> n_h -> n_h -> n_out on standardised data, FP32.
 * Packed floats: x_mean[n_in] x_scale[n_in] y_mean[n_out] y_scale[n_out]
 * W1[n_h][n_in] b1[n_h] W2[n_h][n_h] b2[n_h] W3[n_out][n_h] b3[n_out]
 * (x_std = (x - x_mean) x_scale, y = y_mean + y_std / y_scale).  The
 * trainable part starts at float offset 2 n_in + 2 n_out.
 *
 * rt_record: from the next step on, every step appends one training sample
 * per trajectory, x_(j-1) into X_dev [capacity][8264] and the realised
 * R D_(j-1) into Y_dev [capacity][4096] (device, caller-owned), until
 * capacity rows are written; rt_record_count returns the rows written.
 * The rt_mlp_* calls are context-free kernels on caller device buffers and
 * the given stream: forward (work: rt_mlp_work_floats), mean-square loss of
 * the standardised output (sum (y_std - t_std)^2 / (2 batch n_out)) with the
 * gradients of the trainable part in its layout, one Adam step (Kingma & Ba,
 * b1 0.9, b2 0.999, eps 1e-8, step t >= 1), and per-column mean and
 * 1/max(std, floor) of a [rows][cols] matrix.
 */
void rt_mlp_dims(int* n_in, int* n_h, int* n_out);
int64_t rt_mlp_n_params(int n_in, int n_h, int n_out);
int64_t rt_mlp_work_floats(int n_in, int n_h, int n_out, int batch);
rt_status rt_mlp_forward(void* hip_stream, int n_in, int n_h, int n_out, const float* params_dev,
                         const float* x_dev, float* y_dev, int batch, float* work_dev);
rt_status rt_mlp_loss_grad(void* hip_stream, int n_in, int n_h, int n_out, const float* params_dev,
                           const float* x_dev, const float* target_dev, int batch, float* grads_dev,
                           float* work_dev, float* loss_dev);
rt_status rt_mlp_adam(void* hip_stream, float* train_params_dev, const float* grads_dev, float* m_dev,
                      float* v_dev, int64_t n, int t, float lr);
rt_status rt_mlp_colstats(void* hip_stream, const float* x_dev, int rows, int cols, float* mean_dev,
                          float* scale_dev, float floor_std);
rt_status rt_record(rt_ctx* ctx, float* x_dev, float* y_dev, int capacity);
rt_status rt_record_count(rt_ctx* ctx, int* rows);

/*
 * Ground state on the GPU.  Algorithm 1 starts from the ground-state orbitals
 * and Hamiltonian of the system; this call computes them for a system described
 * as for rt_init: the self-consistent Kohn-Sham problem
 *   H[rho] psi_i = eps_i psi_i,  rho = sum_i f_i psi_i^2,
 * H[rho] = T + V_ion + V_nl + V_H[rho] + v_x[rho] (the operator of rt_apply_h;
 * spectral Hartree, LDA exchange), f_i as for rt_init (2 for the first n_occ).
 *
 * Method: Chebyshev-filtered subspace iteration (Zhou, Saad, Tiago and
 * Chelikowsky, J. Comput. Phys. 219, 172 (2006)) on a block of
 * nb = N + n_guard vectors, N = n_occ + n_virt.  A pass applies the scaled
 * degree-`degree` Chebyshev polynomial of H that damps [largest Ritz value,
 * upper bound of the spectrum], orthonormalises the block (Cholesky QR, twice)
 * and rotates it to the Ritz vectors of H on the block (Jacobi eigensolver of
 * rt_eigh).  The spectral bound is rigorous: kinetic symbol at the zone corner
 * + max|V_loc| + a block Gershgorin bound of V_nl.  Density loop: V_loc[rho_in]
 * -> filter passes until the wanted residuals are below
 * max(tol_res, min(1e-3, 0.01 err)) (at most max_passes) -> rho_out;
 * err = max|rho_out - rho_in|; stop when err < tol_rho, else Pulay (DIIS)
 * mixing of the last pulay_depth densities with residual weight mix.  The
 * final orbitals are the lowest N eigenvectors of H[rho_in] at the converged
 * rho_in, refined until max_i ||(H - eps_i) psi_i|| <= tol_res (norm
 * (h^3 sum |.|^2)^(1/2)), each signed so that its entry of largest modulus
 * (first one on ties) is positive.
 *
 * sys: as for rt_init except that psi0 holds nb = N + n_guard linearly
 *   independent start vectors [nb][nz][ny][nx] (host, or device with
 *   psi0_on_device), orthonormalize and nonorthogonal must be 0.
 * psi_out_dev: device [N][nz][ny][nx], h^3-orthonormal orbitals (caller-owned);
 *   pass it to rt_init as psi0 with psi0_on_device = 1.
 * eps_out_host: [nb] Ritz values in ascending order (nullable).
 * rho_out_dev: device [nz][ny][nx] density of the returned orbitals (nullable).
 * workspace_dev: at least rt_ground_state_workspace_size bytes, caller-owned;
 *   the call allocates no device memory.  All work is on hip_stream and the
 *   call synchronises it (the loop reads its convergence measures).
 * Errors: RT_EINVAL for arguments outside the ranges below (no side effects)
 *   or a start block with non-finite entries,
 *   RT_ENOMEM for a short workspace, RT_ENOCONV when max_scf or max_passes is
 *   exhausted or the block loses rank; rt_last_error(NULL) names the cause.
 *   When the density loop hits max_scf, stats (rho_err: the last
 *   max|rho_out - rho_in|) and eps_out_host still describe the last iterate,
 *   and psi_out_dev / rho_out_dev hold its orbitals and their density.
 */
typedef struct {
  int n_guard;        /* extra block vectors (>= 2; N + n_guard <= 1024)        */
  int degree;         /* Chebyshev filter degree (1..64)                         */
  int max_scf;        /* cap on density iterations (>= 1)                        */
  int max_passes;     /* cap on filter passes per potential (>= 1)               */
  double tol_rho;     /* max|rho_out - rho_in| that ends the density loop        */
  double tol_res;     /* final max_i ||(H - eps_i) psi_i||, i < N                */
  double mix;         /* Pulay residual weight, 0 < mix <= 1                      */
  int pulay_depth;    /* stored iterations, 1..8                                 */
} rt_gs_params;

typedef struct {
  int32_t scf_iters;      /* density iterations                                  */
  int32_t filter_passes;  /* filter + Rayleigh-Ritz passes                        */
  int64_t h_applies;      /* applications of H to the whole block                */
  int64_t eigensolves;    /* Rayleigh-Ritz eigensolves                            */
  int64_t jacobi_sweeps;  /* Jacobi sweeps summed over them                       */
  double rho_err;         /* max|rho(psi_out) - rho_in| at the end               */
  double residual;        /* max_i ||(H - eps_i) psi_i||, i < N                  */
} rt_gs_stats;

rt_status rt_ground_state_workspace_size(const rt_system* sys, const rt_gs_params* params, size_t* bytes);
rt_status rt_ground_state(const rt_system* sys, const rt_gs_params* params, void* workspace_dev,
                          size_t ws_bytes, void* hip_stream, double* psi_out_dev, double* eps_out_host,
                          double* rho_out_dev, rt_gs_stats* stats);

/*
 * Dense symmetric eigensolver (the Rayleigh-Ritz step above): the symmetric
 * part (A + A^T)/2 of a_dev [n][n] (device, row-major, 1 <= n <= 4096) is
 * diagonalised by parallel cyclic Jacobi sweeps (round-robin pair ordering;
 * Golub & Van Loan, Matrix Computations, Sec. 8.5) until the off-diagonal
 * Frobenius norm is below 1e-15 of the matrix norm (or stops shrinking below
 * 1e-13 of it).  evals_dev [n]: eigenvalues in ascending order (ties by
 * index); vecs_dev [n][n]: row k is the unit eigenvector of evals[k]; vecs_dev
 * may alias a_dev.  workspace_dev: rt_eigh_workspace_size bytes.  Synchronises
 * hip_stream.  sweeps_out: sweeps taken (nullable).  RT_EINVAL for bad
 * arguments or non-finite entries, RT_ENOCONV after 60 sweeps.
 */
rt_status rt_eigh_workspace_size(int n, size_t* bytes);
rt_status rt_eigh(void* hip_stream, int n, const double* a_dev, double* evals_dev, double* vecs_dev,
                  void* workspace_dev, size_t ws_bytes, int* sweeps_out);

/*
 * rt_eigh for callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * computation, arguments, results and errors as rt_eigh, without a workspace
 * argument.  Its work matrices live in one static device array per GPU
 * (~6.3 MB, 3 [n][n] FP64 matrices at n = RT_EIGH_NOALLOC_MAX_N, held until the
 * process ends); the call allocates nothing.  Limit: 1 <= n <=
 * RT_EIGH_NOALLOC_MAX_N, else RT_EINVAL with no side effects.  Every call on
 * one GPU uses that GPU's array, so calls that overlap on one GPU (other host
 * threads, other streams) race: the caller serialises them.  Synchronises
 * hip_stream (NULL = the current device's null stream).  RT_EDEVICE if the
 * array's device address cannot be obtained.
 */
#define RT_EIGH_NOALLOC_MAX_N 512
rt_status rt_eigh_noalloc(void* hip_stream, int n, const double* a_dev, double* evals_dev, double* vecs_dev,
                          int* sweeps_out);

/* Releases host-side state; the caller then frees the workspace. */
void rt_free(rt_ctx* ctx);

/* Message for the last failing call on ctx (or of rt_init when ctx is NULL). */
const char* rt_last_error(const rt_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RT_TDDFT_H */
