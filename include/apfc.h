/*
 * apfc.h -- C ABI of the MI355X (gfx950) solver for one time step of the amplitude
 * expansion of the phase-field crystal model (APFC), after Praetorius, Salvalaglio and
 * Voigt, "An efficient numerical framework for the amplitude expansion of the
 * phase-field crystal model".
 *
 * What is solved.  Complex amplitudes eta_j (j = 1..J) of the reciprocal lattice vectors
 * k_j evolve by the L2 gradient flow of the amplitude energy (Eq. (2)-(4)),
 *     d eta_j / dt = -kappa_j ( G_j^2 eta_j + dF^s/d eta_j^* ),  G_j = Lap + 2 i k_j.grad,
 * kappa_j = a0 |k_j|^2, with the bulk energy of Eq. (5) (triangular lattice: Eq. (6)-(7)).
 * Space: Q1 finite elements on a periodic uniform quad (2D) or hex (3D) mesh; the fourth
 * order operator is split with zeta_j = G_j eta_j (Eq. (8)-(9)).  Time: backward Euler with
 * the simplified Newton / amplitude-splitting iteration of Algorithm 1, i.e. per amplitude the
 * block system of Eq. (10)/(11)
 *     [ M          -G_j              ] [zeta_j]   [ 0                                  ]
 *     [ kappa_j G_j  M/dt + kappa_j w D ] [eta_j ] = [ M eta_j^{m-1}/dt - kappa_j w h_j    ]
 * with D = diag(dF), h_j = F^s_j - dF eta_j evaluated node by node (nodal quadrature weight
 * w = h^dim).  Each system is solved by restarted flexible GMRES, right-preconditioned with
 * the block preconditioner of Eq. (12) applied in its four steps (one mass solve, two
 * diffusion solves with L = M/sqrt(dt) + sqrt(kappa_j) K, a G and an M product).
 *
 * Memory and streams.  The library allocates no device memory.  Every device buffer
 * (amplitudes, workspace) is owned by the caller; pass a stream as a hipStream_t cast to
 * void* (NULL = the null stream).  A context is used from one host thread at a time.
 *
 * Layouts.  Node index i = ix + nx*(iy + ny*iz) (x fastest), node (ix,iy,iz) at
 * (ix*h, iy*h, iz*h), h = length[0]/n[0] (uniform: all directions share h).  A field of one
 * instance is stored planar as [J][2][N] doubles: amplitude j, then real part (0) or
 * imaginary part (1), then node.
 *
 * Errors.  Every entry point returns APFC_OK (0) on success, APFC_ERR_NOT_CONVERGED (1) when
 * FGMRES reached max_iters, or a negative APFC_ERR_*.  apfc_step and apfc_step_adjoint are
 * transactional: on any return other than APFC_OK the caller's output buffers are unchanged.
 * apfc_last_error() gives a message for the last failure on the calling thread.
 */
#ifndef APFC_H
#define APFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    APFC_OK = 0,
    APFC_ERR_NOT_CONVERGED = 1,   /* soft: FGMRES did not reach rtol within max_iters   */
    APFC_ERR_INVALID = -1,        /* bad argument (mesh, lattice, params, pointer)       */
    APFC_ERR_HIP = -2,            /* a HIP runtime call failed                           */
    APFC_ERR_WORKSPACE = -3,      /* workspace missing or smaller than apfc_workspace_bytes */
    APFC_ERR_NONFINITE = -4       /* a residual norm became NaN or Inf                   */
};

enum { APFC_TRI2D = 0, APFC_BCC3D = 1, APFC_CUSTOM = 2, APFC_FCC3D = 3 };
enum { APFC_FP64 = 0, APFC_MIXED = 1 };          /* preconditioner + Z basis precision */
enum { APFC_INNER_PCG = 0, APFC_INNER_CHEB = 1, APFC_INNER_MG = 2 }; /* inner solver of the preconditioner */
enum { APFC_MASS_ITER = 0, APFC_MASS_SEPARABLE = 1 };            /* step 1 of the preconditioner (mass_kind) */

/* Periodic uniform Q1 mesh: dim in {2,3}; n[d] nodes (= elements) per direction, n[d] >= 4;
 * length[d] = n[d] * h for one common h (checked to 1e-12 relative).  n[2], length[2] are
 * ignored in 2D. */
typedef struct {
    int dim;
    int64_t n[3];
    double length[3];
} apfc_mesh;

/* Reciprocal lattice vectors.  apfc_lattice_default fills k for APFC_TRI2D (Eq. (7), J = 3),
 * APFC_BCC3D (six unit <110>/sqrt(2) vectors, J = 6) and APFC_FCC3D (the FCC lattice that the paper's 3D
 * runs use, Sec. II after Eq. (7) and Sec. III: four <111>/sqrt(3) vectors summing to zero and three
 * <200>/sqrt(3) vectors, J = 7).  APFC_CUSTOM takes J <= 8 vectors as given; apfc_create rejects sets
 * whose resonant products are not all pair terms or terms with distinct amplitude indices. */
typedef struct {
    int kind;
    int J;
    double k[8][3];
} apfc_lattice;

typedef struct {
    double a0, a1, a2, a3;   /* energy parameters of Eq. (5); Elder: a0 = B^x, a1 = dB/2,
                                a2 = 3 nu / 4, a3 = tau (the cubic coefficient)          */
    int picard_iters;        /* K of Algorithm 1 (>= 1; the adjoint needs K = 1)         */
    double rtol;             /* stop when ||b - A x||_2 <= rtol ||b||_2 over (zeta, eta)  */
    int restart;             /* FGMRES restart length m, 1..32                           */
    int max_iters;           /* FGMRES iterations per solve before APFC_ERR_NOT_CONVERGED */
    int precision;           /* APFC_FP64 or APFC_MIXED                                 */
    int mass_iters;          /* inner iterations of the mass solve (paper: 3)            */
    int diff_iters;          /* inner iterations of each diffusion solve (paper: 5); with
                                APFC_INNER_MG the Chebyshev smoothing iterations before and
                                after each coarse-grid correction                         */
    int inner_kind;          /* APFC_INNER_PCG (paper: Jacobi-PCG), APFC_INNER_CHEB
                                (Chebyshev-Jacobi) or APFC_INNER_MG (the paper's multigrid
                                variant of Sec. III: one V-cycle per diffusion solve, a
                                geometric hierarchy of meshes of 2, 4, ... times the mesh
                                size while every direction of every instance halves to at
                                least 16 (2D) / 8 (3D) nodes, Chebyshev-Jacobi smoothing on
                                the upper quarter of the spectrum, transposed Q1
                                interpolation, the coarsest level (at most 8192 nodes per
                                instance, else APFC_ERR_INVALID) by 24 Chebyshev
                                iterations; the mass solve as APFC_INNER_CHEB)             */
    int x0_order;            /* FGMRES initial guess of the first Picard solve of a step:
                                0 = the state passed in (default); 1 / 2 / 3 = linear /
                                quadratic / cubic extrapolation in time from the states
                                passed to the last x0_order steps of this context (fewer
                                iterations; the stop test is unchanged).  Assumes that
                                consecutive apfc_step calls continue one trajectory per
                                instance with one dt; see apfc_reset_history.             */
    int mass_kind;           /* step 1 of P^{-1} (Sec. II.B, the mass solve M x1 = beta1):
                                APFC_MASS_ITER (default) = mass_iters iterations of the
                                inner solver; APFC_MASS_SEPARABLE = one application of the
                                separable approximate inverse of M: on the uniform periodic
                                mesh M is the Kronecker product of 1D mass matrices
                                (h/6) tridiag(1, 4, 1), whose inverse has the entries
                                (sqrt(3)/h) rho^|k|, rho = sqrt(3) - 2; kept for |k| <=
                                mass_iters (1..4) per direction, so the defect M W - I is
                                below (1 + 0.73 |rho|^R)^dim - 1 in the max norm (0.03 in
                                2D and 0.04 in 3D at R = 3, against 0.06 and 0.28 for five
                                Chebyshev iterations)                                     */
} apfc_params;

/* Device pointers of one instance, each [J][2][N] float64, owned by the caller. */
typedef struct {
    double* eta;
    double* zeta;
} apfc_state;

typedef struct {
    int total_iters;      /* FGMRES iterations summed over all systems (instance, amplitude) */
    int max_iters;        /* largest per-system iteration count                              */
    int cycles;           /* restart cycles of the slowest system                            */
    double max_relres;    /* largest final true relative residual ||b-Ax||/||b||             */
    double ms;            /* host wall time of the call in milliseconds                      */
    int* iters;           /* optional host array [count*J]: iterations per system, or NULL   */
} apfc_stats;

typedef struct apfc_ctx apfc_ctx;

/* Fill params with the paper's values (a0..a3 of Sec. II, 3 and 5 inner PCG iterations of
 * Sec. III) and solver defaults (K = 1, rtol 1e-8, restart 30, max_iters 500, FP64). */
void apfc_params_default(apfc_params* params);

/* Fill lattice for kind APFC_TRI2D, APFC_BCC3D or APFC_FCC3D. Returns APFC_ERR_INVALID for other kinds. */
int apfc_lattice_default(int kind, apfc_lattice* lattice);

/* Relaxed amplitude phi of the uniform crystal eta_j = phi (positive root of d f^s / d phi = 0
 * for the bulk energy of Eq. (5) on this lattice; 0 if only the liquid exists). Host only. */
int apfc_uniform_amplitude(const apfc_lattice* lattice, const apfc_params* params, double* phi);

/* Relaxed real amplitudes phi[J] (host array) of the uniform crystal of the bulk energy of Eq. (5) on this
 * lattice, one value per shell of equal |k_j| (the amplitudes of a shell are equivalent): for one shell
 * (APFC_TRI2D, APFC_BCC3D) the value of apfc_uniform_amplitude; for several (APFC_FCC3D: <111> and
 * <200>) the stationary point of f^s over the shell values found by Newton's method from that value.
 * All zero when only the liquid exists; APFC_ERR_INVALID if the iteration leaves phi > 0.  Host only. */
int apfc_equilibrium_amplitudes(const apfc_lattice* lattice, const apfc_params* params, double* phi);

/* One instance of the problem of Sec. II: amplitudes eta_j of the lattice's reciprocal vectors k_j
 * (Eq. (1); triangular set of Eq. (7)) on a rectangular (2D) or box (3D) domain, here periodic,
 * evolving by Eq. (3)-(4) with the bulk energy of Eq. (5) and its parameters a0..a3; the mesh
 * stands for the finest level of the adaptive mesh of Sec. II.A.  mesh, lattice and params are read
 * once (host memory, caller-owned, not kept); *out receives a context owned by the caller
 * (apfc_destroy).  Validates the arguments (APFC_ERR_INVALID with apfc_last_error() set: non-uniform
 * h, n[d] < 4, |k_j| = 0, resonant products the kernels do not cover, out-of-range solver fields) and
 * builds the host-side tables; no device work happens before apfc_set_workspace. */
int apfc_create(const apfc_mesh* mesh, const apfc_lattice* lattice, const apfc_params* params,
                apfc_ctx** out);

/* count (1..4096) independent instances of the problem of Sec. II (as apfc_create), of possibly
 * different mesh sizes and energy parameters a0..a3 (meshes[count], params[count], host arrays read
 * once; one lattice and one dimension for all; solver fields taken from params[0] and required
 * equal, else APFC_ERR_INVALID), all solved together by the same batched launches.  Instance b's
 * amplitude j is system b*J + j of the batch (the order of apfc_stats.iters). */
int apfc_create_batch(int count, const apfc_mesh* meshes, const apfc_lattice* lattice,
                      const apfc_params* params, apfc_ctx** out);

/* Bytes of device workspace the context needs (256-byte aligned start required). */
size_t apfc_workspace_bytes(const apfc_ctx* ctx);

/* Attach caller-owned device memory of at least apfc_workspace_bytes bytes. The memory must
 * stay valid until the context is destroyed or another workspace is attached. */
int apfc_set_workspace(apfc_ctx* ctx, void* device_ptr, size_t bytes);

/* zeta_j = M^{-1} G_j eta_j for every instance (the initial auxiliary field of Algorithm 1),
 * computed by 60 (2D) / 100 (3D) Chebyshev-Jacobi iterations with the exact spectral bounds of the
 * Jacobi-scaled mass matrix (error below 1e-15 relative). states[count]. */
int apfc_init_zeta(apfc_ctx* ctx, apfc_state* states, void* stream);

/* One time step of Algorithm 1 for every instance: eta, zeta <- eta^m, zeta^m.  source is
 * NULL or a device array per instance ([count] pointers to [J][2][N]) of a manufactured
 * source s added to d eta/dt (enters the RHS as M s).  stats may be NULL.
 * With params.x0_order > 0 the step keeps the states it was given (x0_order device copies of
 * the state, in the workspace) to extrapolate the initial guess of the next steps; a step
 * with another dt than the last, or one that fails, restarts that history. */
int apfc_step(apfc_ctx* ctx, apfc_state* states, double dt, const double* const* source,
              void* stream, apfc_stats* stats);

/* nsteps >= 1 time steps with one dt: the same arithmetic as nsteps calls of apfc_step, but the state
 * stays in the library's layout between the steps (converted from and to the caller's planar
 * arrays once) and no statistics are copied to the host between the steps.  source as in
 * apfc_step (the same for every step).  The caller's state is written only when every step
 * succeeds; otherwise it is unchanged and the first failing step's code is returned.
 * stats (may be NULL): total_iters and iters[] summed over the steps, max_iters, cycles and
 * max_relres the largest of any step.  step_max_iters (host, [nsteps], may be NULL): the largest
 * per-system iteration count of each step (entries after a failing step are not written). */
int apfc_run(apfc_ctx* ctx, apfc_state* states, double dt, int nsteps, const double* const* source,
             void* stream, apfc_stats* stats, int* step_max_iters);

/* Forget the states kept for params.x0_order > 0: the next apfc_step starts a new trajectory
 * (its initial guess is the state passed in).  apfc_init_zeta and apfc_set_workspace do the
 * same.  No effect with x0_order = 0. */
int apfc_reset_history(apfc_ctx* ctx);

/* Energy E = sum_i w f^s(eta_i) + sum_j zeta_j^H M zeta_j with zeta_j = M^{-1} G_j eta_j
 * (Eq. (2) without the 1/2, nodal quadrature of f^s), per instance into host_out[count].
 * The state's zeta is not read: zeta is recomputed by the same mass solve as apfc_init_zeta. */
int apfc_energy(apfc_ctx* ctx, const apfc_state* states, double* host_out, void* stream);

/* Gradient of apfc_energy with respect to eta in PyTorch's convention
 * (dE/dRe eta + i dE/dIm eta = 2 dE/d eta^*), written to grad[count] device arrays
 * [J][2][N]; dE/d(Delta B) at fixed eta is added to host ddB[count] if ddB != NULL. */
int apfc_energy_grad(apfc_ctx* ctx, const apfc_state* states, double* const* grad,
                     double* ddB, void* stream);

/* Adjoint of one K = 1 step taken with the same dt from before[].eta to after[].eta: given
 * lam_after = dL/d eta^m (PyTorch convention, device [J][2][N] per instance), write
 * lam_before = dL/d eta^{m-1} and add dL/d(Delta B) of this step to host dL_ddB[count].
 * Solves A_j^H mu = [0; lam_j] as Sigma A_j^{-1} Sigma^{-1} with Sigma = diag(-kappa_j, 1),
 * reusing the forward FGMRES and preconditioner.  zeta carries no gradient. */
int apfc_step_adjoint(apfc_ctx* ctx, const apfc_state* before, const apfc_state* after, double dt,
                      const double* const* lam_after, double* const* lam_before, double* dL_ddB,
                      void* stream, apfc_stats* stats);

/* Apply one operator of the step to every instance: out_j = A_j in_j (which = APFC_OP_A, the
 * block matrix of Eq. (11) linearised at lin[].eta with step dt) or out_j = P_j^{-1} in_j
 * (which = APFC_OP_PINV, the block preconditioner of Eq. (12) by its four steps with the context's
 * inner solver and precision).  in/out hold (zeta, eta) pairs as [J][2][N] device arrays; lin is
 * read only for APFC_OP_A.  For testing and for callers that drive their own Krylov method. */
enum { APFC_OP_A = 0, APFC_OP_PINV = 1 };
int apfc_apply(apfc_ctx* ctx, int which, const apfc_state* lin, const apfc_state* in, apfc_state* out,
               double dt, void* stream);

/* Parameters of the refinement indicator of Sec. II.C (Eq. (16)-(17)). */
typedef struct {
    double n_per_wavelength;  /* n: h_amp = min_j lambda_j(theta) / n (the paper uses n >= 10)   */
    double grad_A_eps;        /* epsilon: h = h_int where |grad A| >= epsilon                    */
    double A_min;             /* a node is solid ("A > 0") where A > A_min                        */
    double h_int, h_max;      /* finest and coarsest mesh size                                    */
    double tiny;              /* amplitudes with |eta_j|^2 <= tiny carry no phase                 */
} apfc_refine_params;

/* Local lattice rotation and target mesh size at every node (a post-step analysis; Eq. (14)-(17)).
 * omega_ab = (du_a/dx_b - du_b/dx_a)/2 where k_j . u = arg eta_j (Eq. (14)-(15)); the phase gradients
 * are Im(conj(eta_j) grad eta_j)/|eta_j|^2 with central differences, and du/dx_b is the least-squares
 * solution over the amplitudes with |eta_j|^2 > tiny (omega = 0 where fewer than dim remain).
 * omega[count]: device arrays of N doubles (2D: omega_12) or [3][N] (3D: omega_23, omega_31,
 * omega_12).  h[count] (may be NULL): device arrays of N doubles with
 *   h = h_int if |grad A| >= eps;  min(max(h_amp, h_int), h_max) if A > A_min;  h_max otherwise,
 * h_amp = min_j 2 pi / (2 |k_j| sin(theta/2)) / n, theta = asin(max_d |omega_d|) (Eq. (16)-(17)). */
int apfc_rotation(apfc_ctx* ctx, const apfc_state* states, double* const* omega, double* const* h,
                  const apfc_refine_params* params, void* stream);

/* Kernel timing probe: when enabled, every `every`-th launch (every >= 1) of the kernel named
 * `name` inside apfc_step is bracketed by HIP events on the launch stream (an event pair adds
 * a few microseconds of stream idle, hence the sampling); apfc_probe_read returns the number of
 * recorded launches, their summed duration and their mean algorithmic bytes since the last
 * reset, each launch's bytes counting only the systems it worked on (converged systems of a
 * batch are skipped and move nothing); launches in which every system was masked (a cycle queued
 * past convergence) are left out of all three.  name = NULL disables the probe. */
int apfc_probe_enable(apfc_ctx* ctx, const char* name, int every);
int apfc_probe_read(apfc_ctx* ctx, int* launches, double* total_ms, double* bytes_per_launch);

/* name = "all" in apfc_probe_enable samples every kernel family at once, each on its own count (every
 * every-th launch of each).  apfc_probe_read_kernel gives one family's figures from the records kept
 * since the last apfc_probe_read (it does not reset them): sampled working launches, their summed
 * duration, their mean algorithmic bytes (0 for families without a byte model: xupdate, gs's first
 * pass, the small kernels) and, in issued, every launch of the family so far, sampled or not.  Family
 * names: "cheb" (fused and per-iteration Chebyshev preconditioner stages; stages 0 and 1 of the fused 2D
 * preconditioner also form the next basis vector), "apply" (operator apply with
 * the first Gram-Schmidt pass), "residual", "proj_final" (the basis vector where the preconditioner does
 * not form it), "xupdate", "gs", "extrapolate", "rhs",
 * "mass" (the separable mass inverse on bricks), "mg" (multigrid V-cycle kernels), "pcg_spmv",
 * "pcg_update", "pcg_init", "pc_final", "reduce", "small", "other". */
int apfc_probe_read_kernel(apfc_ctx* ctx, const char* name, int* launches, double* total_ms,
                           double* bytes_per_launch, long long* issued);

/* Tile-height autotuner: times the stencil kernels for each candidate tile on the attached
 * workspace and keeps the fastest.  Optional; the default tile is used otherwise. */
int apfc_autotune(apfc_ctx* ctx, void* stream, int* chosen_tile_rows);

/* Set the tiling by hand instead of apfc_autotune: tile_rows in {4, 8, 16, 32} (rows of the 64-wide
 * stencil tiles) and precond_region in 0..5 (LDS region of the fused 2D Chebyshev preconditioner, nodes x
 * rows / threads: 0: 128x32 / 512, 1: 64x32 / 256, 2: 64x64 / 512, 3: 128x36 / 512, 4: 128x64 / 1024,
 * 5: 256x32 / 1024; a Chebyshev stage keeps two LDS copies of its region in FP32 and one in FP64, the
 * separable mass stage one; taller regions recompute less halo, smaller ones leave room for more
 * workgroups per CU).  Needs the workspace.  The 3D bricks of the separable mass inverse and of the
 * Chebyshev L solves (64 x 8 nodes per plane, 8 or 16 planes) are chosen at creation, not here. */
int apfc_set_tiles(apfc_ctx* ctx, int tile_rows, int precond_region);
int apfc_get_tiles(const apfc_ctx* ctx, int* tile_rows, int* precond_region);

/* Use hipGraph replays of whole restart cycles (1) or direct launches (0, default). */
int apfc_set_graphs(apfc_ctx* ctx, int enable);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): apfc_step with the same arguments, results and errors, but run on
 * a static device array of the library instead of the caller's workspace.  The context needs no
 * apfc_set_workspace; its apfc_workspace_bytes must not exceed apfc_noalloc_max_bytes() (64 MiB, e.g.
 * one 192^2 triangular instance in mixed precision with restart 4 and x0_order 3), else
 * APFC_ERR_WORKSPACE and nothing runs.  The call makes no hipMalloc, hipFree or hipHostMalloc and no
 * allocation on the host: pointer tables and statistics go through host arrays sized at create, and
 * the end of each restart cycle is read back with a small synchronous copy.  Graphs (apfc_set_graphs)
 * and the timing probe are not used.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents: a context lays out its tables there again when another context used it since
 * its own last call (its extrapolation history then restarts), a following call of another entry point
 * moves the context back onto its own workspace (history restarts), and calls that overlap in time on
 * one GPU race.  Each GPU keeps its copy of the array until the process ends. */
int apfc_step_noalloc(apfc_ctx* ctx, apfc_state* states, double dt, const double* const* source,
                      void* stream, apfc_stats* stats);
size_t apfc_noalloc_max_bytes(void);

int apfc_destroy(apfc_ctx* ctx);
const char* apfc_status_string(int status);
const char* apfc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* APFC_H */
