/*
 * dnb.h -- C ABI of the differentiable direct N-body library (libdnb.so).
 *
 * The library implements, for one AMD Instinct MI355X (gfx950), the hot path of
 * the differentiable direct N-body method of arXiv 2511.22468 ("Odisseo"):
 * the softened pairwise gravity sum (Sec. 1, "N-body codes": direct pairwise
 * forces with softening, no tree), the analytic NFW-halo and Miyamoto-Nagai-disk
 * accelerations of the host galaxy (Sec. 2.2.1), the fixed-step Velocity-Verlet
 * (kick-drift-kick) integrator (Sec. 2.2.1), reverse-mode gradients of the final
 * state with respect to initial conditions, integration time, particle masses and
 * potential parameters (Sec. 2), the maximum mean discrepancy loss with its
 * gradient (Sec. 2.2.1 and Fig. 2, step 4), and the back-integration of the
 * progenitor's centre of mass and the Plummer-sphere placement that the inference
 * pipeline chains them with (Fig. 2, steps 2-3).
 *
 * Units: every entry point takes internal units, kpc for length, km/s for
 * velocity, Msun for mass, kpc/(km/s) for time; G is passed in dnb_pot.
 *
 * Conventions shared by every entry point:
 *  - Arrays are DEVICE pointers on the current HIP device unless a comment says
 *    "host".  Particle arrays are structure-of-arrays: an array of "[3][n]"
 *    holds n x-values, then n y-values, then n z-values, contiguous; "[n]" is
 *    one value per particle.  All arrays are FP64 and owned by the caller.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL means the
 *    null stream).  Outputs are valid once the stream has been synchronised.
 *    Inputs must stay alive and unmodified until then.
 *  - Arguments are validated on the host before anything is enqueued; a failed
 *    check returns DNB_ERR_ARG and enqueues nothing.  A HIP failure returns
 *    DNB_ERR_HIP.  dnb_last_error() gives a message for the calling thread.
 *    No C++ exception crosses this interface.
 *  - A context may be used by one host thread and one stream at a time.
 *    Contexts on the same device may run concurrently on different streams.
 *  - eps > 0 is required when two distinct particles may coincide; with
 *    eps == 0 the self term is masked, and coincident distinct particles give
 *    inf/NaN accelerations.
 */
#ifndef DNB_H
#define DNB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DNB_OK = 0,
    DNB_ERR_ARG = -1,    /* invalid argument, nothing enqueued */
    DNB_ERR_HIP = -2,    /* a HIP runtime call failed */
    DNB_ERR_NOMEM = -3,  /* device allocation of the context failed */
    DNB_ERR_STATE = -4   /* call sequence or buffer-size violation */
} dnb_status;

/* Precision of the pairwise terms.  Positions, velocities, the drift, the
 * external potential and every reduction are FP64 in both modes.
 *  DNB_FP64  : pair terms in FP64 (reciprocal square root refined by Newton
 *              steps).
 *  DNB_FP32C : pair terms in FP32 on positions staged relative to a per-step
 *              centre computed in FP64, with compensated (TwoSum) accumulation
 *              across tiles of 128 sources and an FP64 sum across slices. */
typedef enum { DNB_FP64 = 0, DNB_FP32C = 1 } dnb_prec;

/* Softening and host potential (Sec. 1 and Sec. 2.2.1).  A zero mass disables
 * that component.  NFW:  Phi = -G m_nfw ln(1 + r/rs_nfw) / r, m_nfw being the
 * scale mass 4 pi rho0 rs^3.  Miyamoto-Nagai:  Phi = -G m_mn /
 * sqrt(R^2 + (a_mn + sqrt(z^2 + b_mn^2))^2).  Pair softening is Plummer:
 * a_i = G sum_j m_j d_ij (|d_ij|^2 + eps^2)^(-3/2), d_ij = x_j - x_i. */
typedef struct {
    double G, eps, m_nfw, rs_nfw, m_mn, a_mn, b_mn;
} dnb_pot;

typedef struct dnb_ctx dnb_ctx;

/* Create a context for up to max_n particles on the current HIP device.  All
 * device workspace (staging, slice partials, reduction scratch) is allocated
 * here, once; no other entry point allocates.  Returns DNB_ERR_ARG for
 * max_n < 1 or max_n > 2^26, DNB_ERR_NOMEM if allocation fails. */
dnb_status dnb_create(dnb_ctx** out, int64_t max_n, dnb_prec prec);

/* Free a context (NULL is ignored).  Synchronises the device first. */
void dnb_destroy(dnb_ctx* ctx);

/* Message of the last failed call on this host thread ("" if none). */
const char* dnb_last_error(void);

/* Library version string. */
const char* dnb_version(void);

/* Accelerations a = a_int + with_ext * a_ext at positions pos (Sec. 1, Sec.
 * 2.2.1).  pos [3][n], mass [n], acc [3][n] (output, must not alias pos).
 * pot is a HOST pointer read during the call. */
dnb_status dnb_accelerations(dnb_ctx* ctx, int64_t n, const double* pos, const double* mass,
                             const dnb_pot* pot, int with_ext, double* acc, void* stream);

/* Largest n that dnb_accelerations_noalloc accepts. */
#define DNB_NOALLOC_MAX_N 65536

/* For callers that cannot allocate device memory: code under HIP stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The accelerations of
 * dnb_accelerations (same arguments, with the pair-term precision given here
 * instead of by a context), computed without a context and without allocating:
 * the kernels' scratch (staged sources, slice partials, block records) is one
 * 16 MiB array of device memory that the library's code object holds on every
 * GPU it runs on, until the process ends.  n must lie in [1, DNB_NOALLOC_MAX_N]
 * (DNB_ERR_ARG otherwise, with a message).  No hipMalloc, hipFree or other
 * allocating call is made (the array's device address is looked up once per
 * device, on the first call there).  The source slices are capped so that the
 * partials fit the array (9 slices at n = 65536 against 32 for the context
 * path), so FP32C results equal dnb_accelerations' to FP32 rounding rather than
 * bit for bit; FP64 results agree to FP64 rounding.  Every call on one GPU uses
 * the same array: calls that overlap on a device (other streams or threads)
 * race, and the caller must serialise them.  pos [3][n], mass [n], acc [3][n]
 * device pointers (acc must not alias pos); pot is a HOST pointer. */
dnb_status dnb_accelerations_noalloc(int64_t n, const double* pos, const double* mass,
                                     const dnb_pot* pot, int with_ext, dnb_prec prec,
                                     double* acc, void* stream);

/* Accelerations of the targets i_begin .. i_begin + i_count - 1 only, each summed
 * over all n sources (the rectangular block one device computes when the targets
 * are split over several devices, Sec. 2 and Fig. 1).  pos [3][n] and mass [n]
 * hold the whole system; acc [3][i_count] (device, must not alias pos) receives
 * row r = target i_begin + r, with the arithmetic of dnb_accelerations (equal
 * to it bit for bit when both split the sources into the same slices).  Requires
 * 0 <= i_begin and 1 <= i_count <= n - i_begin (DNB_ERR_ARG otherwise). */
dnb_status dnb_accelerations_rows(dnb_ctx* ctx, int64_t n, const double* pos, const double* mass,
                                  const dnb_pot* pot, int with_ext, int64_t i_begin,
                                  int64_t i_count, double* acc, void* stream);

/* Vector-Jacobian product of dnb_accelerations (the derivatives the paper's
 * gradients with respect to initial conditions and particle masses are built
 * from, Sec. 2), for the rows i_begin .. i_begin + i_count - 1.  With w [3][n]
 * (device) the cotangent of the accelerations of all n particles, row r of
 * gpos [3][i_count] receives d(sum_j w_j . a_j)/dx_k and gmass [i_count]
 * (nullable) d(sum_j w_j . a_j)/dm_k, for k = i_begin + r; the external field
 * enters gpos through its Hessian when with_ext is nonzero.  pos [3][n] and
 * mass [n] hold the whole system.  The pair part runs in the precision of the
 * context (FP32C: the cotangent is staged with a power-of-two scale, undone in
 * FP64).  Outputs must not alias inputs; 0 <= i_begin and 1 <= i_count <=
 * n - i_begin (DNB_ERR_ARG otherwise). */
dnb_status dnb_accelerations_vjp(dnb_ctx* ctx, int64_t n, const double* pos, const double* mass,
                                 const dnb_pot* pot, int with_ext, const double* w,
                                 int64_t i_begin, int64_t i_count, double* gpos, double* gmass,
                                 void* stream);

/* One kick-drift-kick step of size dt (Sec. 2.2.1, Velocity-Verlet), in place on
 * pos [3][n] and vel [3][n]; the step evaluates a(x_n) and a(x_{n+1}). */
dnb_status dnb_step(dnb_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                    const dnb_pot* pot, double dt, void* stream);

/* Number of doubles of the checkpoint tape that dnb_simulate writes for
 * (n, n_steps, ckpt_every): for each of the ceil(n_steps / ckpt_every)
 * checkpoints the state (6n), two FP32C staging centres (8: those of the
 * checkpoint's positions and of the positions one step later) and the internal
 * (pair) acceleration (3n), plus the internal acceleration at the final
 * positions (3n); 0 for n_steps = 0. */
int64_t dnb_tape_doubles(int64_t n, int64_t n_steps, int64_t ckpt_every);

/* Number of doubles of the segment workspace that dnb_simulate_vjp needs:
 * 16n for ckpt_every = 1; otherwise 16n + 2 (6n ckpt_every + 3n), room for two
 * recomputed checkpoint segments (the next one is recomputed while the sweep
 * reads the current one); -1 for invalid or oversized arguments. */
int64_t dnb_vjp_workspace_doubles(int64_t n, int64_t ckpt_every);

/* n_steps kick-drift-kick steps of size dt (Sec. 2.2.1: fixed steps), in place
 * on pos [3][n] and vel [3][n].  If tape is not NULL it must hold
 * dnb_tape_doubles(n, n_steps, ckpt_every) doubles and receives the state
 * (x, v) at steps 0, K, 2K, ... (K = ckpt_every >= 1), each as [6][n]
 * (x block then v block), and the quantities the reverse sweep reuses (see
 * dnb_tape_doubles).  The tape is what dnb_simulate_vjp differentiates. */
dnb_status dnb_simulate(dnb_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                        const dnb_pot* pot, double dt, int64_t n_steps, int64_t ckpt_every,
                        double* tape, void* stream);

/* Debug scan of a state for values no integration can start from (NaN or
 * infinite): *first_bad (host) receives the smallest particle index i whose
 * position pos [3][n], velocity vel [3][n] or mass mass [n] holds one, or -1
 * when every value is finite.  vel and mass may be NULL (not scanned).  Waits
 * for the stream: a debugging aid, not for the hot loop. */
dnb_status dnb_check_state(dnb_ctx* ctx, int64_t n, const double* pos, const double* vel,
                           const double* mass, int64_t* first_bad, void* stream);

/* With on != 0, dnb_simulate, dnb_simulate_resume and dnb_simulate_batch first
 * scan their initial state as dnb_check_state does (every member of a batch)
 * and return DNB_ERR_ARG, naming the first non-finite particle, before any step
 * runs; each such call then waits for its stream.  Off (0) by default. */
dnb_status dnb_set_checks(dnb_ctx* ctx, int on);

/* Restart of a long forward run from one of its checkpoints (the fixed-step
 * integration of Sec. 2.2.1 is a deterministic map of the state, so a run may
 * be continued from any stored state).  tape is a tape that dnb_simulate (or
 * this call) wrote for (n, tape_steps, tape_ckpt_every) and is only read; ckpt
 * is one of its checkpoints, 0 <= ckpt < ceil(tape_steps / tape_ckpt_every),
 * the state at step ckpt * tape_ckpt_every.  pos [3][n] and vel [3][n] receive
 * that state and are then integrated n_steps >= 0 further with mass, pot and
 * dt: with the source run's mass, pot and dt the result is bit for bit the
 * state the uninterrupted run reached after as many steps (in FP32C the run
 * stages the checkpoint's positions, and the positions one step later, with
 * the two centres the tape stored for them rather than with fresh ones).
 * tape_out (nullable) receives the continuation's own tape, as dnb_simulate
 * writes it for (n, n_steps, ckpt_every), which dnb_simulate_vjp then
 * differentiates.  pos, vel and tape_out must not overlap the source tape or
 * each other; DNB_ERR_ARG for a checkpoint outside the tape, DNB_ERR_STATE when
 * a buffer is smaller than its stated size. */
dnb_status dnb_simulate_resume(dnb_ctx* ctx, int64_t n, const double* tape, int64_t tape_steps,
                               int64_t tape_ckpt_every, int64_t ckpt, double* pos, double* vel,
                               const double* mass, const dnb_pot* pot, double dt,
                               int64_t n_steps, int64_t ckpt_every, double* tape_out,
                               void* stream);

/* Reverse-mode gradient of a scalar loss through dnb_simulate (Sec. 2: the final
 * state is differentiable with respect to initial conditions, integration time,
 * particle masses and external-potential parameters).  This is the exact
 * discrete adjoint of the kick-drift-kick map: positions between checkpoints
 * are recomputed forward from the tape (bitwise identical to the forward run),
 * then the sweep runs newest step first with one pair-VJP per step.
 *
 * Inputs: the same n, mass, pot, dt, n_steps, ckpt_every and tape as the
 * forward call; pos_T [3][n], the final positions the forward call produced
 * (the position array that call moved in place); gpos_T, gvel_T [3][n], the
 * loss cotangents of the final state (gvel_T may be NULL for zero).  workspace
 * holds dnb_vjp_workspace_doubles(n, ckpt_every).  Outputs: gpos_0, gvel_0
 * [3][n]; gmass [n] (nullable): dL/dm_k; gparams [7] (device): dL/dm_nfw,
 * dL/dm_mn, dL/ddt, sum_k m_k dL/dm_k (the derivative with respect to a
 * common log-scale of all particle masses, which is what a progenitor-mass
 * parameter needs), then the derivatives with respect to the host's shape
 * parameters dL/drs_nfw, dL/da_mn and dL/db_mn (Sec. 2.2.2 fits the halo's scale
 * radius and the disk's scale lengths with the masses; where b_mn = 0 and
 * z = 0 the disk's derivatives in z are taken as 0, as its z-acceleration is).
 * Outputs must not alias inputs.
 *
 * Call sequence: the context records each tape that dnb_simulate writes (its
 * address, the position and mass arrays, n, n_steps, ckpt_every, dt and pot;
 * the 16 most recent).  With n_steps > 0 this call returns DNB_ERR_STATE,
 * enqueueing nothing, unless tape is such a record and every one of those
 * arguments matches it.  A later dnb_simulate, dnb_step or dnb_place_plummer
 * on this context that writes the recorded position array, or a dnb_simulate
 * that writes a tape over the recorded one, retires the record (the library
 * cannot see writes made by other code).  DNB_ERR_STATE is also returned when
 * the allocation holding workspace or tape ends before the length these
 * arguments need (checked through the HIP runtime's allocation ranges). */
dnb_status dnb_simulate_vjp(dnb_ctx* ctx, int64_t n, const double* mass, const dnb_pot* pot,
                            double dt, int64_t n_steps, int64_t ckpt_every, const double* tape,
                            const double* pos_T, const double* gpos_T, const double* gvel_T,
                            double* workspace, double* gpos_0, double* gvel_0, double* gmass,
                            double* gparams, void* stream);

/* Number of doubles of the workspace that dnb_simulate_vjp_reversed needs:
 * 17n whatever the checkpoint spacing; -1 for invalid or oversized n. */
int64_t dnb_vjp_reversed_workspace_doubles(int64_t n);

/* The same gradient as dnb_simulate_vjp, with the trajectory between
 * checkpoints rebuilt by stepping it backward instead of recomputing it forward
 * (the kick-drift-kick step is time-reversible, Sec. 2.2.1: its step with -dt
 * undoes it up to rounding).  The sweep starts from the final state and, newest
 * step first, runs one pair launch at x_m that sums the pair VJP and the
 * internal acceleration a(x_m) together; the reverse kick takes the adjoint step
 * and undoes the forward step that led to x_m.  At every checkpoint the stored
 * state replaces the rebuilt one.  One pair launch per step instead of two,
 * and a workspace of 17n doubles instead of two recomputed segments.
 *
 * Accuracy: the rebuilt positions differ from the run's by the rounding of at
 * most ckpt_every backward steps, grown by the dynamics over those steps, and
 * in FP32C mode also by the FP32 rounding of accelerations staged about a
 * different centre than the run's.  With ckpt_every = 1 no state is rebuilt:
 * in FP64 mode the result is then that of dnb_simulate_vjp bit for bit.  Where
 * the dynamics are chaotic over ckpt_every steps the gradient is that of a
 * neighbouring trajectory; choose ckpt_every accordingly.
 *
 * Arguments as dnb_simulate_vjp, plus vel_T [3][n]: the final velocities, the
 * velocity array the forward call moved in place (DNB_ERR_STATE when it is not
 * the array recorded with the tape, or when a later dnb_simulate, dnb_step or
 * dnb_place_plummer on this context wrote that array; dnb_simulate_vjp, which
 * does not read it, still accepts the tape then).  workspace holds
 * dnb_vjp_reversed_workspace_doubles(n).  Outputs must not alias inputs. */
dnb_status dnb_simulate_vjp_reversed(dnb_ctx* ctx, int64_t n, const double* mass,
                                     const dnb_pot* pot, double dt, int64_t n_steps,
                                     int64_t ckpt_every, const double* tape,
                                     const double* pos_T, const double* vel_T,
                                     const double* gpos_T, const double* gvel_T,
                                     double* workspace, double* gpos_0, double* gvel_0,
                                     double* gmass, double* gparams, void* stream);

/* Squared maximum mean discrepancy between the point clouds pos [3][n] and
 * tgt [3][m] (Sec. 2.2.1 and Fig. 2, step 4), with the Gaussian kernel
 * k(x, y) = exp(-|x - y|^2 / (2 h^2)) and the biased (V-statistic) estimate:
 *   L = mean_ij k(x_i,x_j) + mean_ab k(y_a,y_b) - 2 mean_ia k(x_i,y_a).
 * loss: device scalar.  gpos [3][n] (nullable): dL/dpos.  FP64 throughout; each
 * kernel value is within 0.6 ulp of exp at the rounded argument, and a NaN
 * position makes the loss NaN.  Requires n, m <= max_n of the context and
 * h > 0. */
dnb_status dnb_mmd(dnb_ctx* ctx, int64_t n, const double* pos, int64_t m, const double* tgt,
                   double h, double* loss, double* gpos, void* stream);

/* Energies of the system (diagnostic): out3 [3] (device) = kinetic energy,
 * softened pair energy -G sum_{i<j} m_i m_j (r_ij^2 + eps^2)^(-1/2), and
 * sum_i m_i Phi_ext(x_i).  FP64. */
dnb_status dnb_energy(dnb_ctx* ctx, int64_t n, const double* pos, const double* vel,
                      const double* mass, const dnb_pot* pot, double* out3, void* stream);

/* Test-particle orbit in the external potential only (Fig. 2, step 2: the
 * progenitor's centre of mass integrated backward as a single particle).
 * w0 [6] = (x, y, z, vx, vy, vz); n_steps kick-drift-kick steps of dt (dt < 0
 * integrates backward); w_out [6].  traj (nullable) receives the 3 (n_steps+1)
 * positions x_0..x_{n_steps} as [n_steps+1][3], which dnb_orbit_vjp needs. */
dnb_status dnb_orbit(dnb_ctx* ctx, const double* w0, const dnb_pot* pot, double dt,
                     int64_t n_steps, double* w_out, double* traj, void* stream);

/* Adjoint of dnb_orbit.  gw_out [6]: cotangent of w_out.  Outputs gw0 [6] and
 * gparams [3] = dL/dm_nfw, dL/dm_mn, dL/ddt (device). */
dnb_status dnb_orbit_vjp(dnb_ctx* ctx, const double* traj, const dnb_pot* pot, double dt,
                         int64_t n_steps, const double* gw_out, double* gw0, double* gparams,
                         void* stream);

/* Place a Plummer sphere at the phase-space point w [6] (Fig. 2, step 3):
 * pos = w_x + a_p * xi, vel = w_v + sqrt(G m_tot / a_p) * zeta, mass = m_tot / n.
 * xi, zeta [3][n] are unit samples (G = M = a = 1).  m_tot and a_p are host
 * scalars, w is a device pointer. */
dnb_status dnb_place_plummer(dnb_ctx* ctx, int64_t n, const double* w, const double* xi,
                             const double* zeta, double m_tot, double a_p, double G,
                             double* pos, double* vel, double* mass, void* stream);

/* Adjoint of dnb_place_plummer.  gpos, gvel [3][n], gmass [n] (nullable) are the
 * cotangents of its outputs.  Outputs: gw [6] = (sum_i gpos_i, sum_i gvel_i) and
 * gm_tot [1] = dL/dm_tot (device). */
dnb_status dnb_place_plummer_vjp(dnb_ctx* ctx, int64_t n, const double* zeta, double m_tot,
                                 double a_p, double G, const double* gpos, const double* gvel,
                                 const double* gmass, double* gw, double* gm_tot, void* stream);

/* ------------------------------------------------------ batched ensembles ---
 * Many independent systems of the same size advanced together (Sec. 2: running
 * many simulations at once by vectorising over them, which is how training sets
 * for the surrogate and parameter grids are produced).  Member b owns
 * pos[b] and vel[b] ([batch][3][n], device), mass[b] ([batch][n], device) and
 * the row params[b] of a HOST table [batch][8] = (G, eps, m_nfw, rs_nfw, m_mn,
 * a_mn, b_mn, dt).  Every member takes n_steps kick-drift-kick steps of its own
 * dt in place; with tape not NULL (dnb_batch_tape_doubles) every step is
 * recorded for dnb_simulate_batch_vjp.  Pair terms use the DNB_FP32C
 * arithmetic whatever the context's precision, so every eps must be > 0.
 * The table is copied to the context before the call returns; the copy waits
 * for work already queued on the stream.  The ensemble must fit the context:
 * batch <= DNB_BATCH_MAX and roughly batch * n <= max_n (DNB_ERR_ARG names the
 * limit that is exceeded). */
#define DNB_BATCH_MAX 4096

dnb_status dnb_simulate_batch(dnb_ctx* ctx, int64_t batch, int64_t n, double* pos, double* vel,
                              const double* mass, const double* params, int64_t n_steps,
                              double* tape, void* stream);

/* Number of doubles of the tape dnb_simulate_batch writes when tape is not NULL:
 * every step is kept, the states (x, v) of steps 0 .. T-1 ([T][batch][6][n]) and
 * the internal accelerations of steps 0 .. T ([T+1][batch][3][n]); 0 for T = 0,
 * -1 for invalid sizes. */
int64_t dnb_batch_tape_doubles(int64_t batch, int64_t n, int64_t n_steps);

/* Reverse-mode gradient through dnb_simulate_batch for every member (the
 * batched form of dnb_simulate_vjp: the same discrete adjoint, member by member,
 * FP32C pair terms).  Inputs: the same batch, n, mass, params (HOST table) and
 * n_steps >= 1 as the forward call, its tape, the final positions pos_T
 * [batch][3][n] and the loss cotangents gpos_T, gvel_T [batch][3][n] (gvel_T may
 * be NULL).  workspace: 4 batch n doubles.  Outputs gpos_0, gvel_0 [batch][3][n]
 * and gparams [batch][4] (device) = per member (dL/dm_nfw, dL/dm_mn, dL/ddt,
 * sum_k m_k dL/dm_k).  No per-particle mass gradient.  Outputs must not alias
 * inputs.  As for dnb_simulate_vjp, the tape must be one the context recorded
 * (here with the batch size and the parameter table's contents) and pos_T the
 * position array of that forward call, else DNB_ERR_STATE. */
dnb_status dnb_simulate_batch_vjp(dnb_ctx* ctx, int64_t batch, int64_t n, const double* mass,
                                  const double* params, int64_t n_steps, const double* tape,
                                  const double* pos_T, const double* gpos_T, const double* gvel_T,
                                  double* workspace, double* gpos_0, double* gvel_0,
                                  double* gparams, void* stream);

/* Loss of every member of an ensemble (the grid-search stage of the inference
 * pipeline, Sec. 2.2.1: the MMD between simulated and observed streams at many
 * parameter combinations; with a target per member, the bootstrap of Fig. 2
 * step 6, where every member is compared with its own resampled stream).
 * pos [batch][3][n] (device); tgt [3][m] shared by all members
 * (tgt_per_member = 0) or [batch][3][m] (tgt_per_member = 1); loss [batch]
 * (device): loss[b] = the squared MMD of dnb_mmd between pos[b] and its target;
 * gpos [batch][3][n] (nullable) = dL_b/dpos[b] (the gradient of dnb_mmd for
 * every member).  Requires n, m <= max_n, h > 0, batch <= DNB_BATCH_MAX and the
 * partial sums to fit the context (DNB_ERR_ARG otherwise). */
dnb_status dnb_mmd_batch(dnb_ctx* ctx, int64_t batch, int64_t n, const double* pos, int64_t m,
                         const double* tgt, int tgt_per_member, double h, double* loss,
                         double* gpos, void* stream);

/* Loss of every member of an ensemble against each of n_tgt targets (the grid
 * stage of a bootstrap, Fig. 2: every realisation of the observed stream
 * compared with every grid run, the runs made once).  pos [batch][3][n], tgts
 * [n_tgt][3][m] (device); loss [batch][n_tgt] (device): loss[b][t] = the squared
 * MMD of dnb_mmd between pos[b] and tgts[t], equal bit for bit to dnb_mmd_batch
 * with tgt_per_member = 1 and every member's target tgts[t].  The member-member
 * sums are computed once for all targets.  Requires n, m <= max_n, h > 0,
 * batch and n_tgt <= DNB_BATCH_MAX and the partial sums to fit the context
 * (DNB_ERR_ARG otherwise). */
dnb_status dnb_mmd_batch_targets(dnb_ctx* ctx, int64_t batch, int64_t n, const double* pos,
                                 int64_t n_tgt, int64_t m, const double* tgts, double h,
                                 double* loss, void* stream);

/* Plummer spheres for every member of an ensemble (the batched form of
 * dnb_place_plummer, Fig. 2 step 3): member b is centred on w[b] ([batch][6],
 * device) with total mass m_tot[b] ([batch], device, > 0); the unit samples xi,
 * zeta [3][n] are shared.  Outputs pos, vel [batch][3][n] and mass [batch][n]:
 * pos = w_x + a_p xi, vel = w_v + sqrt(G m_tot / a_p) zeta, mass = m_tot / n. */
dnb_status dnb_place_plummer_batch(dnb_ctx* ctx, int64_t batch, int64_t n, const double* w,
                                   const double* xi, const double* zeta, const double* m_tot,
                                   double a_p, double G, double* pos, double* vel, double* mass,
                                   void* stream);

/* Largest batch of systems of n particles that dnb_simulate_batch accepts on
 * this context (0 if ctx is NULL or n < 1).  Host arithmetic only. */
int64_t dnb_batch_capacity(const dnb_ctx* ctx, int64_t n);

/* Test-particle orbits of a batch (the batched form of dnb_orbit): w0, w_out
 * [batch][6] (device), params the same HOST table as dnb_simulate_batch (eps
 * is unused); traj (nullable) receives [batch][n_steps+1][3] positions for
 * dnb_orbit_batch_vjp.  batch <= DNB_BATCH_MAX. */
dnb_status dnb_orbit_batch(dnb_ctx* ctx, int64_t batch, const double* w0, const double* params,
                           int64_t n_steps, double* w_out, double* traj, void* stream);

/* Adjoint of dnb_orbit_batch for every member (the batched form of
 * dnb_orbit_vjp): gw_out [batch][6] in; gw0 [batch][6] and gparams [batch][3] =
 * (dL/dm_nfw, dL/dm_mn, dL/ddt) out (device).  Every dt must be non-zero. */
dnb_status dnb_orbit_batch_vjp(dnb_ctx* ctx, int64_t batch, const double* traj,
                               const double* params, int64_t n_steps, const double* gw_out,
                               double* gw0, double* gparams, void* stream);

/* Adjoint of dnb_place_plummer_batch: gpos, gvel [batch][3][n] in; gw [batch][6]
 * = (sum_i gpos_i, sum_i gvel_i) and gm_tot [batch] = dL/dm_tot through the
 * velocity scale (device).  Requires batch ceil(n / 256) <= ceil(max_n / 256). */
dnb_status dnb_place_plummer_batch_vjp(dnb_ctx* ctx, int64_t batch, int64_t n,
                                       const double* zeta, const double* m_tot, double a_p,
                                       double G, const double* gpos, const double* gvel,
                                       double* gw, double* gm_tot, void* stream);

/* Instrumentation (not part of the method).  With enable != 0, every launch of
 * the two O(N^2) kernels (forward pair sum, pair VJP) issued through this
 * context is bracketed by HIP events recorded on the launch's stream.
 * dnb_profile_read synchronises those events and returns, in the HOST array
 * out4: total milliseconds and launch count of the forward pair kernel, then the
 * same for the VJP kernel, since the last read; it then resets the totals.
 * Event objects are created on demand and kept by the context. */
dnb_status dnb_profile(dnb_ctx* ctx, int enable);
dnb_status dnb_profile_read(dnb_ctx* ctx, double* out4);

#ifdef __cplusplus
}
#endif

#endif /* DNB_H */
