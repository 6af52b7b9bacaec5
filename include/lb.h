/*
 * lb.h -- C ABI of the MI355X (gfx950) D2Q9 lattice-Boltzmann library.
 *
 * The library advances the lattice-Boltzmann model of Basagaoglu, Harwell,
 * Nguyen & Succi (arXiv:2006.12910) on one GPU:
 *   - BGK collision with the velocity-shift body force (Sec. 2, Eqs. LB1-LB2),
 *   - pull streaming with halfway bounce-back on walls and obstacles,
 *     Zou-He density faces for pressure-driven flow,
 *   - moving-wall bounce-back and link momentum exchange on circular particles,
 *     LJ-type repulsion and Newton-Euler updates (Sec. 3, Eqs. MP1-MP8),
 *   - thermal noise on the non-conserved moments (Sec. 4, Eqs. NP1-NP2,
 *     Table t1) from a counter-based Philox4x32-10 generator,
 *   - a local power-law relaxation time (Sec. 5, Eqs. nn1-nn5).
 *
 * Conventions
 *   - Every function returns lb_status (LB_OK = 0, negative on error); no C++
 *     exception and no abort crosses the ABI.  lb_last_error() returns a
 *     thread-local description of the last failure on the calling thread.
 *   - Lattice units (dx = dt = 1).  Host arrays are row-major [ny][nx]
 *     (x fastest); populations are [9][ny][nx] in the paper's direction order:
 *     rest, (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1).
 *   - Device memory: the caller owns every workspace (any device allocation,
 *     e.g. a torch uint8 tensor), keeps it alive and unmodified until the
 *     matching destroy call, and sizes it with the *_workspace_bytes query.
 *     The library allocates no device memory of its own.
 *   - Streams: every call is ordered on the HIP stream given at creation
 *     (hipStream_t passed as void*; NULL is the default stream).  lb_step /
 *     lb_batch_step only enqueue work.  Calls that return data to the host
 *     (lb_moments, lb_get_particles, lb_mass, lb_get_populations) synchronise
 *     that stream and report errors the device latched since the last such
 *     call (LB_EUNSTABLE for a non-finite density or a particle faster than
 *     half a node per step).
 *   - Host arrays passed in are copied before the call returns.
 *   - A handle is not thread-safe; distinct handles may be used concurrently.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Layout version of the descriptor structs: a caller sets abi_version to
 * the value its header carries, and a library built against another layout
 * refuses the descriptor (LB_EINVAL).  2: lb_domain_desc gained collision
 * and magic; lb3_domain_desc gained rounding, seed, lattice and the power
 * law.  3: lb3_domain_desc gained kT. */
#define LB_ABI_VERSION 3u

typedef int32_t lb_status;
#define LB_OK 0
#define LB_EINVAL (-1)        /* bad argument or unsupported value             */
#define LB_ENOMEM (-2)        /* workspace smaller than the query returned     */
#define LB_EHIP (-3)          /* a HIP runtime call failed                     */
#define LB_ESTATE (-4)        /* call not allowed in the handle's state        */
#define LB_EUNSTABLE (-5)     /* device latched a non-finite or runaway value  */
#define LB_EUNSUPPORTED (-6)  /* valid but not implemented combination         */

/* boundary kinds: per axis */
#define LB_PERIODIC 0
#define LB_WALL 1             /* outermost rows (y) / columns (x) are solid     */
#define LB_PRESSURE 2         /* x only: Zou-He density faces rho_in / rho_out  */

/* population storage.  Arithmetic is FP64 for LB_F64 and FP32 otherwise; the
 * stored value is the deviation f_i - w_i rho0 (scaled by 2, 8, 32 for the
 * rest, axis and diagonal directions in the 16-bit formats); see also
 * LB_COMPUTE_* below. */
#define LB_F64 0
#define LB_F32 1
#define LB_F16_DELTA 2
#define LB_BF16_DELTA 3

#define LB_ROUND_NEAREST 0
/* stochastic rounding: FP32 storage (with FP32 arithmetic) and the 16-bit
 * formats.  Each stored value rounds to one of its two neighbours with
 * probability proportional to closeness, the random bits hashed from (node,
 * step, seed, domain_id): unbiased, so slow flows whose per-step change is
 * below half the spacing of the stored values do not stagnate, and
 * reproducible run to run. */
#define LB_ROUND_STOCHASTIC 1

/* arithmetic of the collision: the storage's own precision (FP64 for LB_F64,
 * FP32 otherwise), or FP64 with any storage.  FP32 arithmetic keeps mass and
 * momentum exact by construction, but its rounding still biases flows whose
 * state changes by a near-constant amount each step (the plug-flow core of a
 * channel at tau close to 1/2); FP64 arithmetic with FP32 storage removes that
 * at no memory cost. */
#define LB_COMPUTE_NATIVE 0
#define LB_COMPUTE_F64 1

#define LB_INIT_REST 0        /* rho = rho0, u = 0                               */
#define LB_INIT_FIELDS 1      /* f = equilibrium of init_rho/init_ux/init_uy     */

typedef struct lb_domain_desc {
  uint32_t abi_version;       /* LB_ABI_VERSION                                  */
  int32_t nx, ny;             /* lattice size, each in [3, 65536], with         
                               * 9 * ny * (nx rounded up to 64) * (bytes per    
                               * stored value: 8, 4 or 2) < 2^32                */
  int32_t bc_x, bc_y;         /* LB_PERIODIC | LB_WALL | LB_PRESSURE (x only)   */
  int32_t storage;            /* LB_F64 | LB_F32 | LB_F16_DELTA | LB_BF16_DELTA */
  int32_t rounding;           /* LB_ROUND_NEAREST | LB_ROUND_STOCHASTIC         */
  int32_t compute;            /* LB_COMPUTE_NATIVE | LB_COMPUTE_F64             */
  int32_t obstacles;          /* nonzero: reserve a label plane for lb_set_obstacles */
  int32_t max_particles;      /* capacity of lb_add_particles, 0..250            */
  int32_t power_law;          /* nonzero: local tau* of Sec. 5                   */
  int32_t init_kind;          /* LB_INIT_REST | LB_INIT_FIELDS                   */
  uint32_t domain_id;         /* folded into the noise key                       */
  uint64_t seed;              /* noise key                                       */
  double rho0;                /* reference density (> 0)                         */
  double tau;                 /* relaxation time (> 1/2); unused with power_law  */
  double gx, gy;              /* body acceleration g (Sec. 2)                    */
  double rho_in, rho_out;     /* LB_PRESSURE densities at x = 0 and x = nx-1     */
  double kT;                  /* thermal energy k_B T; 0 disables noise (Sec. 4) */
  double n_index, K;          /* power-law index n and consistency xi (Eq. nn1)  */
  double tau_min, tau_max;    /* clamp of tau*, 1/2 < tau_min <= tau_max         */
  double lj_psi, lj_rit;      /* repulsion stiffness and threshold (Eq. MP2)     */
  double lj_floor;            /* smallest gap used in the repulsion (> 0)        */
  const double *init_rho;     /* LB_INIT_FIELDS: host [ny][nx] fields, copied    */
  const double *init_ux;
  const double *init_uy;
  int32_t collision;          /* LB_BGK (the paper's, Sec. 2) | LB_TRT           */
  double magic;               /* LB_TRT: (tau - 1/2)(tau_minus - 1/2), > 0       */
} lb_domain_desc;

/* Collision.  LB_TRT (an addition to the paper's BGK): the parts of each
 * population pair symmetric and antisymmetric under e -> -e relax with 1/tau
 * and 1/tau_minus, (tau - 1/2)(tau_minus - 1/2) = magic, and the body force
 * shifts the equilibrium velocity by tau_minus g (the antisymmetric parts
 * carry the momentum, so the input per step stays rho g); with the power law
 * tau_minus follows the local tau*.  magic = 3/16 puts the halfway
 * bounce-back walls of a channel exactly halfway whatever tau; magic =
 * (tau - 1/2)^2 is BGK.  Not with thermal noise (LB_EUNSUPPORTED). */
#define LB_BGK 0
#define LB_TRT 1

#define LB_PARTICLE_FIXED 1   /* position and velocities are held fixed          */

typedef struct lb_particle {
  double x, y;                /* centre (lattice units; nodes at integers)       */
  double radius;              /* > 0; interior nodes: |r - r_c| < radius         */
  double density_ratio;       /* rho_p / rho0 (> 0)                              */
  double ux, uy, omega;       /* translational and angular velocity              */
  double fx, fy, torque;      /* output: total force/torque of the last step     */
  int32_t flags;              /* LB_PARTICLE_FIXED                               */
  int32_t reserved;
} lb_particle;

typedef struct lb_domain lb_domain;
typedef struct lb_batch lb_batch;

/* Workspace size in bytes for a domain described by *desc (validates desc). */
lb_status lb_workspace_bytes(const lb_domain_desc *desc, size_t *bytes);

/* Create a domain in the caller's device workspace and initialise the
 * populations (Sec. 2: equilibrium of the initial fields, then the collision
 * of step 0).  dev_workspace must be 256-byte aligned.  *out receives the
 * handle.  Errors: LB_EINVAL (desc), LB_ENOMEM (bytes too small), LB_EHIP. */
lb_status lb_create_domain(const lb_domain_desc *desc, void *dev_workspace, size_t bytes,
                           void *hip_stream, lb_domain **out);

/* Mark stationary solid nodes: host mask [ny][nx] (n = nx*ny), nonzero = solid,
 * bounced back halfway (Sec. 3 obstacles and walls).  Requires desc.obstacles
 * and no particles yet (LB_ESTATE otherwise). */
lb_status lb_set_obstacles(lb_domain *d, const uint8_t *host_mask, size_t n);

/* Add n circular particles (Sec. 3).  *first_id receives the index of the
 * first one.  LB_EINVAL if a disc covers a solid node or another particle,
 * exceeds max_particles, or its bounding box (max(radius + lj_rit + 1,
 * radius + 3) nodes each side) does not fit in a periodic axis or reaches a
 * pressure face; LB_ESTATE if the domain is in a batch. */
lb_status lb_add_particles(lb_domain *d, const lb_particle *p, int32_t n, int32_t *first_id);

/* Enqueue nsteps full time steps (collision, noise, streaming, boundaries,
 * particle coupling; Sec. 2-5) on the domain's stream; nsteps >= 0.  Every
 * step checks the densities it pulls; a call during which the step counter
 * passes a multiple of LB_OPT_MASS_INTERVAL (default 256) ends with the FP64
 * density sum of the final state (see lb_mass, lb_set_mass_check).  A
 * non-finite density, or a sum beyond the drift threshold, latches a flag
 * that the next synchronising call reports as LB_EUNSTABLE.  Steps replay
 * captured hipGraphs of fixed sizes (LB_OPT_GRAPH_CHUNK and the powers of
 * four below it), all captured by the first call with nsteps > 0. */
lb_status lb_step(lb_domain *d, int64_t nsteps);

/* Moments of Sec. 2: density rho = sum_i f_i and velocity u = j/rho + g/2
 * (j = sum_i f_i e_i; the half-step force shift makes u the fluid velocity of
 * the velocity-shift forcing, exact for the steady channel) at every node
 * (zero on solid nodes), host FP64 [ny][nx] each.  Synchronises. */
lb_status lb_moments(lb_domain *d, double *rho, double *ux, double *uy);

/* Same, into device FP64 arrays [ny][nx] (no synchronisation). */
lb_status lb_moments_device(lb_domain *d, double *dev_rho, double *dev_ux, double *dev_uy);

/* Reporting offload (the analogue of the paper's output offloading from the
 * simulation threads, Sec. 7, task-level pipelining): enqueue on the domain's stream the moments of the
 * current state (as lb_moments) into dev_stage, caller-owned device memory of
 * 3 nx ny doubles ([rho][ux][uy], each [ny][nx]), then copy them on
 * copy_stream (another stream of the same device, not the domain's) into the
 * host arrays rho, ux, uy ([ny][nx] each), which should be pinned memory
 * (hipHostMalloc; torch pin_memory) for the copy to run asynchronously.
 * Returns without waiting: steps enqueued afterwards run while the copy
 * proceeds.  dev_stage and the host arrays must stay untouched until
 * lb_moments_wait returns; a later call waits on the device for an earlier
 * call's copy before it writes dev_stage again.  Errors: LB_EINVAL for a null
 * pointer or copy_stream equal to the domain's stream; the state's health is
 * reported by the next synchronising call, as for lb_step. */
lb_status lb_moments_async(lb_domain *d, double *dev_stage, double *rho, double *ux, double *uy,
                           void *copy_stream);
/* Block until the copy of the last lb_moments_async call has landed in host
 * memory (returns at once if none is pending).  Does not wait for the
 * domain's stream. */
lb_status lb_moments_wait(lb_domain *d);

/* Copy out the first n particles' state (n <= count): centre, velocities
 * after the last Newton-Euler update (Sec. 3, Eqs. MP5-MP6) and the total
 * force and torque that update used (Eqs. MP1-MP4).  Synchronises. */
lb_status lb_get_particles(lb_domain *d, lb_particle *out, int32_t n);

/* Global mass check (the FP64 density sum with its non-finite latch): FP64
 * sum of rho = sum_i f_i (Sec. 2) over the non-solid nodes of the current
 * state, computed on the device in a fixed order (bit-reproducible).  The same
 * sum ends the lb_step / lb_batch_step calls that LB_OPT_MASS_INTERVAL
 * selects.
 * Synchronises; LB_EUNSTABLE if the device latched an error (see above). */
lb_status lb_mass(lb_domain *d, double *total);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): lb_mass
 * without the domain's reduction area.  The FP64 density sum of the current
 * state (same blocks, same order, so bit-identical to lb_mass) is written to
 * dev_total, caller-owned device memory of one double, enqueued on the
 * domain's stream without synchronising; it latches a non-finite or drifting
 * sum as lb_mass does.  Its partial sums go to a fixed device array of the
 * library (1024 doubles, 8 KiB, on each GPU used, held until the process
 * ends; every block overwrites its own entry, so nothing needs clearing).
 * Calls on one GPU share that array: calls that may overlap on one GPU (on
 * different streams) race.  LB_EINVAL for a null argument or a domain whose
 * sum needs more partial sums than the array holds (none does: at most 1024);
 * allocates nothing (no hipMalloc, hipFree or allocating library call). */
lb_status lb_mass_static(lb_domain *d, double *dev_total);

/* Mass-drift threshold for the density sums of lb_mass and of lb_step /
 * lb_batch_step (LB_OPT_MASS_INTERVAL): with rel_tol > 0, a sum M that leaves
 * |M - M_ref| <= rel_tol |M_ref| latches LB_EUNSTABLE, where M_ref is the
 * density sum at the time of this call (computed here, as lb_mass does).
 * Collision and streaming conserve mass exactly on periodic, wall, obstacle
 * and particle domains (Sec. 2-3), so the threshold measures accumulated
 * rounding and catches a blow-up before it turns non-finite; density faces
 * (LB_PRESSURE) exchange mass with the outside and are better left at 0 (the
 * default: no drift check).  Synchronises.  LB_EINVAL for a negative or
 * non-finite rel_tol. */
lb_status lb_set_mass_check(lb_domain *d, double rel_tol);

/* Completed step count. */
lb_status lb_time(lb_domain *d, int64_t *t);

/* Post-collision state as deviations f*_i - w_i rho0, host FP64 [9][ny][nx]
 * (get synchronises; set rounds to the storage format, exactly for values
 * that get returned).  With lb_time / lb_set_time and, for particles,
 * lb_get_particle_state / lb_set_particle_state this checkpoints a domain
 * bit-exactly (the paper's dumps for restarts, Sec. 7): a domain created
 * with the same description and obstacles, given the time, the populations
 * and the particle state in that order, continues exactly as the original,
 * noise included (the generator is keyed by node and step). */
lb_status lb_get_populations(lb_domain *d, double *host_dev_f);
lb_status lb_set_populations(lb_domain *d, const double *host_dev_f);

/* Set the completed step count (>= 0), keeping the current state: the state
 * of step t lives in population buffer t mod 2, so a change of parity moves
 * it.  Not allowed in a batch (LB_ESTATE).  Synchronises. */
lb_status lb_set_time(lb_domain *d, int64_t t);

/* Particle state of a checkpoint (Sec. 3): the lb_particle record (centre,
 * velocities, and fx, fy, torque, the totals of the last update, which the
 * two-step force mean of LB_OPT_FORCE_AVERAGE reuses) and the force and
 * torque of the nodes covered or uncovered by the last step (Eq. MP3),
 * pending for the next update. */
typedef struct lb_particle_state {
  lb_particle p;
  double cover_fx, cover_fy, cover_torque;
} lb_particle_state;

/* Copy out the state of all n particles (n == count).  Synchronises. */
lb_status lb_get_particle_state(lb_domain *d, lb_particle_state *out, int32_t n);
/* Replace every particle by the n given states (n <= max_particles; n = 0
 * removes them all), relabelling the nodes they cover.  Same checks as
 * lb_add_particles (LB_EINVAL), except that overlaps between the given
 * particles are accepted as they are (a checkpoint restores whatever state
 * it holds); LB_ESTATE in a batch.  Synchronises. */
lb_status lb_set_particle_state(lb_domain *d, const lb_particle_state *in, int32_t n);

/* Options (see LB_OPT_*).  Changing one drops the cached step graphs. */
#define LB_OPT_USE_GRAPH 1     /* 1 (default): lb_step replays a captured hipGraph */
#define LB_OPT_TILE_WIDTH 2    /* threads per tile row: 64, 128 or 256            */
#define LB_OPT_ROWS_PER_THREAD 3 /* nodes per thread along y: 1..16               */
#define LB_OPT_GRAPH_CHUNK 4   /* steps per captured graph, 1..4096 (default 256) */
/* 0 (default): the particle velocity update is Eqs. MP5-MP6 with the force and
 * torque of the current step, as the paper writes it.  1: with the mean of the
 * current and the previous step's force and torque (the previous ones of a
 * newly added particle are zero).  The explicit update lets a period-two
 * oscillation of neighbouring near-neutral discs grow (e.g. density ratio 1.05
 * at tau = 0.7); the mean damps it.  Not changeable while in a batch. */
#define LB_OPT_FORCE_AVERAGE 5
/* 1 (default): a domain that is periodic on both axes, has no particles and
 * no noise or power law, with native arithmetic, advances two time steps per
 * pass over memory (each four steps as two such launches; the first step is
 * kept in on-chip memory) -- bit-identical to single steps, with half the
 * memory traffic per step.  0: single steps only.  A batch takes it when all
 * its domains do.  Not changeable while in a batch. */
#define LB_OPT_TWO_STEP 6
/* 0 (default) or 1: lb_step of a domain with particles runs the particle
 * coupling (k_post of the previous step, k_pre, then the sweep of the tiles
 * within its reach) on a second stream beside the sweep of all other tiles --
 * the paper's pipelining of particle interaction with streaming (Sec. 7).
 * Bit-identical to the serial order.  Batches keep the serial order.  It
 * pays only where the runtime runs the two branches of a step graph
 * concurrently; where it serialises them the extra launches make it slower. */
#define LB_OPT_OVERLAP 7
/* Steps between the FP64 density sums that lb_step / lb_batch_step run
 * (>= 1, default 256; 1: after every call).  On a batch it counts the batch's
 * own steps. */
#define LB_OPT_MASS_INTERVAL 8
/* Output rows of the two-step sweep's tiles (62 columns each): one of 10, 14,
 * 18 (16-bit storage; default 14), 6, 10, 14 (FP32; default 10), 4, 6, 8
 * (FP64; default 6); results do not depend on it.  On a batch: the height of
 * its launch (at creation the members' common height, else the default). */
#define LB_OPT_TWO_STEP_ROWS 10
lb_status lb_set_option(lb_domain *d, int32_t key, int64_t value);
lb_status lb_get_option(lb_domain *d, int32_t key, int64_t *value);

/* Destroy the handle (the workspace can then be reused).  Synchronises. */
lb_status lb_destroy_domain(lb_domain *d);

/* Batching: several independent domains advance together, one sweep launch
 * per step over the tiles of all of them, replayed from a hipGraph.  The
 * domains must share storage, arithmetic, noise and power-law settings
 * (LB_EUNSUPPORTED otherwise); sizes, boundaries, obstacles, particles and all
 * parameters may differ.  Every domain keeps its own noise key and step
 * counter; a batched run is bit-identical to running each domain alone.  The
 * domains may not change (obstacles, particles, tile options) while in a
 * batch (LB_ESTATE).  The batch runs on its own stream: order it against the
 * domains' streams (e.g. synchronise) when mixing lb_step and lb_batch_step.
 * The batch workspace is caller-owned device memory. */
lb_status lb_batch_workspace_bytes(lb_domain *const *domains, int32_t n, size_t *bytes);
lb_status lb_batch_create(lb_domain *const *domains, int32_t n, void *dev_workspace,
                          size_t bytes, void *hip_stream, lb_batch **out);
/* As lb_step for every domain of the batch, on the batch's stream (Sec. 2-5
 * for each member).  The density sums that LB_OPT_MASS_INTERVAL selects
 * (counted in the batch's own steps) cover every member in two launches. */
lb_status lb_batch_step(lb_batch *b, int64_t nsteps);
/* Batch options: LB_OPT_USE_GRAPH, LB_OPT_GRAPH_CHUNK, LB_OPT_MASS_INTERVAL,
 * LB_OPT_TWO_STEP_ROWS (LB_EINVAL for the others). */
lb_status lb_batch_set_option(lb_batch *b, int32_t key, int64_t value);
lb_status lb_batch_get_option(lb_batch *b, int32_t key, int64_t *value);
lb_status lb_batch_destroy(lb_batch *b);

/* Diagnostic: the six standard normals Theta_3..Theta_8 (Sec. 4, Eq. NP2)
 * that the collision of step `step` adds at nodes node0 .. node0+count-1 of a
 * domain with this seed and domain_id; device FP32 output [count][6]
 * (count <= 2^28).  Both transforms start from the same Philox4x32-10 block
 * and uniforms.  fp32_arithmetic = 0: the transform of collisions in FP64
 * arithmetic (FP64 storage, LB_COMPUTE_F64), every operation a correctly
 * rounded IEEE float operation in a fixed order (an independent
 * implementation of the definition reproduces it bit for bit).  1: the
 * transform of collisions in FP32 arithmetic (FP32 and 16-bit storage),
 * through the hardware's log2, square root, sine and cosine instructions,
 * within ~1e-6 absolute of the former.  Synchronises the stream; LB_EINVAL
 * for a null output, another fp32_arithmetic or a larger count. */
lb_status lb_noise_normals(uint64_t seed, uint32_t domain_id, uint32_t step, uint32_t node0,
                           uint32_t count, int32_t fp32_arithmetic, float *dev_out,
                           void *hip_stream);

/* Autotune this domain's sweep tiles: times each candidate single-step tile
 * width / rows-per-thread pair over `steps` single steps (the two-step sweep
 * off while timing) and keeps the fastest; where the two-step sweep applies,
 * then also its tile height (LB_OPT_TWO_STEP_ROWS), timed over `steps`
 * rounded up to a multiple of four.  The height chosen is cached for the
 * process per (storage, label plane, rounding, size class floor(log2(nx ny)))
 * and later domains of a cached class take it without timing.  The state
 * advances by the steps timed.  *best_ms receives the best time per step. */
lb_status lb_autotune(lb_domain *d, int32_t steps, double *best_ms);

/* Autotune a batch's two-step tile height (LB_OPT_TWO_STEP_ROWS of the
 * batch): each instantiated height is timed over `steps` steps (rounded up to
 * a multiple of four, after an untimed call of as many), the fastest kept
 * and cached for the process per (storage, label plane in any member,
 * rounding, size class of the batch's total sites); a cached class is applied
 * without timing (*best_ms = 0).  A batch that runs single steps is left as
 * it is.  The members' states advance by the steps timed. */
lb_status lb_batch_autotune(lb_batch *b, int32_t steps, double *best_ms);

/* ---------------------------------------------------------------------------
 * 3D domains, D3Q19 or D3Q27: the three-dimensional lattices the paper names
 * as its next step (Sec. 8), with the same BGK collision and velocity-shift
 * body force (Sec. 2, Eqs. LB1-LB2 with c_s^2 = 1/3; D3Q19 weights 1/3, 1/18,
 * 1/36; D3Q27 weights 8/27, 2/27, 1/54, 1/216), pull streaming with
 * periodic wrap and halfway bounce-back on solid nodes.  The velocity set:
 * rest; (+-1,0,0), (0,+-1,0), (0,0,+-1); then (1,1,0), (-1,-1,0), (1,-1,0),
 * (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1),
 * (0,1,-1), (0,-1,1); on D3Q27 also (1,1,1), (-1,-1,-1), (1,1,-1),
 * (-1,-1,1), (1,-1,1), (-1,1,-1), (-1,1,1), (1,-1,-1) (opposites in
 * consecutive pairs).  Host node arrays are [nz][ny][nx] (x fastest),
 * populations [q][nz][ny][nx] (q = 19 or 27).  Storage: deviations
 * f_i - w_i rho0 as LB_F64, LB_F32, or the 16-bit LB_F16_DELTA /
 * LB_BF16_DELTA (Sec. 3's reduced-precision storage carried to 3D: the
 * stored value is the deviation times 2, 16, 32 (D3Q19) or 4, 16, 64, 256
 * (D3Q27) for the rest, axis, edge and corner directions, rounded to nearest
 * or stochastically with bits hashed from (node, step, seed)); arithmetic
 * FP64 for LB_F64 and FP32 otherwise, the FP32 increment holding exactly the
 * collision's mass and momentum change before the one rounding to storage.
 * Collision: BGK, or the two-relaxation-time (TRT) variant, in which the
 * parts of each population pair symmetric and antisymmetric under e -> -e
 * relax with 1/tau and 1/tau_minus, (tau - 1/2)(tau_minus - 1/2) = magic,
 * and the body force shifts the equilibrium velocity by tau_minus g (the
 * antisymmetric parts carry the momentum); magic = 3/16 puts halfway
 * bounce-back walls of a channel exactly halfway whatever tau,
 * magic = (tau - 1/2)^2 is BGK.  Power law (Sec. 5): the local tau* from the
 * non-equilibrium stress as on the 2D domains, with all nine components of
 * the 3D stress in its Frobenius norm (with TRT, tau_minus follows tau*).
 * Thermal noise (Sec. 4, Eqs. NP1-NP2 carried to 3D): kT > 0 adds
 * to every collision the Gaussian whose covariance is
 * 3 rho kT omega (2 - omega) (W - w w^T - 3 (W e)(W e)^T), W = diag(w)
 * (omega = 1/tau*, local with the power law): independent unit noise on
 * every mode that is not mass or momentum, as the D2Q9 method has.  It is
 * drawn as zeta_i = amp (eta_i - w_i S - 3 w_i e_i.V), eta_i = sqrt(w_i) xi_i,
 * S = sum eta, V = sum e eta, amp = sqrt(3 rho kT omega (2 - omega)), from q
 * unit normals xi_i: Philox4x32-10 block b of node n = (z ny + y) nx + x at
 * step t (counter (n, t, b, 0), key (lo32(seed), hi32(seed))) gives
 * xi_{6b} .. xi_{6b+5} by the D2Q9 domains' Box-Muller recipe
 * (lb_noise_normals with domain_id 0 is block 0).  Step t is the collision that produces the
 * state of time t (the one in lb3_create_domain is t = 0).  FP64 storage
 * evaluates the transforms exactly as that recipe defines them, the others
 * through the hardware's log2 / sin / cos (within 1e-6 of it).  With TRT
 * the parts of eta even and odd under e -> -e relax at omega = 1/tau and
 * 1/tau_minus, and each takes its own rate's amplitude:
 * zeta = amp+ (eta_s - w S) + amp- (eta_a - 3 w e.V).  The lattice must
 * have fewer than 2^32 nodes (LB_EUNSUPPORTED).
 * Same conventions as above: caller-owned 256-byte aligned workspace,
 * stream-ordered calls, errors through lb_last_error.  No particles. */
#define LB3_BGK 0
#define LB3_TRT 1
#define LB3_D3Q19 0
#define LB3_D3Q27 1
typedef struct lb3_domain_desc {
  uint32_t abi_version;        /* LB_ABI_VERSION                                  */
  int32_t nx, ny, nz;          /* each in [3, 4096]; rows padded to a pitch of nx */
                               /* rounded up to 64 nodes                          */
  int32_t wall_x, wall_y, wall_z;  /* nonzero: the outermost planes are solid    */
  int32_t storage;             /* LB_F64 | LB_F32 | LB_F16_DELTA | LB_BF16_DELTA  */
  int32_t obstacles;           /* nonzero: lb3_set_obstacles may be called        */
  int32_t init_kind;           /* LB_INIT_REST | LB_INIT_FIELDS                   */
  double rho0, tau;            /* reference density (> 0), relaxation time (> 1/2) */
  double gx, gy, gz;           /* body acceleration                               */
  const double *init_rho, *init_ux, *init_uy, *init_uz;  /* host [nz][ny][nx], copied */
  int32_t collision;           /* LB3_BGK | LB3_TRT                               */
  double magic;                /* TRT: (tau - 1/2)(tau_minus - 1/2), > 0          */
  int32_t rounding;            /* LB_ROUND_NEAREST | LB_ROUND_STOCHASTIC (16-bit) */
  uint64_t seed;               /* stochastic-rounding and noise key               */
  int32_t lattice;             /* LB3_D3Q19 | LB3_D3Q27                           */
  int32_t power_law;           /* nonzero: local tau* (Sec. 5), tau unused        */
  double n_index, K;           /* power-law index n and consistency xi            */
  double tau_min, tau_max;     /* clamp of tau*, 1/2 < tau_min <= tau_max         */
  double kT;                   /* thermal energy k_B T >= 0; 0 disables noise     */
} lb3_domain_desc;
typedef struct lb3_domain lb3_domain;

lb_status lb3_workspace_bytes(const lb3_domain_desc *desc, size_t *bytes);
/* Create and initialise (equilibrium of the fields, then one collision). */
lb_status lb3_create_domain(const lb3_domain_desc *desc, void *dev_workspace, size_t bytes,
                            void *hip_stream, lb3_domain **out);
/* Solid nodes: host mask [nz][ny][nx], nonzero = solid (walls stay solid). */
lb_status lb3_set_obstacles(lb3_domain *d, const uint8_t *host_mask, size_t n);
/* Enqueue nsteps steps (one sweep launch per step); nsteps >= 0. */
lb_status lb3_step(lb3_domain *d, int64_t nsteps);
/* rho and u = j/rho + g/2 at every node (zero on solids), host FP64
 * [nz][ny][nx] each.  Synchronises; LB_EUNSTABLE after a non-finite state. */
lb_status lb3_moments(lb3_domain *d, double *rho, double *ux, double *uy, double *uz);
/* Post-collision deviations, host FP64 [q][nz][ny][nx].  Synchronises. */
lb_status lb3_get_populations(lb3_domain *d, double *host_dev_f);
/* FP64 sum of rho over the non-solid nodes (fixed order).  Synchronises. */
lb_status lb3_mass(lb3_domain *d, double *total);
lb_status lb3_time(lb3_domain *d, int64_t *t);
/* The sweep addresses populations with 32-bit byte offsets while the 19
 * population planes of one buffer stay below 2^32 bytes, with 64-bit offsets
 * above.  value 1 forces the 64-bit form on any lattice (the two give
 * identical states; for testing), 0 restores the 32-bit form where it
 * applies (LB_EINVAL where the buffer is too large for it). */
#define LB3_OPT_WIDE_OFFSETS 1
lb_status lb3_set_option(lb3_domain *d, int32_t option, int64_t value);
lb_status lb3_destroy_domain(lb3_domain *d);

const char *lb_status_string(lb_status s);
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LB_H */
