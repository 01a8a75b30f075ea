/*
 * mrpsim — spectral kinetic simulation of the ideal Multipole Resonance Probe
 * (Gong, Friedrichs, Oberrath, Brinkmann, arXiv:2111.13072) on one MI355X.
 *
 * C ABI of the HIP library libmrpsim.so.  Plain pointers and sizes only.
 *
 * Units are the paper's dimensionless ones (Sec. 4): lengths in the probe
 * radius R, times in 1/omega_pe, charges in e, masses in m_e, densities in
 * n_inf, potentials in e n_inf R^2 / eps0.  Particles are electrons (q = -1,
 * m = 1) and, in batch members, optionally mobile ions (q = +1, mass m_i);
 * ions not simulated as particles are an immobile background, uniform or a
 * radial profile.
 *
 * Device memory: a handle makes one device allocation at creation, through
 * the caller's sim_allocator (e.g. a framework's caching allocator) or
 * hipMalloc, and frees it in sim_destroy.  Every other call allocates no
 * device memory.
 *
 * Error convention: every int-returning call returns SIM_OK (0) or a
 * negative SIM_E* code; no exception crosses the ABI.  A handle whose device
 * work failed enters a failed state and answers SIM_ESTATE afterwards.
 * sim_last_error() gives a human-readable message for the calling thread.
 *
 * Threading: one handle must not be used from two threads at once; distinct
 * handles are independent.
 */
#ifndef MRPSIM_H
#define MRPSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim sim_t;

/*
 * Device memory provider.  alloc returns `bytes` of device memory on the
 * current device, 256-byte aligned, or NULL on failure; free releases it.
 * `stream` is the hipStream_t given at creation, the one the memory is used
 * on, or NULL when the handle runs on a stream of its own (created after the
 * allocation; the memory is used on that stream only).  The library calls
 * alloc once, at creation, and free once, in sim_destroy after all of the
 * handle's work has completed, with the same size and stream.  ctx is passed
 * through.  A NULL sim_allocator means hipMalloc / hipFree.
 */
typedef struct {
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, size_t bytes, void *stream);
    void *ctx;
} sim_allocator;

enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,   /* invalid parameter or particle state */
    SIM_ENOMEM = -2,   /* device allocation failed or mem_limit_bytes exceeded */
    SIM_ERANGE = -3,   /* step or response index outside [0, n_steps) */
    SIM_ESTATE = -4,   /* NULL, destroyed or failed handle */
    SIM_EDEVICE = -5   /* a HIP runtime call failed */
};
enum { SIM_BUSY = 1 };   /* sim_query only: work still running */

enum { SIM_M_FULL = 0, SIM_M_AXISYM = 1 };
enum { SIM_BC_ABSORB = 0, SIM_BC_SPECULAR = 1, SIM_BC_DIFFUSE = 2 };
enum { SIM_FP64 = 0, SIM_FP32_COMP = 1 };

/*
 * Simulation parameters.
 *   d, eps_r    dielectric cover: thickness / R and permittivity; the
 *               electrodes have radius a = 1 - d (Sec. 2).
 *   r_out       outer wall of the particle domain (units of R); the field
 *               domain itself is unbounded (potential -> 0 at infinity).
 *   dt          leapfrog time step (units of 1/omega_pe).
 *   ntilde      super-particles per unit volume R^3 (Sec. 4).
 *   ion_density immobile uniform ion background filling 1 < r < r_out.
 *   q_surface0  initial homogeneous surface charge Q_S (units of the
 *               super-particle charge; absorbed electrons add -1 each).
 *   l_max       truncation of the projection P^: 0 <= l <= l_max (Sec. 3).
 *   m_mode      SIM_M_FULL: all m; SIM_M_AXISYM: m = 0 only (the paper's
 *               dipole kernel of Sec. 3 is l_max = 1, SIM_M_AXISYM).
 *   probe_bc    at r <= 1: absorb (charge goes to Q_S), specular or diffuse.
 *   wall_bc     at r >= r_out: specular or diffuse.
 *   precision   SIM_FP64, or SIM_FP32_COMP: the field evaluation (far-field
 *               harmonics and contraction, near-field pair sums) in FP32 at
 *               tile-scaled coordinates, compensated where a rounding would
 *               act coherently (r^2 and z as hi + lo pairs in the
 *               recurrences, per-m factors and coefficients rounded once from
 *               FP64), with FP64 moments, radial scans, l = 0 (Gauss) term,
 *               pair-sum accumulation, positions and velocities; from
 *               l_max 20 the near-field pair sums run in FP64 too.  Field
 *               error against the FP64 definition: <= 1e-5 of the RMS field
 *               on every tested input up to l_max 64 (FP64: <= 1e-12).
 *   tile        particles per tile of the radial scan: 0 or 64.
 *   seed        key of the counter-based generator of diffuse walls.
 *   mem_limit_bytes  0 = none; otherwise sim_create fails with SIM_ENOMEM
 *               when sim_footprint_bytes exceeds it.
 */
typedef struct {
    uint32_t struct_size; /* sizeof(sim_params) */
    uint32_t reserved0;
    double d;
    double eps_r;
    double r_out;
    double dt;
    double ntilde;
    double ion_density;
    double q_surface0;
    int32_t l_max;
    int32_t m_mode;
    int32_t probe_bc;
    int32_t wall_bc;
    int32_t precision;
    int32_t tile;
    uint64_t seed;
    uint64_t mem_limit_bytes;
    /* Launch sizes that leave the results unchanged up to the rounding order
     * of the radial carries (the autotuner's knobs; 0 = built-in choice):
     * sort_bucket: mean particles per radial sort bucket, 1..256 (built-in 8);
     * carry_chunk: groups of 256 particle slots per carry chunk, 8..1024
     * (built-in: a power of two in [8, 64], about a member's groups / 256);
     * sort_keys: where the next step's radial sort keys and bucket slots
     * are taken: 1 in the tail of the push, -1 in a pass of their own, 0 by
     * launch size (the push from 2048 tiles of 64 particles on).  Results
     * are bit-identical either way.
     * near_split: the near field's pair sums run over blocks of 32 radially
     * consecutive particles (1) or 64 (-1), the pairs across blocks through
     * the radial scan; 0: by member, 32 in FP64 and, in FP32, where
     * l_max^2 <= sqrt(n) (a close pair's force, about l_max^2 / sqrt(n) of the
     * RMS field, keeps FP32 relative precision only inside a block).  The
     * same sum split differently: results agree to rounding. */
    int32_t sort_bucket;
    int32_t carry_chunk;
    int32_t sort_keys;
    int32_t near_split;
} sim_params;

/* Fill *p with the defaults (d = 0.25, eps_r = 4, r_out = 5, dt = 0.05,
 * ntilde = 1, ion_density = 1, l_max = 8, FULL, absorb / specular, FP64). */
void sim_params_default(sim_params *p);

/*
 * Create a simulation and upload its state: the problem of Sec. 4 (the
 * probe geometry of Sec. 2, the plasma as super-particles of density
 * ntilde, an initial particle state and the antisymmetric drive u_asy(t)),
 * in the canonical variables of Sec. 2 (positions, and velocities half a
 * step behind for the leapfrog).
 *   n          number of electrons (> 0).
 *   pos, vel   host arrays [3n], particle-major (x0,y0,z0,x1,...); vel is the
 *              leapfrog half-step velocity v(t_start - dt/2).  Every particle
 *              must satisfy 1 < r < r_out.  Copied; the caller keeps them.
 *   ids        host array [n] of distinct ids, or NULL for 0..n-1.  Ids break
 *              ties of equal radius in the radial order (key (r^2, id)).
 *              sim_create simulates electrons only: ids must have bit 31
 *              clear (batch members may carry mobile ions, see sim_member).
 *   u_asy      host array [n_steps]: antisymmetric electrode voltage
 *              u_1 - u_2 at t_s = s dt (Sec. 3); copied.
 *   start_step first step to run (checkpoint resume); 0 <= start_step <= n_steps.
 *   hip_stream hipStream_t to run on, or NULL for a stream of the handle's own.
 *   alloc      device memory provider, or NULL for hipMalloc.
 * Returns SIM_EINVAL for invalid parameters or particles, SIM_ENOMEM when the
 * footprint exceeds mem_limit_bytes or the allocation fails.
 */
int sim_create(const sim_params *p, int64_t n, const double *pos, const double *vel,
               const uint32_t *ids, const double *u_asy, int64_t n_steps, int64_t start_step,
               void *hip_stream, const sim_allocator *alloc, sim_t **out);

/*
 * Enqueue k time steps (asynchronous, on the handle's stream).  One step is
 * the scheme of Sec. 3-4: radial sort, harmonic moments, prefix/suffix scans,
 * boundary response + drive, field and leapfrog push with the wall rules;
 * Q_diff(t_s) (Sec. 4) is recorded before the push.  SIM_ERANGE if the steps
 * would pass n_steps of any member.
 */
int sim_step(sim_t *h, int64_t k);

/* Wait for all enqueued work of the handle. */
int sim_sync(sim_t *h);

/*
 * Non-blocking check of the handle's enqueued work: SIM_OK when all of it has
 * completed, SIM_BUSY (positive, not an error) while some still runs, a
 * negative code if the device reported a failure (the handle then fails as
 * after sim_sync).  Lets a host loop that drives several handles, such as a
 * server with one resident batch per class, tend whichever finishes first
 * without waiting on the others.
 */
int sim_query(sim_t *h);

/*
 * Copy Q_diff[first .. first+count) to host (synchronises).  Q_diff(t_s) =
 * -(1/ntilde) sum_i q_i Psi_anti,L(x_i(t_s)) (Sec. 4, odd l <= l_max), in
 * units of e n_inf R^3.  SIM_ERANGE if any index is not yet computed.
 */
int sim_read_response(sim_t *h, int64_t first, int64_t count, double *q_diff);

/*
 * Copy the state at the current step boundary to host (synchronises): the
 * canonical variables of Sec. 2 (positions and leapfrog half-step
 * velocities) and the surface charge Q_S of Sec. 2-3, in the
 * order of the arrays given to sim_create.  pos/vel [3n] (vel = v at t - dt/2),
 * alive [n] (0 = absorbed; its pos/vel are those at absorption), q_surface
 * and step may each be NULL.
 */
int sim_read_state(sim_t *h, double *pos, double *vel, uint8_t *alive, double *q_surface,
                   int64_t *step);

/*
 * Electric field E = -grad Phi at every alive particle for the current state
 * and step (Sec. 3 modified potential, truncated at l_max), in the order of
 * the creation arrays, [3n]; zero for absorbed particles.  Does not advance
 * the simulation.  Synchronises.  The evaluation sorts the state itself,
 * using up the sort keys the last step prepared, so the next step computes
 * them again (one extra pass over the particle records).
 */
int sim_eval_field(sim_t *h, double *E);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the field
 * evaluation of sim_eval_field for a state given in device memory, with no
 * handle and no allocation.  Every working array (sort records, tile sums,
 * carries, coefficients, tables) lives in one static device buffer of
 * 64 MiB per GPU, held until the process ends; sim_eval_field_static_bytes
 * gives the part a call needs, and a call that needs more fails with
 * SIM_ENOMEM (FP64: about 1.7e5 particles at l_max 16, 2.5e5 at l_max 8).
 *   p          as for sim_create (ntilde, ion_density, r_out, ... of the one
 *              simulation; mem_limit_bytes is ignored).
 *   n          particles (electrons), ids 0..n-1 in array order (ties of
 *              equal radius go by index, as sim_create with ids NULL).
 *   pos        DEVICE array [3n], particle-major; every particle must satisfy
 *              1 < r < r_out (not checked: other positions give undefined
 *              fields, never an out-of-bounds access).
 *   q_surface  Q_S, u_asy the drive at the evaluated time.
 *   E          DEVICE array [3n] receiving E at every particle, array order.
 *   hip_stream stream to run on (NULL: the null stream).
 * Synchronises the stream before returning.  The buffer is shared by every
 * call on a GPU and keeps the last call's contents (the call clears what
 * must start at zero): calls that overlap on one GPU, from two threads or on
 * two streams, race.
 */
int sim_eval_field_static(const sim_params *p, int64_t n, const double *pos, double q_surface,
                          double u_asy, double *E, void *hip_stream);
int64_t sim_eval_field_static_bytes(const sim_params *p, int64_t n);

/*
 * Run k steps with a HIP event around every kernel and return the average
 * duration in milliseconds of each kernel kind (indices as sim_kernel_name).
 * kernel_ms has n_kernels entries; entries beyond sim_num_kernels() are left
 * untouched.  Advances the simulation by k steps.
 */
int sim_profile(sim_t *h, int64_t k, double *kernel_ms, int32_t n_kernels);
int32_t sim_num_kernels(void);
const char *sim_kernel_name(int32_t i);

/* Device bytes sim_create would allocate (for admission control); < 0 on
 * invalid parameters. */
int64_t sim_footprint_bytes(const sim_params *p, int64_t n, int64_t n_steps);

/* Particle count, tile size and channel count actually used (member 0). */
int sim_info(sim_t *h, int64_t *n, int32_t *tile, int32_t *channels);

void sim_destroy(sim_t *h);

/*
 * Batches: one handle stepping many independent simulations ("members") in
 * the same kernel launches.  Independent runs of the method (Sec. 4: every
 * plasma and drive is its own run) share the probe (d, eps_r), l_max, m_mode
 * and precision; everything else is per member.  A member's results do not
 * depend on the other members: they equal, bit for bit, those of the same
 * member run alone.  A handle from sim_create is a batch of one member
 * (index 0), so every sim_member_* call also applies to it.
 *
 * Each member occupies ceil(n/256) groups of 256 particle slots (four tiles
 * of 64), ceil(groups / carry_chunk) carry chunks (built-in: 8 to 64 groups
 * each) and max(1, n/8) sort buckets of the handle's capacity, and
 * sim_member_data_bytes(n_steps, ion_profile_len) bytes of the batch's
 * member data pool (its drive, response and ion profile).  Admission and
 * retirement take and return these ranges without any device allocation.
 */
typedef struct {
    uint32_t struct_size;  /* sizeof(sim_member) */
    uint32_t reserved0;
    int64_t n;             /* electrons (> 0) */
    const double *pos;     /* host [3n], as in sim_create; copied */
    const double *vel;     /* host [3n], v(t_start - dt/2); copied */
    const uint32_t *ids;   /* host [n] distinct ids, or NULL for 0..n-1 */
    const double *u_asy;   /* host [n_steps]; copied */
    int64_t n_steps;
    int64_t start_step;    /* 0 <= start_step <= n_steps */
    double ntilde;         /* super-particles per unit volume R^3 */
    double ion_density;
    double q_surface0;
    double r_out;
    double dt;
    uint64_t seed;
    int32_t probe_bc;
    int32_t wall_bc;
    /* Optional immobile ion density (units of n_inf) at ion_profile_len >= 2
     * equally spaced radii from 1 to r_out, linear in between, e.g. the ion
     * profile of the floating equilibrium of App. D; replaces the uniform
     * ion_density when non-NULL.  Copied. */
    const double *ion_profile;
    int64_t ion_profile_len;
    /* m_i / m_e of mobile ions: a particle whose id has bit 31 set is an ion
     * (charge +1, this mass); others are electrons.  Must be > 0 when any id
     * has bit 31 set; ignored otherwise. */
    double ion_mass;
} sim_member;

/* Fill *m with the per-member defaults of sim_params_default (arrays NULL). */
void sim_member_default(sim_member *m);

/*
 * Create a batch.  common supplies d, eps_r, l_max, m_mode, precision, tile
 * and mem_limit_bytes (its per-member fields are ignored).  slot_capacity is
 * the number of particle slots to reserve (0: exactly what the initial
 * members need); max_members the size of the member table (0: n_members);
 * member_data_bytes the size of the member data pool (0: exactly what the
 * initial members need; see sim_member_data_bytes).  members[0 .. n_members)
 * are admitted in order as indices 0, 1, ...  alloc as in sim_create.
 * SIM_EINVAL on invalid parameters or members, SIM_ENOMEM when they do not
 * fit the capacities or the memory limit, or the allocation fails.
 */
int sim_batch_create(const sim_params *common, int64_t slot_capacity, int32_t max_members,
                     int64_t member_data_bytes, int32_t n_members, const sim_member *members,
                     void *hip_stream, const sim_allocator *alloc, sim_t **out);

/* Device bytes of a batch (its one allocation) for these capacities; < 0 on
 * invalid parameters. */
int64_t sim_batch_footprint_bytes(const sim_params *common, int64_t slot_capacity,
                                  int32_t max_members, int64_t member_data_bytes);

/* Bytes a member with n_steps steps and an ion profile of ion_profile_len
 * nodes (0: none) takes of a batch's member data pool; < 0 on negative
 * sizes. */
int64_t sim_member_data_bytes(int64_t n_steps, int64_t ion_profile_len);

/*
 * Admit a member between steps (synchronises the handle's stream).  *index
 * receives its slot in the member table.  SIM_ENOMEM when its tiles, chunks,
 * buckets or member data find no free contiguous range or the member table
 * is full; the handle is unchanged then.  Allocates no device memory.
 */
int sim_batch_add(sim_t *h, const sim_member *m, int32_t *index);

/* Retire a member and give its ranges back (synchronises; no device memory is
 * freed).  Read its results first. */
int sim_batch_remove(sim_t *h, int32_t index);

/*
 * Enqueue k steps of the batch: every member takes min(k, steps left) steps;
 * members that reach their n_steps stop.  Asynchronous.
 */
int sim_batch_step(sim_t *h, int64_t k);

/* Host view of a member, without synchronising: particle count, steps
 * enqueued so far (absolute step after them) and n_steps.  SIM_ERANGE for an
 * unused index. */
int sim_member_info(sim_t *h, int32_t index, int64_t *n, int64_t *step, int64_t *n_steps);

/* Particles of a member still in the domain (*alive) and absorbed by the
 * probe so far (*absorbed, Sec. 2: their charge is on Q_S), and its current
 * step (synchronises; each pointer may be NULL). */
int sim_member_counts(sim_t *h, int32_t index, int64_t *alive, int64_t *absorbed, int64_t *step);

/* As sim_read_response / sim_read_state / sim_eval_field, for one member. */
int sim_member_read_response(sim_t *h, int32_t index, int64_t first, int64_t count,
                             double *q_diff);
int sim_member_read_state(sim_t *h, int32_t index, double *pos, double *vel, uint8_t *alive,
                          double *q_surface, int64_t *step);
int sim_member_eval_field(sim_t *h, int32_t index, double *E);

/* Static text for a status code (SIM_OK, SIM_BUSY or a SIM_E* code). */
const char *sim_strerror(int status);

/* Message of the calling thread's last failure; valid until that thread's
 * next call into the library. */
const char *sim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MRPSIM_H */
