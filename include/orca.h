/*
 * orca.h -- C ABI of the MI355X (gfx950) ORCA step library, liborca.so.
 *
 * The library advances crowds of pedestrians and vehicles by one ORCA step
 * ("Simulating Crowds and Autonomous Vehicles", Charlton, Montana Gonzalez,
 * Maddock, Richmond):
 *   1. uniform-grid spatial partition of the agents (Sec. 1, Sec. 3),
 *   2. each agent's k nearest neighbours within the neighbour distance
 *      (Sec. 3: every agent observes the radius, position and velocity of
 *      nearby agents; Sec. 5: fewer neighbours trade realism for memory),
 *   3. one ORCA half-plane per neighbour, shifted by the responsibility
 *      factor f_{A|B} (Fig. 1(b,c), Sec. 3.1),
 *   4. one small 2D linear program per agent for the permitted velocity
 *      closest to the desired one (Sec. 3), with the least-penetration
 *      fallback when the half-planes leave nothing permitted (Sec. 3),
 *   5. explicit Euler update of every agent from the same step-t state.
 *
 * Conventions shared by all entry points
 *  - Agent arrays are structure-of-arrays, FP32 (class: uint8), length n,
 *    in the caller's order, and are DEVICE pointers unless stated.
 *  - Agent class 0 is a pedestrian, 1 a vehicle; f[c_self][c_other] is the
 *    responsibility agent c_self takes for avoiding c_other.  The paper's
 *    values are f = {{1/2, 1}, {0, 1/2}} (person-person 1/2, person-car 1,
 *    car-person 0, car-car 1/2).  All classes run the same code path.
 *  - The caller owns every buffer, including the workspace; no entry point
 *    allocates, frees or synchronises.  Work is enqueued on `stream` and
 *    results are visible in stream order.  Entry points are safe to call
 *    concurrently on different streams with different workspaces.
 *  - A workspace must be zero-filled once before its first use (for example
 *    with orca_workspace_init); the library keeps it reusable after that.
 *  - Errors: every function returns ORCA_OK (0) or a negative ORCA_E* code.
 *    Arguments are validated on the host before anything is enqueued; on an
 *    error nothing is enqueued.  n == 0 is a no-op that returns ORCA_OK.
 *    NaN/Inf inside agent arrays are not checked and propagate.
 */
#ifndef ORCA_H
#define ORCA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORCA_OK 0
#define ORCA_EINVAL (-1)     /* null pointer, negative size, bad parameter */
#define ORCA_EWORKSPACE (-2) /* workspace smaller than orca_workspace_bytes() */
#define ORCA_EHIP (-3)       /* a HIP launch reported an error */
#define ORCA_ERANGE (-4)     /* max_neighbors outside 1..ORCA_K_MAX */
#define ORCA_ETOOBIG (-5)    /* more agents than orca_step_noalloc's scratch holds */

#define ORCA_K_MAX 32
#define ORCA_N_MAX 268435456  /* agents per call (2^28) of the neighbour search */

/* Per-agent inputs (device pointers, length n, caller order).
 * pref_x/pref_y hold the goal position when orca_params.pref_is_goal is 1
 * (desired velocity = (goal - p) * min(max_speed/|goal - p|, 1/dt), zero at
 * the goal; Sec. 3, Sec. 4) and the desired velocity itself otherwise. */
typedef struct {
    const float *px, *py;          /* position [m] */
    const float *vx, *vy;          /* current velocity [m/s], used as v_opt */
    const float *pref_x, *pref_y;  /* goal [m] or desired velocity [m/s] */
    const float *radius;           /* disc radius [m] */
    const float *max_speed;        /* speed cap [m/s] */
    const uint8_t *cls;            /* 0 pedestrian, 1 vehicle */
} orca_agents_in;

/* Per-agent outputs (device pointers, length n, caller order).  They may
 * alias the corresponding inputs (in-place step).  status is optional
 * (NULL): 1 where the least-penetration fallback was used, else 0. */
typedef struct {
    float *px, *py, *vx, *vy;
    uint8_t *status;
} orca_agents_out;

/* Scalar parameters of one scene (host memory for orca_step and
 * orca_build_grid; device memory, one per scene, for orca_step_batched). */
typedef struct {
    float dt;             /* step [s], > 0 */
    float time_horizon;   /* look-ahead tau [s], > 0 (Sec. 3) */
    float neighbor_dist;  /* neighbour range R_n [m], > 0 (strict: dist < R_n) */
    float cell_size;      /* grid cell [m]; 0 selects the library default */
    int32_t max_neighbors;/* k, 1..ORCA_K_MAX */
    int32_t pref_is_goal; /* 1: pref_* are goals, 0: desired velocities */
    float f[2][2];        /* responsibility f[class_self][class_other] (Sec. 3.1) */
    float par_eps;        /* parallel-line tolerance of the LP, e.g. 1e-5 */
    float accel[2];       /* acceleration cap per class [m/s^2], >= 0; 0 = none.
                             Sec. 5 names acceleration-limited vehicles as an
                             extension adding linear constraints of the agent's
                             own motion to the same LP.  With a > 0 the new
                             velocity must lie in the regular octagon inscribed
                             in the disc of radius a*dt about the current
                             velocity (scaled onto the speed circle first when
                             outside it); its 8 edges are hard constraints:
                             they precede the ORCA lines in LP2 and LP3 never
                             relaxes them.  (Should LP2 fail on them, which
                             only rounding can cause, the octagon's centre is
                             taken.)  orca_step_backward differentiates the
                             octagon through its centre (a and dt are
                             constants). */
    float turn[2];        /* turn-rate cap per class [rad/s], >= 0; 0 = none.
                             The non-holonomic half of the same Sec. 5
                             extension: a vehicle moves along its heading (the
                             direction of its current velocity) and turns it by
                             at most turn*dt per step, so the new velocity must
                             lie in the wedge of half-angle
                             phi = min(turn*dt, pi/2) about the heading, apex
                             at the origin.  The wedge's two sides are hard
                             lines after the acceleration lines.  An agent at
                             rest has no heading and no wedge.
                             orca_step_backward differentiates the wedge
                             through the heading v/|v| (turn and dt are
                             constants). */
} orca_params;

/* Bytes of workspace needed for n agents (plain step / grid), or for a
 * batch whose total agent count is n and scene count n_scenes (batched step;
 * pass n_scenes = 0 for the plain step).  For the plain step max_cells bounds
 * the grid cells (0 selects a default of max(2n, 4096)); a batch always gets
 * 2 cells per agent plus 64 per scene (max_cells ignored).  When a scene's
 * bounding box would need more cells the library enlarges the cell size on
 * the device. */
size_t orca_workspace_bytes(int32_t n, int32_t n_scenes, int32_t max_cells);

/* Zero-fills a workspace on `stream` (a fill kernel, no memset node). */
int orca_workspace_init(void *ws, size_t ws_bytes, hipStream_t stream);

/* Builds the grid and the exact neighbour lists (no velocity update).
 * nbr (n x k, row-major, nullable): caller indices of the k nearest agents
 * j != i with |p_j - p_i|^2 < R_n^2, ascending in (squared distance, j),
 * padded with -1; the squared distance is evaluated in double from the FP32
 * positions without fused multiply-add, so lists are exactly reproducible.
 * nbr_count (n, nullable): number of valid entries per agent. */
int orca_build_grid(const orca_agents_in *in, int32_t n, const orca_params *params,
                    void *ws, size_t ws_bytes, int32_t *nbr, int32_t *nbr_count,
                    hipStream_t stream);

/* One ORCA step of one scene (grid, neighbours, half-planes, LP, update). */
int orca_step(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
              const orca_params *params, void *ws, size_t ws_bytes, hipStream_t stream);

/* Optional HIP events recorded on `stream` around the phases of one step
 * (any may be NULL): before the grid build, between the grid build and the
 * fused neighbour/half-plane/LP kernel, and after that kernel.  For timing
 * only; they do not change the computation. */
typedef struct {
    hipEvent_t grid_begin;
    hipEvent_t step_begin;
    hipEvent_t step_end;
} orca_step_events;

/* orca_step with phase events (events may be NULL: then identical to
 * orca_step). */
int orca_step_ex(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                 const orca_params *params, void *ws, size_t ws_bytes,
                 const orca_step_events *events, hipStream_t stream);

/* orca_step that also writes the neighbour lists this step used, in the
 * format of orca_build_grid: nbr (n x max_neighbors, row-major, nullable)
 * the caller indices of each agent's nearest neighbours, ascending in
 * (squared distance, index), padded with -1; nbr_count (n, nullable) their
 * number.  The step itself (outputs, and what the workspace keeps for the
 * next step) is the same as orca_step's, bit for bit; the lists are those
 * of the selection narrowed by the distances the workspace kept from the
 * previous step, which must equal orca_build_grid's exact lists.  For
 * checking and inspection (Sec. 3: each agent observes its nearby agents). */
int orca_step_nbr(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                  const orca_params *params, void *ws, size_t ws_bytes, int32_t *nbr,
                  int32_t *nbr_count, hipStream_t stream);

/* Description of a batch of independent scenes for orca_step_batched.
 * Scene s owns the agents [scene_off[s], scene_off[s+1]) of the agent arrays
 * and uses params[s]; agents of different scenes never interact.  This
 * batched form is not part of the paper (which simulates one scene); it runs
 * every scene of a step in one set of launches. */
typedef struct {
    const int32_t *scene_off;     /* DEVICE, n_scenes + 1 entries, ascending,
                                     scene_off[0] = 0, scene_off[n_scenes] = n */
    int32_t n_scenes;             /* >= 1 */
    const orca_params *params;    /* DEVICE, n_scenes entries (cell_size 0 = R_n) */
    int32_t max_neighbors;        /* HOST: largest max_neighbors over the scenes,
                                     1..ORCA_K_MAX (selects the compiled kernel) */
    int32_t mode;                 /* 0: persistent kernel with per-XCD tile queues
                                     (default); 1: one workgroup per tile */
    int32_t *error_flag;          /* DEVICE, nullable: set to 1 (never cleared) when
                                     an offset or a scene's parameters are invalid
                                     (including an accel or turn cap > 0 while
                                     has_accel is 0); the kernels clamp every
                                     index regardless */
    int32_t has_accel;            /* HOST: 1 if any scene has accel[c] > 0 or
                                     turn[c] > 0 (selects the kernel with hard
                                     lines; without it caps are ignored and
                                     flagged), else 0 */
    int32_t block;                /* HOST: lanes per workgroup of the step kernel,
                                     64, 128 or 256 (1, 2 or 4 wavefronts); 0 = 128 */
    int32_t k_tile;               /* HOST: neighbour-list capacity compiled into the
                                     step kernel, max_neighbors..ORCA_K_MAX, rounded
                                     up to a compiled one (4, 8, 10, 12, 16, 20, 24,
                                     32); 0 = the smallest that holds max_neighbors.
                                     Results do not depend on it (the k nearest are
                                     the first k of any larger nearest set). */
} orca_batch;

/* One ORCA step of every scene of a batch.  n is the total agent count; the
 * workspace must hold orca_workspace_bytes(n, batch->n_scenes, 0) bytes.
 * Each scene's result equals orca_step on that scene alone (same neighbour
 * lists and velocities, bit for bit). */
int orca_step_batched(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                      const orca_batch *batch, void *ws, size_t ws_bytes, hipStream_t stream);

/* orca_step_batched with phase events (any may be NULL): before the batch's
 * grid build, before its step kernel, after it.  Timing only. */
int orca_step_batched_ex(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                         const orca_batch *batch, void *ws, size_t ws_bytes,
                         const orca_step_events *events, hipStream_t stream);

/* Cotangents (gradients of a scalar loss) of an agent state, device
 * pointers, length n, caller order. */
typedef struct {
    const float *px, *py, *vx, *vy;
} orca_cotangents;

/* Outputs of orca_step_backward: px..vy are overwritten with the cotangents
 * of the step-t state (they may alias the inputs of orca_cotangents);
 * pref_x / pref_y (cotangents of the pref input: the desired velocity, or
 * the goal in goal mode) are ACCUMULATED (+=); tau (nullable, one device
 * float) is accumulated with the cotangent of the shared look-ahead time. */
typedef struct {
    float *px, *py, *vx, *vy;
    float *pref_x, *pref_y;
    float *tau;
} orca_cotangents_out;

/* Workspace bytes of orca_step_backward for n agents (max_cells as for
 * orca_workspace_bytes). */
size_t orca_backward_workspace_bytes(int32_t n, int32_t max_cells);

/* Adjoint (vector-Jacobian product) of orca_step at state `in` (the
 * differentiable form; not in the paper).  Given the cotangents g1 of the
 * step's outputs (p' = p + v' dt, v'), writes the cotangents of p and v and
 * accumulates those of the pref input and tau.  The step is recomputed
 * exactly (same neighbours, half-planes and LP); neighbour sets and all
 * branch decisions are held fixed, and the LP result is differentiated
 * through its active constraints (implicit differentiation).  Contributions
 * to neighbours are gathered in a fixed order, so results are
 * bit-reproducible.  Radii, speed caps, f and dt are constants. */
int orca_step_backward(const orca_agents_in *in, int32_t n, const orca_params *params,
                       const orca_cotangents *g1, const orca_cotangents_out *g0, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/* orca_step_backward with phase events (any may be NULL): before the grid
 * build, before the per-agent adjoint kernel (recomputation and VJP), after
 * it (the transpose gather and the tau sum follow).  Timing only. */
int orca_step_backward_ex(const orca_agents_in *in, int32_t n, const orca_params *params,
                          const orca_cotangents *g1, const orca_cotangents_out *g0, void *ws,
                          size_t ws_bytes, const orca_step_events *events, hipStream_t stream);

/* ---- Agent lifecycle (Sec. 4, first experiment) -------------------------
 * In the crossing experiments agents are spawned in start regions at points
 * that keep clear of everyone for a while, walk to a goal in the matching
 * end region, and leave the simulation once they reach it.  The two entry
 * points below implement the leaving and the entering between steps. */

/* A writable agent state (device pointers, length = capacity, caller order). */
typedef struct {
    float *px, *py, *vx, *vy, *pref_x, *pref_y, *radius, *max_speed;
    uint8_t *cls;
} orca_agents_buf;

/* Largest number of spawn candidates one orca_spawn call accepts. */
#define ORCA_SPAWN_MAX 16384

/* Workspace bytes of orca_remove_arrived and orca_spawn for up to n agents
 * and n_cand spawn candidates (zero-filled once, like every workspace). */
size_t orca_lifecycle_workspace_bytes(int32_t n, int32_t n_cand);

/* Removes every agent whose goal (pref_x, pref_y, read as a goal position)
 * lies inside or on its disc, |g - p|^2 <= r^2 (evaluated in double from the
 * FP32 values, each operation rounded separately), and writes the others, in
 * their order, to out[0 .. *n_alive).  out must not overlap in.  n_alive
 * (DEVICE, one int32) receives the count; old_to_new (DEVICE, n entries,
 * nullable) the new index of every agent or -1.  With n == 0 the agent
 * arrays may be null and *n_alive is set to 0. */
int orca_remove_arrived(const orca_agents_in *in, const orca_agents_buf *out, int32_t n,
                        int32_t *n_alive, int32_t *old_to_new, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* Spawns agents.  Candidates cand[0 .. n_cand) (device arrays; all nine
 * fields, as the new agents' initial state) are taken in their order; a
 * candidate enters when, for every agent present -- the n agents of `state`
 * and the candidates that entered before it --
 *     |p_c - p_j|^2 >= D^2,   D = (r_c + r_j) + t_clear (s_c + s_j)
 * (s = max_speed; double from the FP32 values, operations rounded
 * separately in this order): the two cannot touch within t_clear seconds
 * even heading straight for each other at full speed.  Accepted candidates
 * are appended, in order, at state[n ...]; capacity (the length of the state
 * arrays) must be at least n + n_cand.  n_total (DEVICE, one int32) receives
 * n plus the number accepted; accepted (DEVICE, n_cand bytes, nullable) the
 * decision per candidate.  n_cand <= ORCA_SPAWN_MAX; t_clear >= 0.  The
 * candidate arrays may be null when n_cand == 0, the state arrays when
 * n + n_cand == 0; *n_total is written in every case. */
int orca_spawn(const orca_agents_buf *state, int32_t n, int32_t capacity,
               const orca_agents_in *cand, int32_t n_cand, float t_clear, int32_t *n_total,
               uint8_t *accepted, void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of orca_overlap_stats for n agents. */
size_t orca_overlap_workspace_bytes(int32_t n);

/* Collision statistics of a crowd (the measure of the crossing experiments,
 * Sec. 4), over the pairs closer than `reach` (|p_i - p_j|^2 < reach^2;
 * reach >= twice the largest radius covers every overlap), in double from
 * the FP32 positions and radii: out[0] = pairs whose discs overlap,
 * |p_i - p_j|^2 < (r_i + r_j)^2; out[1] = agents in at least one such pair;
 * out[2] = the smallest clearance |p_i - p_j| - (r_i + r_j) (+inf when no
 * pair is that close).  out: DEVICE, 3 doubles, written in stream order
 * (also for n == 0).  reach > 0. */
int orca_overlap_stats(const orca_agents_in *in, int32_t n, float reach, double *out, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/* ---- Stepping without a caller-provided workspace ------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * orca_step_noalloc is orca_step with the workspace replaced by a fixed
 * scratch array inside the library, ORCA_NOALLOC_BYTES bytes of device
 * memory per GPU, held from the first call on that GPU until the process
 * ends.  It allocates and frees nothing.  The first call on a GPU looks the
 * array up for that GPU and clears it with a fill kernel on `stream`; every
 * call uses the array of the current device.
 *  - n <= ORCA_NOALLOC_N_MAX, else ORCA_ETOOBIG (nothing is enqueued).
 *  - Results equal orca_step's on a workspace of orca_workspace_bytes(n, 0,
 *    0) bytes, bit for bit.
 *  - Every call on one GPU shares that GPU's array, which keeps the last
 *    call's contents (only the kept neighbour distances carry over, and they
 *    never change a result).  Calls that overlap on one GPU -- on different
 *    streams, or from different threads without ordering -- race on it and
 *    give undefined results: serialise them on one stream. */
#define ORCA_NOALLOC_N_MAX 262144
#define ORCA_NOALLOC_BYTES (16u << 20)

int orca_step_noalloc(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                      const orca_params *params, hipStream_t stream);

/* Human-readable text for a status code (static storage). */
const char *orca_status_string(int code);

/* Version string of the library build. */
const char *orca_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ORCA_H */
