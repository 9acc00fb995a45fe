/*
 * ii_lbm.h -- C ABI of the MI355X (gfx950) implementation of the D2Q9
 * immersed interface-lattice Boltzmann method (II-LBM) of Qin, Kolahdouz &
 * Griffith, "An immersed interface-lattice Boltzmann method for
 * fluid-structure interaction" (arXiv:2003.12186).
 *
 * The library advances, on one GPU, a fluid on a D2Q9 lattice (Sec. 2.2.1)
 * with a closed immersed interface carried by Lagrangian markers:
 *   - the normal part of the interface force enters through the jump of the
 *     distribution functions on every lattice link the interface cuts
 *     ([[f_i]] = w_i G.n / (c_s^2 |dX/ds|), Sec. 3.1 Eq. (32), applied as in
 *     the jump-corrected update of Sec. 3.2 Eq. (47));
 *   - the tangential part is spread with Peskin's four-point delta
 *     (Sec. 3.2 Eq. (46)) into the simple force term of Sec. 2.2.2 Eq. (16);
 *   - marker velocities are interpolated with the same delta and the markers
 *     move with them (Sec. 2.2.2 Eq. (20)).
 * Lattice units throughout: dx = dt = 1 (Sec. 2.2).
 *
 * Conventions shared by every call
 *   - D2Q9 populations are numbered e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0)
 *     e4=(0,-1) e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1).
 *   - Field planes are row-major [ny][nx], x fastest.
 *   - Markers are interleaved (x, y) pairs in FP64, ordered counter-clockwise;
 *     the interior of the closed curve is Omega^- (Sec. 2, Fig. 1).
 *   - All calls return 0 (II_LBM_OK) or a negative error code; none throws.
 *     Errors raised on the device are sticky: they are reported by the next
 *     call that synchronises (markers, fields, diag, cutlinks, sync) and the
 *     handle then refuses further steps (II_LBM_ESTATE) until destroyed;
 *     with isolation on (ii_lbm_set_isolation) an instance's own errors stay
 *     with that instance instead.
 *   - A handle is used by one host thread at a time.  All device work of a
 *     handle is enqueued on the HIP stream given at init.
 */
#ifndef II_LBM_H
#define II_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define II_LBM_OK 0
#define II_LBM_EINVAL (-1)     /* invalid problem or argument */
#define II_LBM_EWORKSPACE (-2) /* workspace missing, misaligned or too small */
#define II_LBM_EDEVICE (-3)    /* a HIP call failed */
#define II_LBM_EUNSTABLE (-4)  /* non-finite state (the run blew up) */
#define II_LBM_EGEOMETRY (-5)  /* markers left the region the kernels support */
#define II_LBM_ESTATE (-6)     /* call on a handle that already failed */
#define II_LBM_ECAPACITY (-7)  /* interface too dense for a tile's chord list */

/* ---- problem description ----------------------------------------------- */
enum { II_LBM_SRT = 0, II_LBM_MRT = 1 };
enum { II_LBM_BC_PERIODIC = 0, II_LBM_BC_WALL = 1, II_LBM_BC_INLET = 2, II_LBM_BC_OUTLET = 3,
       II_LBM_BC_INLET_UNIFORM = 4 };
enum { II_LBM_IF_NONE = 0, II_LBM_IF_MEMBRANE = 1, II_LBM_IF_RIGID = 2, II_LBM_IF_NORMAL = 3 };
/* Force modes (how the interface force enters the fluid):
 *  II      the paper's method: jumps on cut links for the normal part, the
 *          tangential part g_par in the simple force term (Sec. 3.2);
 *  IB      the comparison IB-LBM: the whole force G spread into the simple
 *          force term, no jumps (Sec. 2.2.2, Eqs. (16)-(17)); a membrane's
 *          markers move with the velocity of the distributions after the
 *          step's force, sum e_i f_i + g;
 *  IB_GUO  IB-LBM with Guo's force term (Sec. 2.2.2, the SRT and MRT forms):
 *          compressible equilibrium w_i rho [1 + e.u/c_s^2 + (e.u)^2/(2 c_s^4)
 *          - u.u/(2 c_s^2)] with rho u = sum e_i f_i + g/2; a membrane's
 *          markers move with that velocity taken from the distributions
 *          after the step's force (momentum sum e_i f_i + g):
 *          (sum e_i f_i + 3 g / 2) / rho;
 *  II_GUO  II-LBM with Guo's term of g_par (Sec. 3.2); the markers move with
 *          rho u = sum e_i f_i + g/2.
 * The body force joins g in every mode; direct forcing's u* carries the body
 * force only.  Field readouts report u = sum e_i f_i in every mode. */
enum { II_LBM_FORCE_II = 0, II_LBM_FORCE_IB = 1, II_LBM_FORCE_IB_GUO = 2, II_LBM_FORCE_II_GUO = 3 };
enum { II_LBM_FP32 = 0, II_LBM_FP16 = 1 };
enum { II_LBM_MATH_FP32 = 0, II_LBM_MATH_FP64 = 1 };

/*
 * One simulation instance.
 *  nx, ny       lattice size, 8 <= nx, ny <= 8192.
 *  tau          relaxation time lambda of Sec. 2.2.1 (nu = (tau - 1/2)/3), > 0.5.
 *  collision    II_LBM_SRT (Eq. (14)) or II_LBM_MRT (Eq. (15)).
 *  mrt_s        the nine MRT rates in the moment order (rho, e, eps, jx, qx,
 *               jy, qy, pxx, pxy); all nine zero selects the rates of
 *               Sec. 2.2.1 (1.63, 1.14, 1.92 and 1/tau for the stresses).
 *  bc           x-low, x-high, y-low, y-high side; an axis is periodic on both
 *               sides or on neither.  Non-periodic sides use non-equilibrium
 *               extrapolation from the inward neighbour (as cited in Sec. 4):
 *               WALL (velocity u_wall along the side), INLET (parabola
 *               4 u_max y (H - y) / H^2 with H = ny - 1; x-low only), OUTLET
 *               (zero gradient, the velocity of the inward neighbour; any
 *               side), INLET_UNIFORM (velocity (u_max, 0); x-low only).
 *               Corner nodes follow the y side.
 *  body_force   uniform Eulerian force density added to the force term.
 *  force_mode   II_LBM_FORCE_II, _IB, _IB_GUO or _II_GUO (above).
 *  interface_kind  NONE, MEMBRANE (spring force kappa (X_{k+1} - 2 X_k +
 *               X_{k-1}) / dX^2, Sec. 2.2.2 Eq. (19)) or RIGID (fixed circle
 *               with direct forcing G = U^D - U*, eta = 1, U^D = 0, Sec. 2.2.2
 *               Eq. (18); cut links from the circle's level set, Sec. 3.2) or
 *               NORMAL (fixed circle carrying the prescribed force G = F n per
 *               unit length along its outward normal n, Sec. 4.1; level-set
 *               cut links as for RIGID).
 *  n_markers    3 <= N <= 1<<20 markers.
 *  kappa, dX    spring constant and marker spacing Delta X (> 0, <= 2).
 *  center, radius  the circle (RIGID and NORMAL).
 *  f_normal     F of the NORMAL interface.
 *  geometry     MEMBRANE representation: 0 the closed polygon through the
 *               markers (exact integer crossing tests), 1 the periodic cubic
 *               spline through them (Sec. 3.2 names a cubic spline for
 *               flexible interfaces): normals and |dX/ds| from the spline,
 *               crossings as roots of a cubic per link and segment, [[p]] at
 *               each crossing from the spline normal with G linear between the
 *               markers.  One instance per handle.
 *  body_free, rho_star, spring, damping, presc_amp, presc_umax
 *               a moving RIGID circle (Sec. 2.3; one instance per handle):
 *               body_free bit 0 / 1 / 2 frees x / y / rotation; rho_star is
 *               rho_s / rho_f (> 0 when any axis is free; m = rho_star pi R^2,
 *               I_s = m R^2 / 2); spring[a] and damping[a] act on a free axis
 *               about the initial centre; presc_umax[a] != 0 prescribes axis a
 *               as D_c = -A sin(U_max t / A), U_c = -U_max cos(U_max t / A)
 *               with A = presc_amp[a] (Sec. 4.4).  Direct forcing drives the
 *               markers to U_c + W x (X - X_c); each step ends with the body
 *               update of Sec. 2.3 (F^ext and T^ext with their interior-inertia
 *               terms, velocity, position and angle) on the device.
 *  storage      II_LBM_FP32 or II_LBM_FP16: distributions are stored as
 *               deviations d_i = f_i - w_i rho0 (rho0 = 1).
 *  fp16_log2_scale  FP16 storage holds d_i * 2^-fp16_log2_scale; 0 lets the
 *               library choose it from the initial interface force.
 *  math         arithmetic of the collision: II_LBM_MATH_FP32, or
 *               II_LBM_MATH_FP64 (loads and stores keep the storage type; only
 *               the per-node moments, equilibrium and relaxation run in FP64).
 * Markers must stay at least 3 lattice units from every side of the lattice,
 * and the initial chords X_{k+1} - X_k be at most 4 lattice units long.
 */
typedef struct ii_lbm_problem {
    int32_t nx, ny;
    double tau;
    int32_t collision;
    double mrt_s[9];
    int32_t bc[4];
    double u_max;
    double u_wall[4];
    double body_force[2];
    int32_t interface_kind;
    int32_t force_mode;
    int32_t n_markers;
    double kappa, dX;
    double center[2];
    double radius;
    int32_t storage;
    int32_t fp16_log2_scale;
    int32_t math;
    double f_normal;
    int32_t body_free;
    double rho_star;
    double spring[2];
    double damping[2];
    double presc_amp[2];
    double presc_umax[2];
    int32_t geometry;
} ii_lbm_problem;

/* One cut link (see ii_lbm_cutlinks for which step): the link from source
 * node (x, y) to (x, y) + e_dir crosses the interface; sigma = +1 when it
 * runs from the interior to the exterior and -1 otherwise (Sec. 3.2).  seg is
 * the chord (markers seg, seg+1) for membranes, the marker interval
 * [seg, seg+1] for the rigid circle; q is the fraction along the link to the
 * cut point, theta the fraction along the chord/interval, jp = [[p]] there. */
typedef struct ii_lbm_link {
    int32_t x, y, dir, sigma, seg, inst;
    double q, theta, jp;
} ii_lbm_link;

typedef struct ii_lbm_diag_t {
    int64_t step;          /* steps taken since init */
    double mass;           /* sum of rho over the lattice (FP64) */
    double momentum[2];    /* sum of u = sum_i e_i f_i */
    double area;           /* shoelace area of the marker polygon */
    double force[2];       /* force on the body F = -sum_k G_k dX (Sec. 2.3 Eq. (25)) */
    int32_t n_cut_links;   /* directed (link, chord) crossings, as ii_lbm_cutlinks counts them */
    int32_t error_bits;    /* device error flags (0 when healthy) */
    /* Mean pressure p = rho c_s^2 over the nodes farther than 3 lu from the
     * marker polygon, inside (p_in) and outside (p_out) it, with the node
     * counts: p_in - p_out is the pressure jump across the interface
     * (Sec. 3.1), Laplace's T / R at equilibrium for a tensioned circle.
     * NaN (and count 0) where a side has no such node or there are no
     * markers.  Sums in FP64, in a fixed order. */
    double p_in, p_out;
    int64_t n_in, n_out;
} ii_lbm_diag_t;

typedef struct ii_lbm_handle ii_lbm_handle;

/* State of a moving RIGID circle after the last step (Sec. 2.3), 14 doubles:
 * centre (2), velocity U_c (2), angle theta, angular velocity W, F^ext (2)
 * and T^ext of the last step, acceleration (2), angular acceleration, the
 * step count, and 0.  Synchronises the handle's stream.  EINVAL for an
 * instance whose body does not move.  The checkpoint of ii_lbm_save_state
 * carries this state too. */
int ii_lbm_body(ii_lbm_handle* h, int32_t inst, double* out14);

/* Device bytes that init needs for n_inst instances (problems p[0..n_inst-1]).
 * Pure function of its arguments; no device access. */
int ii_lbm_workspace_size(const ii_lbm_problem* p, int32_t n_inst, size_t* bytes);

/*
 * Creates a handle.
 *  p          n_inst problems (copied).
 *  X0         n_inst host pointers, X0[j] holds 2 * p[j].n_markers doubles
 *             (interleaved, counter-clockwise); copied.
 *  d_workspace device memory of at least ws_bytes = ii_lbm_workspace_size
 *             bytes, 256-byte aligned, owned by the caller and kept alive until
 *             ii_lbm_destroy; NULL makes the library allocate (and free) it.
 *  hip_stream hipStream_t on which all work is enqueued (NULL = default);
 *             membrane handles also create one internal non-blocking stream
 *             (default priority) that the handle's stream joins every step.
 * Several instances advance together and must share storage, math and force
 * mode, and their interfaces one kind (EINVAL otherwise).
 * The fluid starts at rest, f_i = w_i rho0.  Synchronises before returning.
 */
int ii_lbm_init(const ii_lbm_problem* p, int32_t n_inst, const double* const* X0,
                void* d_workspace, size_t ws_bytes, void* hip_stream, ii_lbm_handle** out);

/* Enqueues n_steps time steps of every instance and returns without waiting.
 * For membranes the marker force depends on the positions only, so the
 * geometry and tile pass of step n+1 (at X^{n+1}) runs on an internal stream
 * while the sweep of step n runs on the handle's stream; the handle's stream
 * waits for it before the step ends.  Rigid bodies, whose direct-forcing
 * force needs U^n, run their phases in order on the handle's stream. */
int ii_lbm_step(ii_lbm_handle* h, int64_t n_steps);

/* Waits for the handle's stream and reports sticky device errors. */
int ii_lbm_sync(ii_lbm_handle* h);

/* Synchronises, then copies 2N doubles each of the current marker positions
 * X^n, of the velocity U^{n-1} that moved them there, and of the force G
 * (membranes: G^n at the current positions; rigid bodies: the direct forcing
 * of the last step) into caller-owned host buffers (any may be NULL). */
int ii_lbm_markers(ii_lbm_handle* h, int32_t inst, double* X, double* U, double* G);

/* Replaces the marker positions of one instance (2N doubles, host) and, for
 * membranes, rebuilds the force, cut links and tile corrections of the
 * current step from them. */
int ii_lbm_set_markers(ii_lbm_handle* h, int32_t inst, const double* X);

#define II_LBM_F_RHO 1u     /* rho = sum_i f_i */
#define II_LBM_F_UX 2u      /* u_x = sum_i e_ix f_i */
#define II_LBM_F_UY 4u      /* u_y */
#define II_LBM_F_P 8u       /* p = rho / 3 */
#define II_LBM_F_DISTRIB 16u /* the nine f_i^n planes, population order */
enum { II_LBM_DT_F32 = 0, II_LBM_DT_F64 = 1 };

/* Synchronises, then writes the requested planes of the current state f^n
 * (the distributions after streaming, jumps and boundaries, i.e. what the
 * next collision reads), in bit order RHO, UX, UY, P, DISTRIB, each [ny][nx],
 * as FP32 or FP64, into `out` (device memory when on_device, else host). */
int ii_lbm_fields(ii_lbm_handle* h, int32_t inst, uint32_t what, void* out, int32_t dtype,
                  int32_t on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * host-output form of ii_lbm_fields (on_device = 0) without its per-call
 * staging allocation.  The planes are staged through a static device array
 * of 64 MiB that the library holds on each GPU it runs on until the process
 * ends; the call allocates nothing (no hipMalloc, hipFree or host heap).
 * Same `what`, `dtype` and layout as ii_lbm_fields; `out` is host memory of
 * planes * ny * nx elements.  II_LBM_ECAPACITY when the requested planes
 * exceed 64 MiB (e.g. more than one FP32 plane of a 4096^2 lattice); the
 * state is not touched then.  All calls on one GPU share its array: calls
 * that overlap in time on one GPU (several host threads, or handles on
 * different streams) race and must be serialised by the caller.
 * Synchronises the handle's stream. */
int ii_lbm_fields_noalloc(ii_lbm_handle* h, int32_t inst, uint32_t what, void* out,
                          int32_t dtype);

/* Sets the state of one instance from nine host planes f[9][ny][nx] (FP64,
 * full distributions): the next step collides exactly this field (periodic
 * axes; on non-periodic sides the boundary nodes are re-derived by the
 * extrapolation). */
int ii_lbm_set_distrib(ii_lbm_handle* h, int32_t inst, const double* f);

/* Raw state for checkpoint/restart: the stored lattice in its storage
 * precision plus the markers and the step counter.  A handle restored with
 * ii_lbm_load_state continues bit-identically. */
int ii_lbm_state_size(ii_lbm_handle* h, int32_t inst, size_t* bytes);
int ii_lbm_save_state(ii_lbm_handle* h, int32_t inst, void* host_buf, size_t bytes);
int ii_lbm_load_state(ii_lbm_handle* h, int32_t inst, const void* host_buf, size_t bytes);

/* Synchronises, then copies up to `cap` cut-link records of one instance into
 * a host buffer; *count receives the total number (which may exceed cap).
 * Membranes: the links cut by the polygon through the current markers X^n,
 * which the next step applies; steps do not write them, the first call after
 * a step builds them (one interface pass on the handle's stream).  Rigid
 * bodies: the links of the last step (none before the first step).  Records
 * are in no particular order. */
int ii_lbm_cutlinks(ii_lbm_handle* h, int32_t inst, ii_lbm_link* out, int32_t cap, int32_t* count);

/* Synchronises and fills FP64 diagnostics of one instance (the fields of
 * ii_lbm_diag_t): mass, momentum, area, force, cut-link count and the
 * pressure on either side of the interface.  The sums over the lattice are
 * taken in FP64 per block and added on the host in block order, so repeated
 * calls on one state return identical values. */
int ii_lbm_diag(ii_lbm_handle* h, int32_t inst, ii_lbm_diag_t* out);

/* Kernel timing of the dense collide-and-stream sweep: while enabled, every
 * sweep launch of ii_lbm_step is bracketed by HIP events on the handle's
 * stream; get_timing synchronises and returns the summed milliseconds and
 * the number of timed launches, then clears them. */
int ii_lbm_set_timing(ii_lbm_handle* h, int32_t enable);
int ii_lbm_get_timing(ii_lbm_handle* h, double* sweep_ms, int64_t* launches);

/* Bytes of HBM one sweep of one instance (inst = -1: of all instances) must
 * move: nine loads and nine stores of the stored deviation per node. */
int ii_lbm_sweep_bytes(ii_lbm_handle* h, int32_t inst, double* bytes);

/* Replays the steps as HIP graphs when enable != 0: graphs of S steps
 * (enable = 1: S = 64; an even enable from 2 to 256: S = enable), then of
 * each power of two below S down to 4, each for as many whole runs as the
 * rest of a call holds, then two-step graphs, then a last direct step when
 * the count is odd (20 steps with S = 64: one graph of 16 and one of 4).
 * Fewer graph launches shorten the gaps between steps.  Enabling captures
 * and instantiates every graph (per length and starting lattice buffer) at
 * once, without running them; a later change of schedule, learned
 * correction, tuning or S drops them and the next step rebuilds all, so no
 * replay ever captures.  Timing mode uses direct launches.  Results are
 * identical either way.  EINVAL for an odd enable above 1 or one above 256;
 * ESTATE on a failed handle. */
int ii_lbm_set_graph(ii_lbm_handle* h, int32_t enable);

/* Schedule of a membrane step (rigid bodies always run in order).  The sweep
 * of step n and the marker/tile pass of step n+1 touch disjoint buffers:
 *   SERIAL        all phases in order on the handle's stream;
 *   FULL          interpolation and the next step's interface pass on an
 *                 internal stream, concurrent with the sweep (the default);
 *   INTERP_FIRST  interpolation first, then the interface pass concurrent
 *                 with the sweep.
 * Results are bit-identical in every mode. */
enum { II_LBM_OVERLAP_SERIAL = 0, II_LBM_OVERLAP_FULL = 1, II_LBM_OVERLAP_INTERP_FIRST = 2 };
int ii_lbm_set_overlap(ii_lbm_handle* h, int32_t mode);

/* Handles with several instances advance them all through one launch per
 * phase and step, driven by work tables.  This autotuner picks their schedule
 * on the current state, in two stages:
 *  1. the batched sweep (writing only the buffer the next step overwrites)
 *     for slices of 128, 256 and 512 nodes and two instance orders (as
 *     given, largest first), `trials` launches each;
 *  2. for membranes, whose interface pass runs beside the sweep, the slice
 *     size again (in the order of stage 1) together with the footprint of the
 *     tile pass (ii_lbm_set_tile_blocks: 0, 24, 16, 12, 8, 4, 2 and 1 blocks per CU),
 *     timed on `trials` whole steps per pair.  A step started again from the
 *     same state recomputes the same results, so the state is left as it was.
 * It keeps the fastest order of stage 1 and the fastest pair of stage 2 (the
 * fastest slice of stage 1 without it).  Outputs (may be NULL): the slice
 * size, the order and that schedule's sweep time alone in us
 * (ii_lbm_get_schedule reports the rest).
 * A single-instance handle reports 0 and keeps its row-segment sweep. */
int ii_lbm_autotune(ii_lbm_handle* h, int32_t trials, int32_t* unit, int32_t* order, double* best_us);

/* Footprint of a batched handle's tile pass: about per_cu blocks per compute
 * unit in all (1 ... 64), shared among the instances in proportion to their
 * estimated interface tiles, each block walking several tiles; 0 (the
 * initial setting) gives one block per estimated tile.  A single-instance
 * membrane handle runs per_cu blocks per CU (0: one, the initial setting)
 * when its tile pass runs beside the sweep.  Results do not depend on it.
 * Synchronises a batched handle; EINVAL for per_cu outside 0 ... 64. */
int ii_lbm_set_tile_blocks(ii_lbm_handle* h, int32_t per_cu);

/* The batched schedule in use: sweep slice size, instance order, tile-pass
 * blocks per CU, and the whole-step time in us that the autotuner measured
 * for it (0 before ii_lbm_autotune or without its second stage).  Outputs may
 * be NULL; a single-instance handle reports zeros. */
int ii_lbm_get_schedule(ii_lbm_handle* h, int32_t* unit, int32_t* order, int32_t* tile_per_cu,
                        double* step_us);

/* Failure isolation of the instances of a handle.  Instances share no data,
 * so one that becomes non-finite (EUNSTABLE), leaves the lattice (EGEOMETRY)
 * or overflows a list (ECAPACITY) does not corrupt the others.  Enabled, such
 * an error is kept in that instance's error bits (ii_lbm_instance_errors,
 * ii_lbm_diag) and the handle keeps stepping all instances (the failed ones
 * carry meaningless values); disabled (the default), the first synchronising
 * call reports it and the handle stops (ESTATE afterwards).  Device errors
 * always stop the handle. */
int ii_lbm_set_isolation(ii_lbm_handle* h, int32_t enable);

/* Synchronises and copies the error bits of the first n instances (bit 0
 * capacity, bit 1 record buffer, bit 2 unstable, bit 3 geometry; 0 = healthy). */
int ii_lbm_instance_errors(ii_lbm_handle* h, int32_t* bits, int32_t n);

int ii_lbm_destroy(ii_lbm_handle* h);
const char* ii_lbm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
