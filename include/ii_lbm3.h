/*
 * ii_lbm3.h -- C ABI of the D3Q19 (three-dimensional) form of the immersed
 * interface-lattice Boltzmann method of Qin, Kolahdouz & Griffith
 * (arXiv:2003.12186), whose conclusion calls the extension to three
 * dimensions straightforward, on one MI355X (gfx950).
 *
 * The library advances a periodic box with nineteen velocities, a single- or
 * multiple-relaxation-time collision with the He-Luo equilibrium and the simple
 * force term (Sec. 2.2.1-2.2.2 written for D3Q19), and an optional fixed sphere
 * carrying a uniform normal force F per unit area along its outward normal:
 *   - II_LBM_FORCE_II: the jump [[f_i]] = sigma w_i [[p]] / c_s^2 with [[p]] = F
 *     on every link the sphere's level set |x - c|^2 - R^2 cuts (sigma = +1
 *     from the interior; Sec. 3.1 Eq. (32), Sec. 3.2 Eq. (47)), applied inside
 *     the sweep;
 *   - II_LBM_FORCE_IB: F n spread from markers on the sphere with the product of
 *     Peskin's four-point delta, dA = 4 pi R^2 / N (Sec. 2.2.2, Eq. (17)).
 * Lattice units (dx = dt = 1).
 *
 * Population numbering: 0 rest; 1..6 = +x, -x, +y, -y, +z, -z (w = 1/18);
 * 7..18 = (+x+y), (-x-y), (+x-y), (-x+y), (+x+z), (-x-z), (+x-z), (-x+z),
 * (+y+z), (-y-z), (+y-z), (-y+z) (w = 1/36); w_0 = 1/3.
 * Fields are [c][nz][ny][nx] with x fastest.  Error codes are those of
 * ii_lbm.h; every call returns II_LBM_OK (0) or a negative code.
 */
#ifndef II_LBM3_H
#define II_LBM3_H

#include <stdint.h>

#include "ii_lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * nx, ny, nz   box size, 8 .. 1024 each (periodic on every side).
 * tau          relaxation time (> 0.5).
 * force_mode   II_LBM_FORCE_II or II_LBM_FORCE_IB.
 * body_force   uniform force density.
 * center, radius, f_normal  the sphere (radius 0: none); it must stay at least
 *              3 lattice units from every side of the box.
 * n_markers    IB-LBM only: markers on the sphere, X0 holds 3 n_markers doubles.
 * collision    II_LBM_SRT, or II_LBM_MRT: the orthogonal 19-moment basis of
 *              d'Humieres et al. (2002), the three-dimensional counterpart of
 *              the basis behind the paper's MRT (Sec. 2.2.1), m_eq = M f_eq,
 *              rates 0 for rho and j, 1/tau for the five viscous stresses,
 *              1.19 (e), 1.4 (eps and the two fourth-order stresses), 1.2 (the
 *              heat fluxes), 1.98 (the three third-order moments); the force
 *              term stays in velocity space.
 */
typedef struct ii_lbm3_problem {
    int32_t nx, ny, nz;
    int32_t force_mode;
    double tau;
    double body_force[3];
    double center[3];
    double radius;
    double f_normal;
    int32_t n_markers;
    int32_t collision;
} ii_lbm3_problem;

typedef struct ii_lbm3_handle ii_lbm3_handle;

/* Creates a handle; the library takes its device memory with hipMalloc (two
 * lattices of 19 FP32 deviation planes, three 64-bit fixed-point force planes
 * under IB-LBM or with a membrane, and the buffers of ii_lbm3_set_mesh,
 * ii_lbm3_set_membrane and the rigid surfaces) and frees it in
 * ii_lbm3_destroy.  The fluid starts at rest.  hip_stream: the stream for all
 * work (NULL = default).  Synchronises before returning.  EINVAL for an
 * invalid problem, EDEVICE when allocation fails. */
int ii_lbm3_init(const ii_lbm3_problem* p, const double* X0, void* hip_stream,
                 ii_lbm3_handle** out);

/* Device memory from the caller: a handle created by ii_lbm3_init_with takes
 * every device buffer it ever needs (including the temporaries of
 * ii_lbm3_set_distrib and ii_lbm3_fields) from alloc(bytes, ctx), which must
 * return device memory aligned to 256 bytes or NULL, and hands each back
 * through release(ptr, ctx) once the handle's stream has finished with it
 * (at the latest in ii_lbm3_destroy).  Both are called from the host calls of
 * the handle only, never during ii_lbm3_step.  For callers whose device
 * memory is owned elsewhere, e.g. PyTorch's caching allocator. */
typedef struct ii_lbm3_allocator {
    void* (*alloc)(size_t bytes, void* ctx);
    void (*release)(void* ptr, void* ctx);
    void* ctx;
} ii_lbm3_allocator;

/* ii_lbm3_init with device memory from `alloc` (NULL: hipMalloc, as
 * ii_lbm3_init).  EINVAL also when alloc has a NULL callback. */
int ii_lbm3_init_with(const ii_lbm3_problem* p, const double* X0, void* hip_stream,
                      const ii_lbm3_allocator* alloc, ii_lbm3_handle** out);

/* Enqueues n_steps steps; returns without waiting. */
int ii_lbm3_step(ii_lbm3_handle* h, int64_t n_steps);

/* Sets the state to the host distributions f[19][nz][ny][nx] (FP64). */
int ii_lbm3_set_distrib(ii_lbm3_handle* h, const double* f);

/* Copies rho, u_x, u_y, u_z of the current state (u = sum e_i f_i) into the
 * host array out[4][nz][ny][nx] (FP64).  Synchronises. */
int ii_lbm3_fields(ii_lbm3_handle* h, double* out);

/* HIP-event timing of every sweep launch while enabled; get_timing returns the
 * summed milliseconds and the launch count since enabling.  Synchronises. */
int ii_lbm3_set_timing(ii_lbm3_handle* h, int32_t enable);
int ii_lbm3_get_timing(ii_lbm3_handle* h, double* ms, int64_t* launches);

/* Algorithmic bytes of one sweep launch: 19 loads + 19 stores of 4 bytes per
 * node, plus 24 bytes per node of force field under IB-LBM. */
int ii_lbm3_sweep_bytes(ii_lbm3_handle* h, double* bytes);

/*
 * A fixed closed triangulated surface carrying a pressure jump [[p]] given at
 * its vertices: on every link P -> P + e_i that crosses a triangle, the jump
 * [[f_i]] = sigma w_i [[p]] / c_s^2 of Sec. 3.1 (Eq. (32)) and Sec. 3.2
 * (Eq. (47)), sigma = +1 when P is inside, with [[p]] interpolated
 * barycentrically at the crossing.  The surface is the triangulation the
 * paper's conclusion names for three dimensions; its links are found once
 * here and their jumps applied after every sweep.
 *
 * Vertices X[n_vert][3] (FP64, lattice units) are snapped to multiples of
 * 2^-16 and every side test is an exact integer determinant; ties (a node on
 * a face's plane, a link through an edge or vertex) are broken by translating
 * the lattice by (e, e^2, e^3) with e -> 0+.  Triangles tri[n_tri][3] index
 * the vertices counter-clockwise seen from outside.  A link that runs into the
 * surface through one face and out through another has two records.
 *
 * ii_lbm3_check_mesh validates without touching the GPU; ii_lbm3_set_mesh
 * validates the same way and installs the surface:
 *   EINVAL     force mode not II_LBM_FORCE_II, a NULL array, fewer than 4 or
 *              more than 2^20 vertices or triangles, an index out of range or
 *              repeated in a triangle, a non-finite coordinate or jump value;
 *   EGEOMETRY  a vertex outside [2, n - 3] on some axis, an edge longer than
 *              4 lattice units, a degenerate triangle, a surface that is not
 *              closed and consistently oriented (every directed edge once and
 *              its reverse once), or one whose enclosed volume is not positive;
 *   ECAPACITY  more cut links than 64 n_tri + 4096.
 * The library copies every array.  set_mesh synchronises and replaces any
 * surface installed before; n_vert = n_tri = 0 removes it.  *n_links (may be
 * NULL) receives the number of cut-link records.
 */
int ii_lbm3_check_mesh(const ii_lbm3_problem* p, int32_t n_vert, const double* X, int32_t n_tri,
                       const int32_t* tri);
int ii_lbm3_set_mesh(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri,
                     const int32_t* tri, const double* jump_p, int64_t* n_links);

/* The installed surface's cut links, in no particular order: rec[k] =
 * {x, y, z, dir, sigma, tri} of the sending node, jp[k] = [[p]] at the
 * crossing.  *n_links receives the count; ECAPACITY (nothing copied) when cap
 * is smaller.  Synchronises. */
int ii_lbm3_mesh_links(ii_lbm3_handle* h, int64_t cap, int32_t* rec, double* jp, int64_t* n_links);

/*
 * A deformable closed triangulated membrane under surface tension gamma (>= 0),
 * the three-dimensional counterpart of the flexible interfaces of Sec. 2.1 and
 * Sec. 3.2.  Each step, in the paper's order:
 *   1. U_v = sum_x u^n(x) delta_h(x - X_v) (Peskin's four-point delta in each
 *      axis, Sec. 2.1.2, Eq. (10));
 *   2. the force on the fluid at vertex v, G_v = -gamma dA/dX_v (A the total
 *      area); the vertex area A_v (a third of its triangles'), the
 *      area-weighted outward normal n_v, [[p]]_v = G_v . n_v / A_v and the
 *      tangential part G_v - (G_v . n_v) n_v (Sec. 3.2, Eq. (47)-(49));
 *   3. the tangential parts spread as a force field (Sec. 2.2.2, Eq. (17));
 *   4. the links the surface cuts at X^n carry the jumps (as for the fixed
 *      surface above, found again every step);
 *   5. X^{n+1} = X^n + U^n (Sec. 2.1.2, Eq. (11)).
 * With the problem's force_mode II_LBM_FORCE_IB the membrane runs as IB-LBM
 * instead: the whole G_v is spread and no links carry jumps (Sec. 2.2.2).
 * Validation as ii_lbm3_check_mesh's geometry rules (either force mode), plus
 * EINVAL for a non-finite or negative gamma or a sphere in the problem
 * (radius > 0: the membrane's sweep reads the force field and applies no
 * level-set jumps).  The
 * library copies the arrays; a fixed surface installed before is removed, as
 * a membrane is by a later ii_lbm3_set_mesh; n_vert = n_tri = 0 removes it.
 * Synchronises.
 *
 * On the device, a vertex that leaves [2, n - 3] on some axis, an edge longer
 * than 4 lu or a degenerate triangle stops the membrane (the fluid keeps
 * stepping without it); so do more cut links than 64 n_tri + 4096.
 * ii_lbm3_membrane copies the vertices X[n_vert][3] and the last step's
 * velocities U[n_vert][3] (either may be NULL) and reports such a stop as
 * EGEOMETRY or ECAPACITY; ESTATE without a membrane.  Synchronises.
 */
int ii_lbm3_set_membrane(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri,
                         const int32_t* tri, double gamma);
int ii_lbm3_membrane(ii_lbm3_handle* h, double* X, double* U);

/*
 * A fixed rigid closed triangulated surface held at rest by direct forcing
 * (Sec. 2.1.2, Eq. (9) with eta = 1 and U^D = 0): each step the force on the
 * fluid at vertex v is G_v = (U^D - U_v) A_v, entered as for the membrane
 * above (jump of the normal part on the cut links, spread of the tangential
 * part); the vertices do not move.  Same validation, storage and replacement
 * rules as ii_lbm3_set_membrane; ii_lbm3_membrane reads its vertices and
 * velocities.  The problem's force mode must be II_LBM_FORCE_II (EINVAL
 * otherwise).  Synchronises.
 *
 * ii_lbm3_surface_force writes the force the fluid exerted on the membrane or
 * surface in the last step, F = -sum_v G_v (Sec. 2.1.3), into F[3] (host);
 * ESTATE without a surface, EGEOMETRY / ECAPACITY after a stop (F still
 * written).  Synchronises.
 */
int ii_lbm3_set_rigid_surface(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri,
                              const int32_t* tri);
int ii_lbm3_surface_force(ii_lbm3_handle* h, double* F);

/*
 * A free rigid sphere, triangulated by X / tri about center (host, 3
 * doubles), of radius and density ratio rho_star = rho_s / rho_f, starting
 * with velocity U0 and angular velocity W0 (host, 3 doubles each): the
 * rigid-body dynamics of Sec. 2.3 in three dimensions.  Each step the
 * surface is held at U^D = U + W x (X_v - c) by direct forcing (as the rigid
 * surface above); then
 *   F = -sum G_v + rho_f V_s (U^n - U^{n-1}),
 *   T = -sum (X_v - c) x G_v + (I_s / rho*) (W^n - W^{n-1})
 * (rho_f = 1, V_s = 4 pi R^3 / 3, m = rho* V_s, I_s = 2 m R^2 / 5);
 * a^{n+1} = F / m, U^{n+1} = U^n + a^{n+1}, c^{n+1} = c^n + U^n +
 * (a^n + a^{n+1}) / 2, W^{n+1} = W^n + T / I_s; every vertex moves with c (a
 * rotation leaves a sphere's surface the same set).  The first step takes
 * U^{n-1} = U0 and W^{n-1} = W0.  Same validation and replacement rules as
 * ii_lbm3_set_membrane, plus EINVAL for a non-positive radius or rho_star,
 * non-finite vectors, or the IB-LBM force mode.  The sphere stops like a
 * membrane when it leaves [2, n - 3].  Synchronises.
 *
 * ii_lbm3_body writes out[27] = {c, U, a, W, wdot, U^{n-1}, W^{n-1}, F, T}
 * (3 each; F and T of the last step) to host memory; ESTATE without a free
 * sphere, EGEOMETRY / ECAPACITY after a stop (out still written).
 * Synchronises.
 */
int ii_lbm3_set_free_sphere(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri,
                            const int32_t* tri, const double* center, double radius, double rho_star,
                            const double* U0, const double* W0);
int ii_lbm3_body(ii_lbm3_handle* h, double* out);

int ii_lbm3_destroy(ii_lbm3_handle* h);

#ifdef __cplusplus
}
#endif

#endif
