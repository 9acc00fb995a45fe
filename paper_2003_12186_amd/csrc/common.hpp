// Internal definitions shared by the HIP translation units of the II-LBM
// library: the per-instance descriptor, the device pointer table, the D2Q9
// lattice, storage conversion, the pull gather (with non-equilibrium
// extrapolation on bounded sides) and the collision operators.
//
// Method: Qin, Kolahdouz & Griffith, arXiv:2003.12186.  Lattice units
// (dx = dt = 1, Sec. 2.2).  Distributions are stored as deviations
// d_i = f_i - w_i rho0 with rho0 = 1, so that FP32 (and scaled FP16) keep the
// small physical signal instead of the constant rest populations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ii_learned.h"

namespace iilbm {

// ---------------------------------------------------------------------------
// Geometry of the launch grids.
// ---------------------------------------------------------------------------
// The sweep runs one block per row segment of 512, 256 or 64 nodes (the
// widest that divides the row): whole rows of distributions stream through
// each block and the y +- 1 rows its neighbours need are read by blocks
// dispatched close in time on the same XCD.
constexpr int kTile = 16;        // interface tiles are 16 x 16 nodes
constexpr int kTileCap = 128;    // chords listed per interface tile (II-LBM)
constexpr int kTileCapIB = 512;  // markers listed per tile under IB-LBM (dense markers, no jumps)
constexpr int kTileNodes = kTile * kTile;
// Planes of a tile's correction slot: the additions to the eight moving
// populations, then (under Guo's force term) the spread force g_x, g_y.
constexpr int kCorrPlanes = 10;
constexpr int kPitchAlign = 64;  // row pitch in elements
constexpr double kSnap = 65536.0;  // marker snap grid 2^-16 lu for exact tests

enum ErrBits : int {
    kErrCapacity = 1,   // a tile had more chords than its list holds
    kErrRecords = 2,    // cut-link record buffer full (records only)
    kErrUnstable = 4,   // non-finite marker velocity
    kErrGeometry = 8,   // a marker left the supported region
};

// Per-instance descriptor, passed by value to the kernels.
struct InstDev {
    int nx, ny, pitch;
    int px, py;           // axis periodic?
    int bounded;          // any non-periodic side
    int bc[4];
    int collision, storage, iface;
    int jumps;            // force mode with jumps on cut links (II-LBM)
    int guo;              // force mode with Guo's force term
    int math;             // II_LBM_MATH_FP32 or II_LBM_MATH_FP64 collision arithmetic
    int n_markers;
    int mk_off;           // offset of this instance in the marker arrays
    int tiles_x, tiles_y;
    int tile_off;         // offset in tile_count and tile_slot (tiles)
    int tile_cap;         // chord list capacity of a tile (kTileCap or kTileCapIB)
    long long list_off;   // offset in tile_list (ints)
    int act_off, act_cap;
    int rec_off, rec_cap;
    int mk_blocks;        // 256-thread blocks of the marker kernel (16 markers each)
    int tile_blocks;      // blocks of the tile kernel (they stride over the active tiles)
    int inst;
    long long lat_off;    // element offset of plane 0 in either lattice buffer
    long long plane;      // elements per population plane (pitch * ny)
    float omega;          // 1 / tau
    double omega_d;
    float s[9];           // MRT rates
    float u_max;
    float u_wall[4];
    float body[2];
    float scale, inv_scale;  // FP16: value = stored * scale
    double kappa, dX, cx, cy, radius;
    double f_normal;      // prescribed normal force per unit length (NORMAL circle)
    int geometry;         // membrane: 0 polygon through the markers, 1 cubic spline
    int spl_periodic;     // spline taps: 1 = periodic sum over all N, 0 = |j| <= 32
    int tap_off;          // offset of this instance's taps
    int moving;           // a moving rigid circle (body state on the device)
    int body_free;        // bit 0 x, bit 1 y, bit 2 rotation
    double rho_star, spring[2], damping[2], presc_amp[2], presc_umax[2];
};

// State of a moving rigid circle (Sec. 2.3) for the step about to run.
struct BodyDev {
    double c[2], U[2], a[2];   // centre, velocity, acceleration
    double theta, W, wdot;     // angle, angular velocity and acceleration
    double Uprev[2], Wprev;    // the previous step's velocities
    double F[2], T;            // F^ext, T^ext of the last step
    double c0[2];              // initial centre (the springs' rest point)
    double theta_mod;          // theta reduced to [0, 2 pi)
    long long n;               // steps taken
};

// Device buffers of a handle (all carved from one workspace).
struct DevPtrs {
    void* lat[2];          // lattice ping-pong buffers
    double2* X[2];         // marker position ping-pong
    double2* U;            // interpolated marker velocity of the last step
    double2* G;            // marker force of the last step
    double2* Gt;           // its tangential part
    double* jp;            // [[p]] at the markers
    double* wx;            // [4 N] delta weights of the 4 stencil columns of each marker
    double* wy;            // [4 N] ... and of its 4 stencil rows
    int2* f0;              // first stencil column and row of each marker
    int* tile_count;       // chords appended per tile (reset by the tile kernel)
    int* tile_list;        // chord ids per tile
    int* tile_slot[2];     // correction slot of a tile at step m (plane m & 1), -1 when none
    float* corr[2];        // per slot: kCorrPlanes x 256 (population additions, then g)
    unsigned long long* cmask[2];   // per slot: 4 words, bit n set when node n has corrections
    int2* act_list[2];     // (instance, tile) of the tiles that hold chords, by parity
    int* act_count;        // [2 * n_inst], double-buffered by step parity
    ii_lbm_link* rec;      // cut-link records
    int* rec_count;        // [2 * n_inst]
    int* err;              // [n_inst] error bits
    double* diag;          // reduction partials
    BodyDev* body;         // [n_inst] moving-body states
    double2* M;            // spline second derivatives per marker
    const double* spline_taps;
};

// ---------------------------------------------------------------------------
// D2Q9 (Sec. 2.1.1 velocities, Sec. 2.2.1 weights).
// ---------------------------------------------------------------------------
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr float WF[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                         1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
constexpr double WD[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// ---------------------------------------------------------------------------
// Storage precision.
// ---------------------------------------------------------------------------
template <typename T>
struct Store;

// st_stream: the sweep's stores, which the next step reads back only after the
// whole lattice has streamed through (non-temporal hint).
template <>
struct Store<float> {
    static __device__ __forceinline__ float ld(const float* p, float) { return *p; }
    static __device__ __forceinline__ void st(float* p, float v, float) { *p = v; }
    static __device__ __forceinline__ void st_stream(float* p, float v, float)
    {
        __builtin_nontemporal_store(v, p);
    }
};

template <>
struct Store<_Float16> {
    static __device__ __forceinline__ float ld(const _Float16* p, float scale)
    {
        return (float)(*p) * scale;
    }
    static __device__ __forceinline__ void st(_Float16* p, float v, float inv_scale)
    {
        *p = (_Float16)(v * inv_scale);
    }
    static __device__ __forceinline__ void st_stream(_Float16* p, float v, float inv_scale)
    {
        __builtin_nontemporal_store((_Float16)(v * inv_scale), p);
    }
};

// ---------------------------------------------------------------------------
// Pull gather: the populations that arrive at node (x, y) were stored by the
// previous step at x - e_i (the stored value already carries that step's
// force term and jump).  Periodic wrap; callers only pull across a bounded
// side from a node that extrapolation then overrides.  M is the arithmetic
// type of the collision (float, or double for FP64 collision arithmetic).
// ---------------------------------------------------------------------------
template <typename T, typename M>
__device__ __forceinline__ void pull(const InstDev& I, const T* __restrict__ A, int x, int y,
                                     M d[9])
{
    const int xm = (x == 0) ? I.nx - 1 : x - 1;
    const int xp = (x == I.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? I.ny - 1 : y - 1;
    const int yp = (y == I.ny - 1) ? 0 : y + 1;
    const T* base = A + I.lat_off;
    const long long r0 = (long long)y * I.pitch, rm = (long long)ym * I.pitch,
                    rp = (long long)yp * I.pitch;
    const long long P = I.plane;
    const float sc = I.scale;
    d[0] = (M)Store<T>::ld(base + 0 * P + r0 + x, sc);
    d[1] = (M)Store<T>::ld(base + 1 * P + r0 + xm, sc);
    d[2] = (M)Store<T>::ld(base + 2 * P + rm + x, sc);
    d[3] = (M)Store<T>::ld(base + 3 * P + r0 + xp, sc);
    d[4] = (M)Store<T>::ld(base + 4 * P + rp + x, sc);
    d[5] = (M)Store<T>::ld(base + 5 * P + rm + xm, sc);
    d[6] = (M)Store<T>::ld(base + 6 * P + rm + xp, sc);
    d[7] = (M)Store<T>::ld(base + 7 * P + rp + xp, sc);
    d[8] = (M)Store<T>::ld(base + 8 * P + rp + xm, sc);
}

template <typename M>
__device__ __forceinline__ void moments(const M d[9], M& r, M& ux, M& uy)
{
    r = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    ux = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    uy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
}

template <typename M>
struct Lat;
template <>
struct Lat<float> {
    static __device__ __forceinline__ float w(int i) { return WF[i]; }
};
template <>
struct Lat<double> {
    static __device__ __forceinline__ double w(int i) { return WD[i]; }
};

// Odd part of the D2Q9 equilibrium, w_i 3 e_i.u: u/3 on the axes and
// (+-ux +- uy)/12 on the diagonals.  The axis parts are rounded first; the
// remainders u - 2 a are then exact (their operands are within a factor of
// two of each other), and the diagonal parts close the momentum, which is u
// up to the rounding of the two sums alone.  Nothing here adds a constant
// to values on a common rounding grid, so the rounding has no bias: with the
// axis parts closing the momentum instead (u/2 minus the rounded diagonal
// parts), FP32 collisions lose momentum at a fixed relative rate of ~5e-9
// per step, ~1e-5 of the velocity after 1000 steps.
template <typename M>
__device__ __forceinline__ void odd_part(M ux, M uy, M& a1, M& a2, M& a5, M& a6)
{
    const M c3 = (M)(1.0 / 3.0);
    a1 = c3 * ux;
    a2 = c3 * uy;
    const M rx = ux - (M)2 * a1, ry = uy - (M)2 * a2;
    a5 = (M)0.25 * (rx + ry);
    a6 = (M)0.25 * (ry - rx);
}

// Deviation of the He-Luo incompressible equilibrium (Sec. 2.2.1),
// f_eq_i - w_i rho0 = w_i [ drho + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u ], written so
// that its zeroth and first moments are drho and u up to unbiased rounding:
// the rest population takes drho minus the others, and the odd part closes
// the momentum (odd_part).  (With rounded weights the plain form changes the
// momentum by a fixed relative 1e-8 every step.)
template <typename M>
__device__ __forceinline__ void equilibrium(M r, M ux, M uy, M e[9])
{
    const M uu = ux * ux + uy * uy;
    M s[9];
#pragma unroll
    for (int i = 1; i < 9; i++) {
        const M eu = (M)EX[i] * ux + (M)EY[i] * uy;
        s[i] = Lat<M>::w(i) * (r + (M)4.5 * eu * eu - (M)1.5 * uu);
    }
    s[0] = r - (((s[1] + s[2]) + (s[3] + s[4])) + ((s[5] + s[6]) + (s[7] + s[8])));
    M a1, a2, a5, a6;
    odd_part<M>(ux, uy, a1, a2, a5, a6);
    e[0] = s[0];
    e[1] = s[1] + a1;
    e[2] = s[2] + a2;
    e[3] = s[3] - a1;
    e[4] = s[4] - a2;
    e[5] = s[5] + a5;
    e[6] = s[6] + a6;
    e[7] = s[7] - a5;
    e[8] = s[8] - a6;
}

// Deviation of the compressible equilibrium of Guo's force term (Sec. 2.2.2),
// f_eq_i - w_i = w_i [ drho + 3 e.J + (4.5 (e.J)^2 - 1.5 J.J) / rho ] with
// J = rho u, in the same moment-preserving arrangement as above (zeroth and
// first moments drho and J).
template <typename M>
__device__ __forceinline__ void equilibrium_guo(M r, M jx, M jy, M inv_rho, M e[9])
{
    const M jj = jx * jx + jy * jy;
    M s[9];
#pragma unroll
    for (int i = 1; i < 9; i++) {
        const M ej = (M)EX[i] * jx + (M)EY[i] * jy;
        s[i] = Lat<M>::w(i) * (r + ((M)4.5 * ej * ej - (M)1.5 * jj) * inv_rho);
    }
    s[0] = r - (((s[1] + s[2]) + (s[3] + s[4])) + ((s[5] + s[6]) + (s[7] + s[8])));
    M a1, a2, a5, a6;
    odd_part<M>(jx, jy, a1, a2, a5, a6);
    e[0] = s[0];
    e[1] = s[1] + a1;
    e[2] = s[2] + a2;
    e[3] = s[3] - a1;
    e[4] = s[4] - a2;
    e[5] = s[5] + a5;
    e[6] = s[6] + a6;
    e[7] = s[7] - a5;
    e[8] = s[8] - a6;
}

// Guo's force distribution G~_i = w_i [ 3 (e_i - u).g + 9 (e_i.u)(e_i.g) ]
// (Sec. 2.2.2) with u = J / rho; its rest entry closes the zero sum.
template <typename M>
__device__ __forceinline__ void guo_force(M ux, M uy, M gx, M gy, M G[9])
{
    const M ug = ux * gx + uy * gy;
    M t = 0;
#pragma unroll
    for (int i = 1; i < 9; i++) {
        const M eu = (M)EX[i] * ux + (M)EY[i] * uy, eg = (M)EX[i] * gx + (M)EY[i] * gy;
        G[i] = Lat<M>::w(i) * ((M)3 * (eg - ug) + (M)9 * eu * eg);
        t += G[i];
    }
    G[0] = -t;
}

// Is (x, y) a node that non-equilibrium extrapolation sets?
__device__ __forceinline__ bool is_edge(const InstDev& I, int x, int y)
{
    return (!I.px && (x == 0 || x == I.nx - 1)) || (!I.py && (y == 0 || y == I.ny - 1));
}

// f at a bounded-side node: f_b = f_eq(rho_f, u_b) + (f_f - f_eq(rho_f, u_f)),
// f_f the pulled populations of the inward neighbour (corners: the diagonal
// neighbour, velocity rule of the y side).
template <typename T, typename M>
__device__ void nee(const InstDev& I, const T* __restrict__ A, int x, int y, M d[9])
{
    int inx = 0, iny = 0;
    if (!I.px && x == 0) inx = 1;
    if (!I.px && x == I.nx - 1) inx = -1;
    if (!I.py && y == 0) iny = 1;
    if (!I.py && y == I.ny - 1) iny = -1;
    M df[9];
    pull<T, M>(I, A, x + inx, y + iny, df);
    M r, ux, uy;
    moments<M>(df, r, ux, uy);
    M ubx = 0, uby = 0;
    int type;
    if (iny != 0) {
        const int s = iny > 0 ? 2 : 3;
        type = I.bc[s];
        if (type == II_LBM_BC_WALL) ubx = (M)I.u_wall[s];
    } else {
        const int s = inx > 0 ? 0 : 1;
        type = I.bc[s];
        if (type == II_LBM_BC_WALL) uby = (M)I.u_wall[s];
    }
    if (type == II_LBM_BC_INLET) {
        const M H = (M)(I.ny - 1);
        ubx = (M)4 * (M)I.u_max * (M)y * (H - (M)y) / (H * H);
        uby = 0;
    } else if (type == II_LBM_BC_INLET_UNIFORM) {
        ubx = (M)I.u_max;
        uby = 0;
    } else if (type == II_LBM_BC_OUTLET) {
        ubx = ux;
        uby = uy;
    }
    M eb[9], ef[9];
    equilibrium<M>(r, ubx, uby, eb);
    equilibrium<M>(r, ux, uy, ef);
#pragma unroll
    for (int i = 0; i < 9; i++) d[i] = eb[i] + (df[i] - ef[i]);
}

// f^n at node (x, y): the pulled populations, or the extrapolated ones on a
// bounded side.
template <typename T, typename M>
__device__ __forceinline__ void gather(const InstDev& I, const T* __restrict__ A, int x, int y,
                                       M d[9])
{
    if (I.bounded && is_edge(I, x, y))
        nee<T, M>(I, A, x, y, d);
    else
        pull<T, M>(I, A, x, y, d);
}

// ---------------------------------------------------------------------------
// Collision with the simple force term (Sec. 2.2.1 Eq. (14)/(15), Sec. 2.2.2
// Eq. (16)); in deviation form the constant w_i rho0 drops out of both.
// The force term and the interface correction x (x[0] = 0; zero away from
// the interface) join the relaxation increment before the increment is added
// to d, so that d takes one rounding.  Added on its own, a uniform force
// would moreover be rounded the same way at every node (d and d_eq share a
// grid, and omega (d_eq - d) is then a multiple of a fixed fraction of it), a
// bias that builds up step by step.
// ---------------------------------------------------------------------------
template <typename M>
__device__ __forceinline__ M force_term(int i, M gx, M gy)
{
    return i == 0 ? (M)0 : (M)3 * Lat<M>::w(i) * ((M)EX[i] * gx + (M)EY[i] * gy);
}


// D2Q9 moment basis of Lallemand & Luo in the order (rho, e, eps, jx, qx, jy,
// qy, pxx, pxy), and the inverse row norms.
constexpr int MB[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};
constexpr double MBN[9] = {1.0 / 9.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 6.0, 1.0 / 12.0,
                           1.0 / 6.0, 1.0 / 12.0, 1.0 / 4.0, 1.0 / 4.0};

// MRT: d* = d - M^-1 S M (d - d_eq); only the six non-conserved moments
// relax, and the integer basis keeps the correction free of any density or
// momentum.
template <typename M>
__device__ __forceinline__ void collide_mrt(M d[9], const float s[9], M gx, M gy, const M x[9])
{
    M r, ux, uy, e[9];
    moments<M>(d, r, ux, uy);
    equilibrium<M>(r, ux, uy, e);
    M ne[9];
#pragma unroll
    for (int i = 0; i < 9; i++) ne[i] = d[i] - e[i];
    M m[9];
#pragma unroll
    for (int a = 0; a < 9; a++) {
        M acc = 0;
#pragma unroll
        for (int i = 0; i < 9; i++)
            if (MB[a][i] != 0) acc += (M)MB[a][i] * ne[i];
        m[a] = (a == 0 || a == 3 || a == 5) ? (M)0 : (M)s[a] * (M)MBN[a] * acc;
    }
#pragma unroll
    for (int i = 0; i < 9; i++) {
        M acc = 0;
#pragma unroll
        for (int a = 0; a < 9; a++)
            if (MB[a][i] != 0 && a != 0 && a != 3 && a != 5) acc += (M)MB[a][i] * m[a];
        d[i] = d[i] + ((force_term<M>(i, gx, gy) - acc) + x[i]);
    }
}

// SRT, d* = d + omega (d_eq - d).  With FP64 arithmetic it is evaluated
// directly.  With FP32 arithmetic the computed density and velocity, and so
// d_eq, carry roundings of the size of d's own, and the direct form would
// change the momentum by omega times that rounding at every node and step:
// after 1000 steps a velocity error several times that of the storage
// rounding alone.  The FP32 form therefore takes the density and momentum
// that d - d_eq still holds (the rounding residue, exactly zero in exact
// arithmetic) and removes them as the equilibrium-shaped w_i (r + 3 e_i.j):
// the increment then changes density and momentum only by roundings at the
// increment's own, much finer, scale.  RESIDUE = false skips that step where
// FP16 storage rounds every value far more coarsely anyway.
template <typename M, bool RESIDUE = true>
__device__ __forceinline__ void collide_srt(M d[9], M omega, M gx, M gy, const M x[9])
{
    if constexpr (sizeof(M) == 4 && RESIDUE) {
        M r, ux, uy, e[9], ne[9];
        moments<M>(d, r, ux, uy);
        equilibrium<M>(r, ux, uy, e);
#pragma unroll
        for (int i = 0; i < 9; i++) ne[i] = d[i] - e[i];
        M nr, nx, ny;
        moments<M>(ne, nr, nx, ny);
#pragma unroll
        for (int i = 0; i < 9; i++) {
            const M p = ne[i] - Lat<M>::w(i) * (nr + (M)3 * ((M)EX[i] * nx + (M)EY[i] * ny));
            d[i] = d[i] + ((force_term<M>(i, gx, gy) - omega * p) + x[i]);
        }
    } else {
        M r, ux, uy, e[9];
        moments<M>(d, r, ux, uy);
        equilibrium<M>(r, ux, uy, e);
#pragma unroll
        for (int i = 0; i < 9; i++)
            d[i] = d[i] + ((omega * (e[i] - d[i]) + force_term<M>(i, gx, gy)) + x[i]);
    }
}

// Collisions with Guo's force term (Sec. 2.2.2): rho u = J = j + g/2, the
// compressible equilibrium of J and
//   SRT: d* = d + omega (d_eq - d) + (1 - omega/2) G~,
//   MRT: d* = d - M^-1 [ S M (d - d_eq) - (I - S/2) M G~ ].
// The momentum moments gain exactly g whatever their rate (the relaxation of
// j - J = -g/2 and (1 - s/2) g add up to g), so they take g directly.
template <typename M>
__device__ __forceinline__ void guo_prepare(const M d[9], M gx, M gy, M e[9], M G[9])
{
    M r, jx, jy;
    moments<M>(d, r, jx, jy);
    const M inv_rho = (M)1 / ((M)1 + r);
    const M Jx = jx + (M)0.5 * gx, Jy = jy + (M)0.5 * gy;
    equilibrium_guo<M>(r, Jx, Jy, inv_rho, e);
    guo_force<M>(Jx * inv_rho, Jy * inv_rho, gx, gy, G);
}

template <typename M>
__device__ __forceinline__ void collide_guo_mrt(M d[9], const float s[9], M gx, M gy, const M x[9])
{
    M e[9], G[9];
    guo_prepare<M>(d, gx, gy, e, G);
    M m[9];
#pragma unroll
    for (int a = 0; a < 9; a++) {
        M ne = 0, mg = 0;
#pragma unroll
        for (int i = 0; i < 9; i++)
            if (MB[a][i] != 0) {
                ne += (M)MB[a][i] * (d[i] - e[i]);
                mg += (M)MB[a][i] * G[i];
            }
        const M sa = (M)s[a];
        m[a] = (M)MBN[a] * (sa * ne - ((M)1 - (M)0.5 * sa) * mg);
    }
    m[0] = 0;
    m[3] = -(M)MBN[3] * gx;
    m[5] = -(M)MBN[5] * gy;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        M acc = 0;
#pragma unroll
        for (int a = 0; a < 9; a++)
            if (MB[a][i] != 0) acc += (M)MB[a][i] * m[a];
        d[i] = d[i] + (x[i] - acc);
    }
}

// Guo's SRT is Guo's MRT with every rate omega.  With FP32 arithmetic it is
// evaluated in that moment form, where the density and momentum moments of
// the increment are set exactly (for the reason given at collide_srt).
template <typename M>
__device__ __forceinline__ void collide_guo_srt(M d[9], M omega, M gx, M gy, const M x[9])
{
    if constexpr (sizeof(M) == 4) {
        float rates[9];
#pragma unroll
        for (int a = 0; a < 9; a++) rates[a] = omega;
        collide_guo_mrt<M>(d, rates, gx, gy, x);
    } else {
        M e[9], G[9];
        guo_prepare<M>(d, gx, gy, e, G);
        const M h = (M)1 - (M)0.5 * omega;
#pragma unroll
        for (int i = 0; i < 9; i++) d[i] = d[i] + ((omega * (e[i] - d[i]) + h * G[i]) + x[i]);
    }
}

// Whether node `node` (0 ... 255, row-major in its tile) of correction slot
// `slot` holds corrections: only those nodes' planes are written by the tile
// pass (most nodes of an interface tile have none).
__device__ __forceinline__ bool corr_present(const unsigned long long* __restrict__ cmask, int slot,
                                             int node)
{
    return (cmask[(long long)slot * 4 + (node >> 6)] >> (node & 63)) & 1ull;
}

// Work tables of the batched launches: one entry (instance, unit) per block.
struct Batch {
    const InstDev* insts;  // device copy of the descriptors
    const int2* mk_table;  // (instance, block within the instance)
    const int2* tile_table;
    const int2* sweep_table;  // (instance, first node of a slice of `sweep_unit` nodes)
    int mk_units, tile_units, sweep_units;
    int sweep_unit;        // 128, 256 or 512 nodes per sweep block
    int storage, math, iface;
    int guo;               // Guo's force term (uniform over the batch)
    int jumps;             // II-LBM force mode (uniform over the batch)
    const int2* geo_table; // (instance, block of 256 markers): membrane geometry
    int geo_units;
};

// What other translation units may see of a handle: descriptors (host and
// device copies), the device buffers, the current parity and the stream.
struct HandleView {
    int n_inst;
    const InstDev* inst;     // host copies
    const InstDev* d_inst;   // device copies
    DevPtrs P;
    int parity;              // lattice and marker buffers of the current state
    hipStream_t stream;
    int failed;
    int n_cu;                // compute units of the handle's device
};
int handle_view(ii_lbm_handle* h, HandleView* v);

// The learned coarse correction: network, scales and the caller's scratch
// (tiles, counts, patches, flags, amplitudes of n_inst * cap slots).
struct LearnedCfg {
    bool on = false;
    const float* params = nullptr;
    const void* packed = nullptr;
    ii_cnn_scales sc{};
    int cap = 0;
    int* tiles = nullptr;
    int* count = nullptr;
    uint16_t* in = nullptr;
    uint8_t* flags = nullptr;
    float* pscale = nullptr;
};
// Its phases (learned.hip), enqueued on v.stream for the state of plane
// v.parity: band tiles and patch geometry need only the markers, patch flow
// only the lattice, and the network + masked add both of those.
int learned_validate(const HandleView& v, int cap);
hipError_t learned_band(const HandleView& v, const LearnedCfg& c);
hipError_t learned_geom(const HandleView& v, const LearnedCfg& c);
hipError_t learned_flow(const HandleView& v, const LearnedCfg& c);
hipError_t learned_infer(const HandleView& v, const LearnedCfg& c);

// ---------------------------------------------------------------------------
// Launch helpers implemented in the .hip files (host side).
// ---------------------------------------------------------------------------
// par: parity of the step whose correction planes the sweep adds.
hipError_t launch_sweep(const InstDev& I, const DevPtrs& P, const void* A, void* B, int par,
                        hipStream_t s);
hipError_t launch_fill_zero(const InstDev& I, void* A, hipStream_t s);
hipError_t launch_fields(const InstDev& I, const void* A, uint32_t what, void* out, int dtype,
                         hipStream_t s);
hipError_t launch_set_distrib(const InstDev& I, const double* f, void* A, hipStream_t s);
hipError_t launch_diag(const InstDev& I, const void* A, double* partials, int nblocks,
                       hipStream_t s);
// Per-block (sum p, count) inside and outside the marker polygon over the
// nodes farther than `margin` lu from it (X: the instance's markers).
hipError_t launch_pjump(const InstDev& I, const void* A, const double2* X, double margin,
                        double* part, int nblocks, hipStream_t s);
// Marker pass modes (bit 1: interpolation and marker update, bit 2: force,
// geometry, delta weights and tile binning).
enum MarkerMode { kModeInterp = 1, kModeGeom = 2, kModeFull = 3 };
hipError_t launch_markers(const InstDev& I, const DevPtrs& P, const void* A, int par, int mode,
                          hipStream_t s);
hipError_t launch_slot_reset(const InstDev& I, const DevPtrs& P, int par, hipStream_t s);
hipError_t launch_slot_reset_batch(const Batch& b, int n_inst, const DevPtrs& P, int par,
                                   hipStream_t s);
hipError_t launch_tiles(const InstDev& I, const DevPtrs& P, int parity, bool records, hipStream_t s);
hipError_t launch_fill_ints(int* p, long long n, int value, hipStream_t s);
hipError_t launch_body(const InstDev& I, const DevPtrs& P, int par, hipStream_t s);
hipError_t launch_spline(const InstDev& I, const DevPtrs& P, int par, hipStream_t s);
hipError_t launch_markers_batch(const Batch& b, const DevPtrs& P, const void* A, int par, int mode,
                                hipStream_t s);
hipError_t launch_tiles_batch(const Batch& b, const DevPtrs& P, int parity, bool records,
                              hipStream_t s);
hipError_t launch_sweep_batch(const Batch& b, const DevPtrs& P, const void* A, void* B, int par,
                              hipStream_t s);

}  // namespace iilbm
