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

#include "../../include/ii_lbm.h"

namespace iilbm {

// ---------------------------------------------------------------------------
// Geometry of the launch grids.
// ---------------------------------------------------------------------------
constexpr int kSweepBX = 64;     // one wavefront spans 64 consecutive x
constexpr int kSweepBY = 4;      // four rows per 256-thread block
constexpr int kTile = 16;        // interface tiles are 16 x 16 nodes
constexpr int kTileCap = 128;    // chords listed per interface tile
constexpr int kPitchAlign = 64;  // row pitch in elements
constexpr double kSnap = 65536.0;  // marker snap grid 2^-16 lu for exact tests

enum ErrBits : int {
    kErrCapacity = 1,   // a tile had more chords than kTileCap
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
    int n_markers;
    int mk_off;           // offset of this instance in the marker arrays
    int tiles_x, tiles_y;
    int tile_off;         // offset in tile_count (tiles), tile_list (tiles * kTileCap)
    int act_off, act_cap;
    int rec_off, rec_cap;
    int inst;
    long long lat_off;    // element offset of plane 0 in either lattice buffer
    long long plane;      // elements per population plane (pitch * ny)
    float omega;          // 1 / tau
    float s[9];           // MRT rates
    float u_max;
    float u_wall[4];
    float body[2];
    float scale, inv_scale;  // FP16: value = stored * scale
    double kappa, dX, cx, cy, radius;
};

// Device buffers of a handle (all carved from one workspace).
struct DevPtrs {
    void* lat[2];          // lattice ping-pong buffers
    double2* X[2];         // marker position ping-pong
    double2* U;            // interpolated marker velocity of the last step
    double2* G;            // marker force of the last step
    double2* Gt;           // its tangential part
    double* jp;            // [[p]] at the markers
    int* tile_count;       // chords appended per tile (reset by the tile kernel)
    int* tile_list;        // chord ids per tile
    int2* act_list;        // (instance, tile) of the tiles that hold chords
    int* act_count;        // [2 * n_inst], double-buffered by step parity
    ii_lbm_link* rec;      // cut-link records
    int* rec_count;        // [2 * n_inst]
    int* err;              // [n_inst] error bits
    double* diag;          // reduction partials
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

template <>
struct Store<float> {
    static __device__ __forceinline__ float ld(const float* p, float) { return *p; }
    static __device__ __forceinline__ void st(float* p, float v, float) { *p = v; }
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
};

// ---------------------------------------------------------------------------
// Pull gather: the populations that arrive at node (x, y) were stored by the
// previous step at x - e_i (the stored value already carries that step's
// force term and jump).  Periodic wrap; callers only pull across a bounded
// side from a node that extrapolation then overrides.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void pull(const InstDev& I, const T* __restrict__ A, int x, int y,
                                     float d[9])
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
    d[0] = Store<T>::ld(base + 0 * P + r0 + x, sc);
    d[1] = Store<T>::ld(base + 1 * P + r0 + xm, sc);
    d[2] = Store<T>::ld(base + 2 * P + rm + x, sc);
    d[3] = Store<T>::ld(base + 3 * P + r0 + xp, sc);
    d[4] = Store<T>::ld(base + 4 * P + rp + x, sc);
    d[5] = Store<T>::ld(base + 5 * P + rm + xm, sc);
    d[6] = Store<T>::ld(base + 6 * P + rm + xp, sc);
    d[7] = Store<T>::ld(base + 7 * P + rp + xp, sc);
    d[8] = Store<T>::ld(base + 8 * P + rp + xm, sc);
}

__device__ __forceinline__ void moments(const float d[9], float& r, float& ux, float& uy)
{
    r = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    ux = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    uy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
}

// Deviation of the He-Luo incompressible equilibrium (Sec. 2.2.1):
// f_eq_i - w_i rho0 = w_i [ drho + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u ].
__device__ __forceinline__ float deq(int i, float r, float ux, float uy, float uu)
{
    const float eu = (float)EX[i] * ux + (float)EY[i] * uy;
    return WF[i] * (r + 3.f * eu + 4.5f * eu * eu - 1.5f * uu);
}

// Is (x, y) a node that non-equilibrium extrapolation sets?
__device__ __forceinline__ bool is_edge(const InstDev& I, int x, int y)
{
    return (!I.px && (x == 0 || x == I.nx - 1)) || (!I.py && (y == 0 || y == I.ny - 1));
}

// f at a bounded-side node: f_b = f_eq(rho_f, u_b) + (f_f - f_eq(rho_f, u_f)),
// f_f the pulled populations of the inward neighbour (corners: the diagonal
// neighbour, velocity rule of the y side).
template <typename T>
__device__ void nee(const InstDev& I, const T* __restrict__ A, int x, int y, float d[9])
{
    int inx = 0, iny = 0;
    if (!I.px && x == 0) inx = 1;
    if (!I.px && x == I.nx - 1) inx = -1;
    if (!I.py && y == 0) iny = 1;
    if (!I.py && y == I.ny - 1) iny = -1;
    float df[9];
    pull<T>(I, A, x + inx, y + iny, df);
    float r, ux, uy;
    moments(df, r, ux, uy);
    float ubx = 0.f, uby = 0.f;
    int type;
    if (iny != 0) {
        const int s = iny > 0 ? 2 : 3;
        type = I.bc[s];
        if (type == II_LBM_BC_WALL) ubx = I.u_wall[s];
    } else {
        const int s = inx > 0 ? 0 : 1;
        type = I.bc[s];
        if (type == II_LBM_BC_WALL) uby = I.u_wall[s];
    }
    if (type == II_LBM_BC_INLET) {
        const float H = (float)(I.ny - 1);
        ubx = 4.f * I.u_max * (float)y * (H - (float)y) / (H * H);
        uby = 0.f;
    } else if (type == II_LBM_BC_OUTLET) {
        ubx = ux;
        uby = uy;
    }
    const float uub = ubx * ubx + uby * uby, uuf = ux * ux + uy * uy;
#pragma unroll
    for (int i = 0; i < 9; i++) d[i] = deq(i, r, ubx, uby, uub) + (df[i] - deq(i, r, ux, uy, uuf));
}

// f^n at node (x, y): the pulled populations, or the extrapolated ones on a
// bounded side.
template <typename T>
__device__ __forceinline__ void gather(const InstDev& I, const T* __restrict__ A, int x, int y,
                                       float d[9])
{
    if (I.bounded && is_edge(I, x, y))
        nee<T>(I, A, x, y, d);
    else
        pull<T>(I, A, x, y, d);
}

// ---------------------------------------------------------------------------
// Collision with the simple force term (Sec. 2.2.1 Eq. (14)/(15), Sec. 2.2.2
// Eq. (16)); in deviation form the constant w_i rho0 drops out of both.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void collide_srt(float d[9], float omega, float gx, float gy)
{
    float r, ux, uy;
    moments(d, r, ux, uy);
    const float uu = ux * ux + uy * uy;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        const float e = deq(i, r, ux, uy, uu);
        d[i] = d[i] + omega * (e - d[i]) + 3.f * WF[i] * ((float)EX[i] * gx + (float)EY[i] * gy);
    }
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
constexpr float MBN[9] = {1.f / 9.f, 1.f / 36.f, 1.f / 36.f, 1.f / 6.f, 1.f / 12.f,
                          1.f / 6.f, 1.f / 12.f, 1.f / 4.f, 1.f / 4.f};

// MRT: d* = d - M^-1 S M (d - d_eq); only the six non-conserved moments relax.
__device__ __forceinline__ void collide_mrt(float d[9], const float s[9], float gx, float gy)
{
    float r, ux, uy;
    moments(d, r, ux, uy);
    const float uu = ux * ux + uy * uy;
    float ne[9];
#pragma unroll
    for (int i = 0; i < 9; i++) ne[i] = d[i] - deq(i, r, ux, uy, uu);
    float m[9];
#pragma unroll
    for (int a = 0; a < 9; a++) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < 9; i++)
            if (MB[a][i] != 0) acc += (float)MB[a][i] * ne[i];
        m[a] = (a == 0 || a == 3 || a == 5) ? 0.f : s[a] * MBN[a] * acc;
    }
#pragma unroll
    for (int i = 0; i < 9; i++) {
        float acc = 0.f;
#pragma unroll
        for (int a = 0; a < 9; a++)
            if (MB[a][i] != 0 && a != 0 && a != 3 && a != 5) acc += (float)MB[a][i] * m[a];
        d[i] = d[i] - acc + 3.f * WF[i] * ((float)EX[i] * gx + (float)EY[i] * gy);
    }
}

// ---------------------------------------------------------------------------
// Launch helpers implemented in the .hip files (host side).
// ---------------------------------------------------------------------------
hipError_t launch_sweep(const InstDev& I, const void* A, void* B, hipStream_t s);
hipError_t launch_fill_zero(const InstDev& I, void* A, hipStream_t s);
hipError_t launch_fields(const InstDev& I, const void* A, uint32_t what, void* out, int dtype,
                         hipStream_t s);
hipError_t launch_set_distrib(const InstDev& I, const double* f, void* A, hipStream_t s);
hipError_t launch_diag(const InstDev& I, const void* A, double* partials, int nblocks,
                       hipStream_t s);
hipError_t launch_markers(const InstDev& I, const DevPtrs& P, const void* A, int parity,
                          hipStream_t s);
hipError_t launch_tiles(const InstDev& I, const DevPtrs& P, void* B, int parity, int records,
                        hipStream_t s);
hipError_t launch_zero_ints(int* p, long long n, hipStream_t s);

}  // namespace iilbm
