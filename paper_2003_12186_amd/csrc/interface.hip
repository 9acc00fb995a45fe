// Interface kernels of one II-LBM step (compiled without FP contraction so
// that the FP64 geometry is evaluated exactly as written):
//   k_markers  16 lanes per marker (one per stencil node): interpolated
//              velocity U^n, force G^n, outward normal, |dX/ds|, [[p]] and the
//              tangential part; the new position X^{n+1}; binning of chord
//              (k, k+1) into 16x16 tiles.
//   k_geom_batch  the geometry and binning of batched membranes, one thread
//              per marker, tile counts gathered per block in LDS.
//   k_tiles    one block per tile that holds chords: spreads the tangential
//              force (the whole force under IB-LBM) onto its nodes, finds
//              (under II-LBM) every cut link leaving its nodes
//              with exact integer predicates, writes the force term plus the
//              jumps of every outgoing population into the tile's correction
//              slot (added by the sweep before its store), and compacts the
//              cut-link records.
#include "common.hpp"

namespace iilbm {

constexpr double kCs2 = 1.0 / 3.0;

// Peskin's four-point regularized delta (cited in Sec. 2.1.2), one axis.
__device__ __forceinline__ double peskin(double r)
{
    const double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) * 0.125;
    return 0.0;
}

__device__ __forceinline__ int wrap_or_clamp(int v, int n, int periodic)
{
    if (periodic) return ((v % n) + n) % n;
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// Spring force kappa (X_{k+1} - 2 X_k + X_{k-1}) / dX^2 (Sec. 2.2.2,
// Eq. (19)) of membrane marker k, its outward normal and |dX/ds|: from the
// spline tangent at the knot (geometry 1), else from the central chord with
// the mean length of the two chords at the marker.
__device__ __forceinline__ void membrane_geometry(const InstDev& I, const DevPtrs& P, int m, int kp,
                                                  double2 Xm, double2 Xk, double2 Xp, double& gx,
                                                  double& gy, double& nx_, double& ny_, double& jac)
{
    const double d2 = I.dX * I.dX;
    gx = I.kappa * (Xp.x - 2.0 * Xk.x + Xm.x) / d2;
    gy = I.kappa * (Xp.y - 2.0 * Xk.y + Xm.y) / d2;
    if (I.geometry == 1) {
        // spline tangent at the knot, T = S_k'(0), its normal and |T| / dX
        const double2 Mk = P.M[m], Mp = P.M[I.mk_off + kp];
        const double tx = Xp.x - Xk.x - (2.0 * Mk.x + Mp.x) / 6.0;
        const double ty = Xp.y - Xk.y - (2.0 * Mk.y + Mp.y) / 6.0;
        const double tl = sqrt(tx * tx + ty * ty);
        nx_ = ty / tl;
        ny_ = -tx / tl;
        jac = tl / I.dX;
    } else {
        // outward normal of the counter-clockwise curve, from the central chord
        const double tx = Xp.x - Xm.x, ty = Xp.y - Xm.y;
        const double tl = sqrt(tx * tx + ty * ty);
        nx_ = ty / tl;
        ny_ = -tx / tl;
        // |dX/ds|: mean length of the two chords at the marker over Delta X
        const double lp = hypot(Xp.x - Xk.x, Xp.y - Xk.y);
        const double lm = hypot(Xk.x - Xm.x, Xk.y - Xm.y);
        jac = (lp + lm) / (2.0 * I.dX);
    }
}

// [[p]] = G.n / |dX/ds| (Sec. 3.1, Eq. (40)) and G_par = G - (G.n) n (Eq. (46))
// of marker m.
__device__ __forceinline__ void store_marker_force(const DevPtrs& P, int m, double gx, double gy,
                                                   double nx_, double ny_, double jac)
{
    const double gn = gx * nx_ + gy * ny_;
    P.G[m] = make_double2(gx, gy);
    P.jp[m] = gn / jac;
    P.Gt[m] = make_double2(gx - gn * nx_, gy - gn * ny_);
}

// The tiles within 2.5 lu of chord (k, k+1), [tx0, tx1] x [ty0, ty1]: those
// tiles hold the nodes whose links it can cut and the support of marker k's
// delta.  False when the chord is not finite.
__device__ __forceinline__ bool chord_tiles(const InstDev& I, const DevPtrs& P, int m, int kp,
                                            double2 Xk, double2 Xp, int& tx0, int& tx1, int& ty0,
                                            int& ty1)
{
    double xmin = fmin(Xk.x, Xp.x) - 2.5, xmax = fmax(Xk.x, Xp.x) + 2.5;
    double ymin = fmin(Xk.y, Xp.y) - 2.5, ymax = fmax(Xk.y, Xp.y) + 2.5;
    if (I.geometry == 1) {
        // the spline segment lies in the hull of its Bezier control points
        const double2 Mk = P.M[m], Mp = P.M[I.mk_off + kp];
        const double bx = Xp.x - Xk.x - (2.0 * Mk.x + Mp.x) / 6.0;
        const double by = Xp.y - Xk.y - (2.0 * Mk.y + Mp.y) / 6.0;
        const double ex_ = Xp.x - Xk.x + (Mk.x + 2.0 * Mp.x) / 6.0;   // S'(1)
        const double ey_ = Xp.y - Xk.y + (Mk.y + 2.0 * Mp.y) / 6.0;
        const double c1x = Xk.x + bx / 3.0, c1y = Xk.y + by / 3.0;
        const double c2x = Xp.x - ex_ / 3.0, c2y = Xp.y - ey_ / 3.0;
        xmin = fmin(xmin, fmin(c1x, c2x) - 2.5);
        xmax = fmax(xmax, fmax(c1x, c2x) + 2.5);
        ymin = fmin(ymin, fmin(c1y, c2y) - 2.5);
        ymax = fmax(ymax, fmax(c1y, c2y) + 2.5);
    }
    if (!(xmin == xmin) || !(ymin == ymin) || !(xmax == xmax) || !(ymax == ymax)) return false;
    tx0 = max(0, (int)floor(fmax(xmin, 0.0) / kTile));
    tx1 = min(I.tiles_x - 1, (int)floor(fmin(xmax, (double)I.nx) / kTile));
    ty0 = max(0, (int)floor(fmax(ymin, 0.0) / kTile));
    ty1 = min(I.tiles_y - 1, (int)floor(fmin(ymax, (double)I.ny) / kTile));
    return true;
}

// Chord k at position `pos` of tile t's list (pos taken from the tile's
// count); the tile's first chord also lists the tile as active.
__device__ __forceinline__ void list_chord(const InstDev& I, const DevPtrs& P, int par, int k, int t,
                                           int pos)
{
    if (pos < I.tile_cap)
        P.tile_list[I.list_off + (long long)t * I.tile_cap + pos] = k;
    else
        atomicOr(&P.err[I.inst], (int)kErrCapacity);
    if (pos == 0) {
        const int a = atomicAdd(&P.act_count[2 * I.inst + par], 1);
        if (a < I.act_cap)
            P.act_list[par][I.act_off + a] = make_int2(I.inst, t);
        else
            atomicOr(&P.err[I.inst], (int)kErrCapacity);
    }
}

// Bin chord (k, k+1) into its tiles; the calling lanes take the tiles first,
// first + stride, ...
__device__ __forceinline__ void bin_chord(const InstDev& I, const DevPtrs& P, int par, int k, int m,
                                          int kp, double2 Xk, double2 Xp, int first, int stride)
{
    int tx0, tx1, ty0, ty1;
    if (!chord_tiles(I, P, m, kp, Xk, Xp, tx0, tx1, ty0, ty1)) return;
    const int tw = tx1 - tx0 + 1, ntile = tw * (ty1 - ty0 + 1);
    for (int q = first; q < ntile; q += stride) {
        const int t = (ty0 + q / tw) * I.tiles_x + tx0 + q % tw;
        list_chord(I, P, par, k, t, atomicAdd(&P.tile_count[I.tile_off + t], 1));
    }
}

// ---------------------------------------------------------------------------
// Markers: 16 lanes per marker, one per node of the 4 x 4 delta stencil.
//
// Step m uses three marker phases:
//   INTERP  U^m = sum_x u^m delta_h (Sec. 2.2.2, Eq. (20)) from f^m and, for a
//           membrane, X^{m+1} = X^m + U^m;
//   GEOM    from X^m: force, outward normal, |dX/ds|, [[p]] (Sec. 3.1,
//           Eq. (40)), tangential part (Sec. 3.2, Eq. (46)), the delta weights
//           used by the spread, and the binning of chord (k, k+1) into tiles;
//   FULL    both in one pass, for direct forcing, whose force needs U^m.
// A membrane's force depends on X only, so GEOM/tiles of step m+1 can run
// while the sweep of step m streams the lattice.
// ---------------------------------------------------------------------------
// Marker slots of the step: X^m lives in X[m & 1].
template <typename T, typename M, int MODE>
__device__ __forceinline__ void markers_body(const InstDev& I, const DevPtrs& P,
                                             const T* __restrict__ A, int par, int blk)
{
    const int gtid = blk * blockDim.x + threadIdx.x;
    const int N = I.n_markers;
    const int k = gtid >> 4;          // marker of this 16-lane group
    const int s = threadIdx.x & 15;   // stencil node of this lane
    const bool live = k < N;
    const double2* X = P.X[par] + I.mk_off;
    double2* Xn = P.X[par ^ 1] + I.mk_off;
    const double2 Xk = live ? X[k] : make_double2(0.0, 0.0);
    const bool inside =
        live && Xk.x >= 0.0 && Xk.x < (double)I.nx && Xk.y >= 0.0 && Xk.y < (double)I.ny;

    const int fx0 = inside ? (int)floor(Xk.x) - 1 : 0, fy0 = inside ? (int)floor(Xk.y) - 1 : 0;
    const int sx = s & 3, sy = s >> 2;
    const double wx = inside ? peskin((double)(fx0 + sx) - Xk.x) : 0.0;
    const double wy = inside ? peskin((double)(fy0 + sy) - Xk.y) : 0.0;

    double us = 0.0, vs = 0.0;
    if (MODE & kModeInterp) {
        // u^m of the pre-collision f^m at this lane's stencil node, weighted,
        // summed in FP64 over the group in a fixed tree.  Under Guo's term
        // u = (sum e f + g/2) / rho (Sec. 2.2.2): g is the body force plus,
        // for a membrane, the force this step's tile pass spread (the node's
        // slot of plane `par`); direct forcing's u* has the body force only.
        // A membrane under the IB-LBM comparison modes moves with its scheme's
        // velocity taken from the distributions after this step's force
        // (momentum sum e f + g): sum e f + g under the simple term,
        // (sum e f + 3 g / 2) / rho under Guo's.
        const double w = wx * wy;
        double cu = 0.0, cv = 0.0;
        if (w != 0.0) {
            M d[9];
            const int xs = wrap_or_clamp(fx0 + sx, I.nx, I.px);
            const int ys = wrap_or_clamp(fy0 + sy, I.ny, I.py);
            gather<T, M>(I, A, xs, ys, d);
            double u = 0.0, v = 0.0;
#pragma unroll
            for (int i = 1; i < 9; i++) {
                u += (double)EX[i] * (double)d[i];
                v += (double)EY[i] * (double)d[i];
            }
            const bool ib_membrane = !I.jumps && I.iface == II_LBM_IF_MEMBRANE;
            if (I.guo || ib_membrane) {
                double r = 0.0;
                if (I.guo) {
#pragma unroll
                    for (int i = 0; i < 9; i++) r += (double)d[i];
                }
                double gx = (double)I.body[0], gy = (double)I.body[1];
                if (!(MODE & kModeGeom)) {
                    const int slot =
                        P.tile_slot[par][I.tile_off + (ys / kTile) * I.tiles_x + (xs / kTile)];
                    const int node = (ys % kTile) * kTile + (xs % kTile);
                    if (slot >= 0 && corr_present(P.cmask[par], slot, node)) {
                        const float* c = P.corr[par] + (long long)slot * kCorrPlanes * kTileNodes + node;
                        gx += (double)c[8 * kTileNodes];
                        gy += (double)c[9 * kTileNodes];
                    }
                }
                const double c = ib_membrane ? (I.guo ? 1.5 : 1.0) : 0.5;
                u = (u + c * gx) / (1.0 + r);
                v = (v + c * gy) / (1.0 + r);
            }
            cu = u * w;
            cv = v * w;
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            cu += __shfl_xor(cu, off, 16);
            cv += __shfl_xor(cv, off, 16);
        }
        us = cu;
        vs = cv;
    }
    if (!live) return;
    const int m = I.mk_off + k;
    if (s == 0 && !inside) {
        // non-finite or outside the lattice: keep the marker, flag the handle
        atomicOr(&P.err[I.inst], isfinite(Xk.x) && isfinite(Xk.y) ? (int)kErrGeometry
                                                                  : (int)kErrUnstable);
        if (MODE & kModeInterp) {
            P.U[m] = make_double2(0.0, 0.0);
            Xn[k] = Xk;
        }
        if (MODE & kModeGeom) {
            P.G[m] = make_double2(0.0, 0.0);
            P.Gt[m] = make_double2(0.0, 0.0);
            P.jp[m] = 0.0;
        }
    }
    if (!inside) return;

    if ((MODE & kModeInterp) && s == 0) {
        P.U[m] = make_double2(us, vs);
        // X^{m+1} = X^m + U^m (Sec. 2.2.2, Eq. (20)); a fixed body stays put.
        double2 Xnew = Xk;
        if (I.iface == II_LBM_IF_MEMBRANE) Xnew = make_double2(Xk.x + us, Xk.y + vs);
        Xn[k] = Xnew;
        if (!isfinite(us) || !isfinite(vs)) atomicOr(&P.err[I.inst], (int)kErrUnstable);
        if (!(Xnew.x >= 3.0 && Xnew.x <= (double)(I.nx - 4) && Xnew.y >= 3.0 &&
              Xnew.y <= (double)(I.ny - 4)))
            atomicOr(&P.err[I.inst], (int)kErrGeometry);
    }
    if (!(MODE & kModeGeom)) return;

    // the per-axis delta weights, reused by the spread of this step
    if (sy == 0) P.wx[4 * m + sx] = wx;
    if (sx == 0) P.wy[4 * m + sy] = wy;
    const int km = (k + N - 1) % N, kp = (k + 1) % N;
    const double2 Xp = X[kp];
    if (s == 0) {
        P.f0[m] = make_int2(fx0, fy0);
        const double2 Xm = X[km];
        double gx, gy, nx_, ny_, jac;
        if (I.iface == II_LBM_IF_MEMBRANE) {
            membrane_geometry(I, P, m, kp, Xm, Xk, Xp, gx, gy, nx_, ny_, jac);
        } else if (I.iface == II_LBM_IF_NORMAL) {
            // prescribed uniform normal force F n on the fixed circle (Sec. 4.1)
            nx_ = (Xk.x - I.cx) / I.radius;
            ny_ = (Xk.y - I.cy) / I.radius;
            gx = I.f_normal * nx_;
            gy = I.f_normal * ny_;
            jac = 1.0;
        } else {
            // direct forcing to U^D with eta = 1 (Sec. 2.2.2, Eq. (18)): U^D = 0
            // for a fixed circle, U_c + W x (X - X_c) for a moving one;
            // |dX/ds| = 1 and the radial normal of the circle (Sec. 3.1)
            double ccx = I.cx, ccy = I.cy, ux_d = 0.0, uy_d = 0.0, wd = 0.0;
            if (I.moving) {
                const BodyDev& bd = P.body[I.inst];
                ccx = bd.c[0]; ccy = bd.c[1];
                ux_d = bd.U[0]; uy_d = bd.U[1]; wd = bd.W;
            }
            const double rx = Xk.x - ccx, ry = Xk.y - ccy;
            gx = (ux_d - wd * ry) - us;
            gy = (uy_d + wd * rx) - vs;
            nx_ = rx / I.radius;
            ny_ = ry / I.radius;
            jac = 1.0;
        }
        store_marker_force(P, m, gx, gy, nx_, ny_, jac);
    }
    bin_chord(I, P, par, k, m, kp, Xk, Xp, s, 16);   // one tile per lane of the group
}

// Membrane geometry (GEOM) of batched membranes, one thread per marker: the
// same values as the 16-lane form, whose per-marker arithmetic would run on
// one lane of 16.  The block's 256 consecutive chords bin to a few tiles:
// they are counted per tile in LDS first, so that each tile's global count
// takes one atomic per block (a chord's fifth and later tiles, and tiles
// beyond the LDS table, take theirs directly).  With hundreds of thousands
// of markers the per-chord atomics had made this pass 4.5 times longer.  The
// lists' order is immaterial: the tile pass orders every tile's chords by
// index.  (A single membrane of a few thousand markers keeps the 16-lane
// form, whose pass is shorter there.)
constexpr int kGeoHash = 128;   // distinct tiles of a block counted in LDS
constexpr int kGeoTiles = 4;    // tiles of one chord counted in LDS

__device__ __forceinline__ void geom_body(const InstDev& I, const DevPtrs& P, int par, int k)
{
    __shared__ int hkey[kGeoHash], hcnt[kGeoHash], hbase[kGeoHash];
    const int tid = threadIdx.x;
    for (int i = tid; i < kGeoHash; i += blockDim.x) {
        hkey[i] = -1;
        hcnt[i] = 0;
    }
    const int N = I.n_markers;
    int nt = 0, tx0 = 0, ty0 = 0, tw = 1;   // this thread's chord's tiles
    if (k < N) {
        const double2* X = P.X[par] + I.mk_off;
        const int m = I.mk_off + k;
        const double2 Xk = X[k];
        if (Xk.x >= 0.0 && Xk.x < (double)I.nx && Xk.y >= 0.0 && Xk.y < (double)I.ny) {
            const int fx0 = (int)floor(Xk.x) - 1, fy0 = (int)floor(Xk.y) - 1;
            // the per-axis delta weights, reused by the spread of this step
#pragma unroll
            for (int q = 0; q < 4; q++) {
                P.wx[4 * m + q] = peskin((double)(fx0 + q) - Xk.x);
                P.wy[4 * m + q] = peskin((double)(fy0 + q) - Xk.y);
            }
            P.f0[m] = make_int2(fx0, fy0);
            const int km = (k + N - 1) % N, kp = (k + 1) % N;
            const double2 Xm = X[km], Xp = X[kp];
            double gx, gy, nx_, ny_, jac;
            membrane_geometry(I, P, m, kp, Xm, Xk, Xp, gx, gy, nx_, ny_, jac);
            store_marker_force(P, m, gx, gy, nx_, ny_, jac);
            int tx1, ty1;
            if (chord_tiles(I, P, m, kp, Xk, Xp, tx0, tx1, ty0, ty1)) {
                tw = tx1 - tx0 + 1;
                nt = tw * (ty1 - ty0 + 1);
            }
        } else {
            // non-finite or outside the lattice: keep the marker, flag the handle
            atomicOr(&P.err[I.inst], isfinite(Xk.x) && isfinite(Xk.y) ? (int)kErrGeometry
                                                                      : (int)kErrUnstable);
            P.G[m] = make_double2(0.0, 0.0);
            P.Gt[m] = make_double2(0.0, 0.0);
            P.jp[m] = 0.0;
        }
    }
    __syncthreads();
    int hs[kGeoTiles], lp[kGeoTiles];
#pragma unroll
    for (int q = 0; q < kGeoTiles; q++) {
        hs[q] = -1;
        lp[q] = 0;
        if (q >= nt) continue;
        const int t = (ty0 + q / tw) * I.tiles_x + tx0 + q % tw;
        unsigned h = ((unsigned)t * 2654435761u) >> 25;   // 7 bits: kGeoHash = 128
        for (int probe = 0; probe < kGeoHash; probe++) {
            const int prev = atomicCAS(&hkey[h], -1, t);
            if (prev == -1 || prev == t) {
                hs[q] = (int)h;
                break;
            }
            h = (h + 1) & (kGeoHash - 1);
        }
        if (hs[q] >= 0)
            lp[q] = atomicAdd(&hcnt[hs[q]], 1);
        else
            list_chord(I, P, par, k, t, atomicAdd(&P.tile_count[I.tile_off + t], 1));
    }
    for (int q = kGeoTiles; q < nt; q++) {
        const int t = (ty0 + q / tw) * I.tiles_x + tx0 + q % tw;
        list_chord(I, P, par, k, t, atomicAdd(&P.tile_count[I.tile_off + t], 1));
    }
    __syncthreads();
    for (int i = tid; i < kGeoHash; i += blockDim.x)
        if (hkey[i] >= 0) hbase[i] = atomicAdd(&P.tile_count[I.tile_off + hkey[i]], hcnt[i]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kGeoTiles; q++)
        if (hs[q] >= 0) list_chord(I, P, par, k, hkey[hs[q]], hbase[hs[q]] + lp[q]);
}

// Before the tiles of step m are binned: the tiles of step m-2 (same slot
// plane) give their correction slots back, and the active-tile and record
// counts of that plane restart.  One block per instance.
__device__ __forceinline__ void slot_reset_body(const InstDev& I, const DevPtrs& P, int par)
{
    const int prev = min(P.act_count[2 * I.inst + par], I.act_cap);
    int* slot = P.tile_slot[par];
    for (int a = threadIdx.x; a < prev; a += blockDim.x)
        slot[I.tile_off + P.act_list[par][I.act_off + a].y] = -1;
    __syncthreads();
    if (threadIdx.x == 0) {
        P.act_count[2 * I.inst + par] = 0;
        P.rec_count[2 * I.inst + par] = 0;
    }
}

template <typename T, typename M, int MODE>
__global__ __launch_bounds__(256) void k_markers(InstDev I, DevPtrs P, const T* __restrict__ A,
                                                 int par)
{
    // The interpolation of step m (for membranes) or the marker pass of step m
    // (FULL, direct forcing) also resets the slot plane of step m+1, last
    // read by the sweep of step m-1, which has finished: the interface pass
    // of step m+1 needs no launch of its own for it.
    if ((MODE == kModeInterp || MODE == kModeFull) && blockIdx.x == 0)
        slot_reset_body(I, P, par ^ 1);
    markers_body<T, M, MODE>(I, P, A, par, blockIdx.x);
}

// Batched: every block looks its (instance, block) up in a work table.
template <typename T, typename M, int MODE>
__global__ __launch_bounds__(256) void k_markers_batch(const InstDev* __restrict__ insts,
                                                       const int2* __restrict__ units, int n_units,
                                                       DevPtrs P, const T* __restrict__ A, int par)
{
    // workgroup b runs on XCD b mod 8: give each XCD one contiguous run of
    // the table, so that neighbouring markers share that XCD's L2
    const int per = gridDim.x / 8;
    const int idx = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (idx >= n_units) return;   // padding of the grid (whole block)
    const int2 u = units[idx];
    const InstDev I = insts[u.x];
    if ((MODE == kModeInterp || MODE == kModeFull) && u.y == 0)
        slot_reset_body(I, P, par ^ 1);   // as in k_markers
    markers_body<T, M, MODE>(I, P, A, par, u.y);
}

__global__ __launch_bounds__(256) void k_geom_batch(const InstDev* __restrict__ insts,
                                                    const int2* __restrict__ units, DevPtrs P,
                                                    int par)
{
    const int2 u = units[blockIdx.x];
    const InstDev I = insts[u.x];
    geom_body(I, P, par, u.y * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_slot_reset(InstDev I, DevPtrs P, int par)
{
    slot_reset_body(I, P, par);
}

__global__ __launch_bounds__(64) void k_slot_reset_batch(const InstDev* __restrict__ insts,
                                                           DevPtrs P, int par)
{
    const InstDev I = insts[blockIdx.x];
    if (I.n_markers > 0) slot_reset_body(I, P, par);
}

template <typename T, int MODE>
static hipError_t markers_t(const InstDev& I, const DevPtrs& P, const void* A, int par,
                            hipStream_t s)
{
    const int nb = I.mk_blocks;
    if (I.math == II_LBM_MATH_FP64)
        hipLaunchKernelGGL((k_markers<T, double, MODE>), dim3(nb), dim3(256), 0, s, I, P,
                           (const T*)A, par);
    else
        hipLaunchKernelGGL((k_markers<T, float, MODE>), dim3(nb), dim3(256), 0, s, I, P,
                           (const T*)A, par);
    return hipGetLastError();
}

template <int MODE>
static hipError_t markers_m(const InstDev& I, const DevPtrs& P, const void* A, int par,
                            hipStream_t s)
{
    return I.storage == II_LBM_FP16 ? markers_t<_Float16, MODE>(I, P, A, par, s)
                                    : markers_t<float, MODE>(I, P, A, par, s);
}

hipError_t launch_markers(const InstDev& I, const DevPtrs& P, const void* A, int par, int mode,
                          hipStream_t s)
{
    if (I.n_markers == 0) return hipSuccess;
    if (mode == kModeInterp) return markers_m<kModeInterp>(I, P, A, par, s);
    if (mode == kModeGeom) return markers_m<kModeGeom>(I, P, A, par, s);
    return markers_m<kModeFull>(I, P, A, par, s);
}

template <typename T, int MODE>
static hipError_t markers_batch_t(const Batch& b, const DevPtrs& P, const void* A, int par,
                                  hipStream_t s)
{
    const dim3 grid(8 * ((b.mk_units + 7) / 8));
    if (b.math == II_LBM_MATH_FP64)
        hipLaunchKernelGGL((k_markers_batch<T, double, MODE>), grid, dim3(256), 0, s, b.insts,
                           b.mk_table, b.mk_units, P, (const T*)A, par);
    else
        hipLaunchKernelGGL((k_markers_batch<T, float, MODE>), grid, dim3(256), 0, s, b.insts,
                           b.mk_table, b.mk_units, P, (const T*)A, par);
    return hipGetLastError();
}

template <int MODE>
static hipError_t markers_batch_m(const Batch& b, const DevPtrs& P, const void* A, int par,
                                  hipStream_t s)
{
    return b.storage == II_LBM_FP16 ? markers_batch_t<_Float16, MODE>(b, P, A, par, s)
                                    : markers_batch_t<float, MODE>(b, P, A, par, s);
}

hipError_t launch_markers_batch(const Batch& b, const DevPtrs& P, const void* A, int par, int mode,
                                hipStream_t s)
{
    if (b.mk_units == 0) return hipSuccess;
    if (mode == kModeInterp) return markers_batch_m<kModeInterp>(b, P, A, par, s);
    if (mode == kModeGeom && b.iface == II_LBM_IF_MEMBRANE) {
        hipLaunchKernelGGL(k_geom_batch, dim3(b.geo_units), dim3(256), 0, s, b.insts, b.geo_table,
                           P, par);
        return hipGetLastError();
    }
    if (mode == kModeGeom) return markers_batch_m<kModeGeom>(b, P, A, par, s);
    return markers_batch_m<kModeFull>(b, P, A, par, s);
}

hipError_t launch_slot_reset(const InstDev& I, const DevPtrs& P, int par, hipStream_t s)
{
    if (I.n_markers == 0) return hipSuccess;
    hipLaunchKernelGGL(k_slot_reset, dim3(1), dim3(256), 0, s, I, P, par);
    return hipGetLastError();
}

hipError_t launch_slot_reset_batch(const Batch& b, int n_inst, const DevPtrs& P, int par,
                                   hipStream_t s)
{
    if (b.mk_units == 0) return hipSuccess;
    hipLaunchKernelGGL(k_slot_reset_batch, dim3(n_inst), dim3(64), 0, s, b.insts, P, par);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact link/chord crossing on the 2^-16 snapped grid.
//
// For the chord A->B and the link P->P+e (P a lattice node, e a D2Q9 vector)
// every orientation is an int64 (|coordinates| < 2^29, products < 2^61):
//   oP = orient(A, B, P) = dx (P.y - A.y) - dy (P.x - A.x),  (dx, dy) = B - A
//   orient(A, B, P + e) = oP + 2^16 (dx e_y - dy e_x)
//   orient(P, P + e, A) = 2^16 (e_x (A.y - P.y) - e_y (A.x - P.x))
// Ties are broken as if every lattice node sat at (+eps, +eps^2): the side of
// a node on the chord's line follows -dy, then dx; the side of a chord end on
// the link's line follows e_y, then -e_x.  No orientation is then zero and the
// count of crossings of a link equals inside(P) != inside(P + e).
// ---------------------------------------------------------------------------
struct Chord {
    long long ax, ay, bx, by;
};

__device__ __forceinline__ int node_sign(long long o, long long dx, long long dy)
{
    if (o != 0) return o > 0 ? 1 : -1;
    if (dy != 0) return dy > 0 ? -1 : 1;
    return dx > 0 ? 1 : -1;
}

__device__ __forceinline__ int end_sign(long long o, int ex, int ey)
{
    if (o != 0) return o > 0 ? 1 : -1;
    if (ey != 0) return ey;
    return -ex;
}

// Crossing of the link leaving lattice node (x, y) along e_i with chord c.
// On a hit returns true with the sign sigma (+1 from the interior, which lies
// left of A->B, to the exterior) and, when wanted, q and theta.
template <bool FRACS>
__device__ __forceinline__ bool link_crossing(int x, int y, int i, const Chord& c, long long oP,
                                              int sP, int& sigma, double& q, double& theta)
{
    const long long dx = c.bx - c.ax, dy = c.by - c.ay;
    const int ex = EX[i], ey = EY[i];
    const long long oQ = oP + ((dx * ey - dy * ex) << 16);
    if (node_sign(oQ, dx, dy) == sP) return false;
    const long long px = (long long)x << 16, py = (long long)y << 16;
    const long long oA = (long long)ex * (c.ay - py) - (long long)ey * (c.ax - px);
    const long long oB = (long long)ex * (c.by - py) - (long long)ey * (c.bx - px);
    if (end_sign(oA, ex, ey) == end_sign(oB, ex, ey)) return false;
    sigma = sP;
    const double a = (double)(oA << 16), b = (double)(oB << 16);
    theta = a / (a - b);
    if (FRACS) q = (double)oP / ((double)oP - (double)oQ);
    return true;
}

// Cut point of the link from node (x, y) along e_i on the rigid circle
// |x - c| = R (the root of |P + q e_i - c|^2 = R^2 inside the link), and the
// marker interval that brackets it by angle: [[p]] there is linear in the
// angle between markers k and k+1.
// (cx, cy, th0): the circle's centre and orientation this step (a moving
// body's marker k sits at angle th0 + 2 pi k / N, th0 in [0, 2 pi)).
// Velocity and weight of link direction i (1..8) when i differs across the
// lanes of a wave: decoded from packed constants rather than read from a table.
__device__ __forceinline__ int link_ex(int i) { return (int)((0x20919u >> (2 * i)) & 3u) - 1; }
__device__ __forceinline__ int link_ey(int i) { return (int)((0x2865u >> (2 * i)) & 3u) - 1; }
__device__ __forceinline__ double link_w(int i) { return i < 5 ? WD[1] : WD[5]; }

__device__ __forceinline__ void rigid_cut(const InstDev& I, double cx, double cy, double th0,
                                          int x, int y, int i, bool inP, double& q, double& th,
                                          int& k)
{
    const int N = I.n_markers;
    const int ex = link_ex(i), ey = link_ey(i);
    const double R2 = I.radius * I.radius;
    const double dx = (double)x - cx, dy = (double)y - cy;
    const double ee = (double)(ex * ex + ey * ey);
    const double de = dx * ex + dy * ey;
    const double dd = dx * dx + dy * dy - R2;
    const double disc = sqrt(de * de - ee * dd);
    q = inP ? (-de + disc) / ee : (-de - disc) / ee;
    const double cxp = (double)x + q * ex - cx, cyp = (double)y + q * ey - cy;
    double ang = atan2(cyp, cxp) - th0;
    if (ang < 0.0) ang += 2.0 * M_PI;
    if (ang < 0.0) ang += 2.0 * M_PI;
    if (ang >= 2.0 * M_PI) ang -= 2.0 * M_PI;
    // an angle an ulp below 2 pi can round sN up to exactly N: that crossing
    // belongs to the last interval, at its far end (th = 1)
    const double sN = ang * N / (2.0 * M_PI);
    k = sN >= 0.0 ? min((int)floor(sN), N - 1) : 0;
    th = sN - k;
}

// ---------------------------------------------------------------------------
// Tiles.
// ---------------------------------------------------------------------------
constexpr int kTileRec = 1024;  // cut links recorded per tile (packed in LDS, then written)
static_assert(kTileCap <= 256, "chord ranks of a tile are kept in bytes");

// LDS of one tile block: about 24 KB (six blocks share a CU), and 4 KB more
// with the cut-link record stage.  kTileCap <= 256 (chord ranks fit a byte).
template <bool REC>
struct TileShared {
    union {
        int raw[kTileCap];       // chord ids as binned
        int start[kTileCap];     // first flattened candidate of each sorted chord
    };
    int key[kTileCap];           // chord ids in increasing order
    Chord ch[kTileCap];
    short box[kTileCap][4];      // candidate source nodes of the chord's links
    int winv[kTileCap];          // ceil(2^16 / box width): q / w as (q * winv) >> 16
    double jpa[kTileCap], jpb[kTileCap];
    float wx[kTileCap][4], wy[kTileCap][4];
    int2 f0[kTileCap];
    double gtx[kTileCap], gty[kTileCap];   // G_par dX of each chord's marker
    int acc[8][kTileNodes];      // jump sums of the eight outgoing populations per node
    unsigned char strip[4][kTileCap];   // per wave: chords whose stencil meets its 4 rows
    int strip_n[4];
    unsigned rec[REC ? kTileRec : 1];   // packed (node, direction, chord) of each cut link
    int cnt, total, nrec, base;
    unsigned jmax;               // bits of the largest |[[p]]| at the tile's chords' ends
};

// [[f_i]] of one cut link into the node's accumulator: sigma w_i [[p]] / c_s^2
// (Sec. 3.1, Eq. (32); Sec. 3.2, Eq. (47)).  A link cut by several chords
// (a wrinkled membrane) gets one term per crossing.  The sums are kept in
// fixed point, so that they are exact and do not depend on the order in which
// the threads add their crossings; a non-finite term marks the instance
// unstable.
//  - The membrane and rigid tile pass sums in 32 bits at a power-of-two scale
//    of its own: each term is at most (max |[[p]]| over the tile's chord ends)
//    w_1 / c_s^2, which the scale maps to at most 2^27 (sixteen crossings of
//    one link fit in an int), so a term keeps at least 27 bits relative to
//    the tile's largest, finer than the FP32 correction slot it ends in.
//  - The spline tile pass (whose [[p]] comes from the spline) sums in 64 bits
//    at 2^-56 resolution, terms clamped to 64 in magnitude.
constexpr double kJumpFix = 72057594037927936.0;   // 2^56

template <class TS>
__device__ __forceinline__ void add_jump(TS& S, int node, int i, int sigma, double jpc, int* err,
                                         double scale = kJumpFix)
{
    const double v = (double)sigma * link_w(i) * jpc / kCs2;
    if (!isfinite(v)) {
        atomicOr(err, (int)kErrUnstable);
        return;
    }
    if constexpr (sizeof(S.acc[0][0]) == 8) {
        const long long q = __double2ll_rn(fmin(fmax(v, -64.0), 64.0) * kJumpFix);
        atomicAdd((unsigned long long*)&S.acc[i - 1][node], (unsigned long long)q);
    } else {
        const double b = 134217728.0;   // 2^27
        atomicAdd(&S.acc[i - 1][node], __double2int_rn(fmin(fmax(v * scale, -b), b)));
    }
}

__device__ __forceinline__ double jump_sum(long long acc) { return (double)acc * (1.0 / kJumpFix); }
// (inv_scale is the exact reciprocal of the tile's power-of-two scale)
__device__ __forceinline__ double jump_sum(int acc, double inv_scale) { return (double)acc * inv_scale; }

// The power of two that maps the tile's largest jump term to at most 2^27.
__device__ __forceinline__ double jump_scale(unsigned jmax_bits)
{
    const float jm = __uint_as_float(jmax_bits) * (float)(WD[1] / kCs2);
    if (!(jm > 0.f) || !isfinite(jm)) return 1.0;
    int e;
    frexpf(jm, &e);                 // jm < 2^e
    return ldexp(1.0, 27 - e);
}

template <class TS>
__device__ __forceinline__ void stage_record(TS& S, int node, int i, int j)
{
    const int r = atomicAdd(&S.nrec, 1);
    if (r < kTileRec) S.rec[r] = (unsigned)node | ((unsigned)(i - 1) << 8) | ((unsigned)j << 11);
}

// REC: also write the cut-link records of the tile (packed in LDS, then
// expanded by recomputing each crossing).
template <int IFACE, bool REC>
__device__ __forceinline__ void tiles_body(const InstDev& I, const DevPtrs& P, int parity, int blk,
                                           int nblk)
{
    __shared__ TileShared<REC> S;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int N = I.n_markers;
    const double2* X = P.X[parity] + I.mk_off;
    const int nact = min(P.act_count[2 * I.inst + parity], I.act_cap);
    for (int a = blk; a < nact; a += nblk) {
        const int t = P.act_list[parity][I.act_off + a].y;
        const int gt = I.tile_off + t;
        const int tx = t % I.tiles_x, ty = t / I.tiles_x;
        const int x0 = tx * kTile, y0 = ty * kTile;
        // the list is read whole (its slots beyond the count are stale but
        // allocated) while thread 0 reads the count
        if (tid < kTileCap) S.raw[tid] = P.tile_list[I.list_off + (long long)t * kTileCap + tid];
        if (tid == 0) {
            S.cnt = min(P.tile_count[gt], kTileCap);
            S.nrec = 0;
            S.jmax = 0u;
        }
#pragma unroll
        for (int i = 0; i < 8; i++) S.acc[i][tid] = 0;
        __syncthreads();
        const int c = S.cnt;
        if (tid == 0) {
            P.tile_count[gt] = 0;  // ready for the next step
            P.tile_slot[parity][gt] = I.act_off + a;
        }
        // deterministic order: chord k goes to its rank among the (distinct)
        // ids; its marker data are requested first and arrive during the rank
        // count
        int k = 0, r = 0;
        double2 a0 = make_double2(0.0, 0.0), b0 = a0, g = a0;
        double jpa = 0.0, jpb = 0.0, wxd[4] = {0.0, 0.0, 0.0, 0.0}, wyd[4] = {0.0, 0.0, 0.0, 0.0};
        int2 f0 = make_int2(0, 0);
        if (tid < c) {
            k = S.raw[tid];
            const int kp = (k + 1) % N, mk = I.mk_off + k;
            a0 = X[k];
            b0 = X[kp];
            jpa = P.jp[mk];
            jpb = P.jp[I.mk_off + kp];
            f0 = P.f0[mk];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                wxd[q] = P.wx[4 * mk + q];
                wyd[q] = P.wy[4 * mk + q];
            }
            g = I.jumps ? P.Gt[mk] : P.G[mk];
            for (int m = 0; m < c; m++) r += (S.raw[m] < k) ? 1 : 0;
            // |[[p]]| bits order as the values for non-negative floats
            atomicMax(&S.jmax, __float_as_uint((float)fmax(fabs(jpa), fabs(jpb))));
        }
        __syncthreads();   // raw is reused as start below
        const double jscale = jump_scale(S.jmax), jinv = 1.0 / jscale;
        if (tid < c) {
            S.key[r] = k;
            const long long ax = (long long)rint(a0.x * kSnap), ay = (long long)rint(a0.y * kSnap);
            const long long bx = (long long)rint(b0.x * kSnap), by = (long long)rint(b0.y * kSnap);
            S.ch[r].ax = ax; S.ch[r].ay = ay; S.ch[r].bx = bx; S.ch[r].by = by;
            // Source nodes of the links the chord can cut.  A link's span in x
            // is [P.x, P.x + e_x] with the node shifted by the tie-breaking
            // +eps; it meets the chord's [lo, hi] only if ceil(lo) - 1 <=
            // P.x <= ceil(hi) (e_x = +1 gives the low end, e_x = -1 the high
            // one), and likewise in y.  Keep that box's part in this tile.
            const int bx0 = max((int)(-((-min(ax, bx)) >> 16)) - 1, x0);
            const int bx1 = min((int)(-((-max(ax, bx)) >> 16)), min(x0 + kTile, I.nx) - 1);
            const int by0 = max((int)(-((-min(ay, by)) >> 16)) - 1, y0);
            const int by1 = min((int)(-((-max(ay, by)) >> 16)), min(y0 + kTile, I.ny) - 1);
            S.box[r][0] = (short)bx0; S.box[r][1] = (short)bx1;
            S.box[r][2] = (short)by0; S.box[r][3] = (short)by1;
            S.start[r] = (IFACE == II_LBM_IF_MEMBRANE && I.jumps && bx0 <= bx1 && by0 <= by1)
                             ? (bx1 - bx0 + 1) * (by1 - by0 + 1) : 0;
            // exact for widths up to 16 and candidates q < 256 (the box lies in the tile)
            S.winv[r] = bx0 <= bx1 ? (65536 + bx1 - bx0) / (bx1 - bx0 + 1) : 0;
            S.jpa[r] = jpa;
            S.jpb[r] = jpb;
            S.f0[r] = f0;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                S.wx[r][q] = (float)wxd[q];
                S.wy[r][q] = (float)wyd[q];
            }
            S.gtx[r] = g.x * I.dX; S.gty[r] = g.y * I.dX;   // G_par dX
        }
        __syncthreads();

        // Each wave spreads onto four rows of the tile (y0 + 4 wid ...): list,
        // in rank order, the chords whose marker stencil (rows f0.y ...
        // f0.y + 3) meets them.
        {
            const int r0 = y0 + 4 * wid;
            int n = 0;
            for (int base = 0; base < c; base += 64) {
                const int j = base + lane;
                const bool hit = j < c && S.f0[j].y <= r0 + 3 && S.f0[j].y + 3 >= r0;
                const unsigned long long m = __ballot(hit);
                if (hit) S.strip[wid][n + __popcll(m & ((1ull << lane) - 1ull))] = (unsigned char)j;
                n += __popcll(m);
            }
            if (lane == 0) S.strip_n[wid] = n;
        }
        if (IFACE != II_LBM_IF_MEMBRANE) __syncthreads();

        // Cut links of a membrane.  The (chord, source node) candidates of all
        // chords are numbered consecutively and every thread of the block takes
        // every 256th; a thread finds the side of its node once and then tests
        // the eight links the node sends.
        if (IFACE == II_LBM_IF_MEMBRANE) {
            if (wid == 0) {
                // exclusive scan of the candidate counts, two chords per lane
                const int v0 = 2 * lane < c ? S.start[2 * lane] : 0;
                const int v1 = 2 * lane + 1 < c ? S.start[2 * lane + 1] : 0;
                int sc = v0 + v1;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int u = __shfl_up(sc, off);
                    if (lane >= off) sc += u;
                }
                if (2 * lane < c) S.start[2 * lane] = sc - v0 - v1;
                if (2 * lane + 1 < c) S.start[2 * lane + 1] = sc - v1;
                if (lane == 63) S.total = sc;
            }
            __syncthreads();
            const int total = S.total;
            for (int g = tid; g < total; g += blockDim.x) {
                int lo = 0, hi = c - 1;   // last chord whose range starts at or before g
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (S.start[mid] <= g) lo = mid; else hi = mid - 1;
                }
                const int j = lo, q = g - S.start[j];
                const int bx0 = S.box[j][0], by0 = S.box[j][2];
                const int w = S.box[j][1] - bx0 + 1;
                const int qy = (q * S.winv[j]) >> 16;
                const int x = bx0 + q - qy * w, y = by0 + qy;
                const Chord ch = S.ch[j];
                const long long dx = ch.bx - ch.ax, dy = ch.by - ch.ay;
                const long long oP = dx * (((long long)y << 16) - ch.ay) - dy * (((long long)x << 16) - ch.ax);
                const int sP = node_sign(oP, dx, dy);
                const int node = (y - y0) * kTile + (x - x0);
#pragma unroll
                for (int i = 1; i < 9; i++) {
                    int sg;
                    double qq, th;
                    if (!link_crossing<false>(x, y, i, ch, oP, sP, sg, qq, th)) continue;
                    add_jump(S, node, i, sg, (1.0 - th) * S.jpa[j] + th * S.jpb[j], P.err + I.inst,
                             jscale);
                    if constexpr (REC) stage_record(S, node, i, j);
                }
            }
        }

        const int lx = tid & (kTile - 1), ly = tid / kTile;
        const int x = x0 + lx, y = y0 + ly;
        const bool valid = x < I.nx && y < I.ny;
        double gx = 0.0, gy = 0.0;
        if (valid) {
            // tangential force g_par(x) = sum_k G_par,k delta_h(x - X_k) dX (Sec. 3.2, Eq. (46))
            // with the delta weights of marker k from the marker pass, over
            // the markers whose stencil meets the wave's rows; those that miss
            // this node add an exact zero
            const int nw = S.strip_n[wid];
#pragma unroll 4
            for (int n = 0; n < nw; n++) {
                const int j = S.strip[wid][n];
                const int2 f = S.f0[j];
                const int ix = x - f.x, iy = y - f.y;
                const bool in = (unsigned)ix <= 3u && (unsigned)iy <= 3u;
                const double wgt = in ? (double)S.wx[j][ix & 3] * (double)S.wy[j][iy & 3] : 0.0;
                gx += S.gtx[j] * wgt;
                gy += S.gty[j] * wgt;
            }
            if (IFACE == II_LBM_IF_RIGID && I.jumps) {
                // Rigid circle: level set phi = |x - c|^2 - R^2, interior phi < 0.
                double ccx = I.cx, ccy = I.cy, th0 = 0.0;
                if (I.moving) {
                    ccx = P.body[I.inst].c[0];
                    ccy = P.body[I.inst].c[1];
                    th0 = P.body[I.inst].theta_mod;
                }
                const double R2 = I.radius * I.radius;
                const double dx = (double)x - ccx, dy = (double)y - ccy;
                const double phP = dx * dx + dy * dy - R2;
                const bool inP = phP < 0.0;
                // the links whose far end lies on the other side; the wave then
                // walks each lane's cut links together (as many passes as the
                // most any lane has, not one per direction any lane cuts)
                unsigned cut = 0u;
#pragma unroll
                for (int i = 1; i < 9; i++) {
                    const double qxd = (double)(x + EX[i]), qyd = (double)(y + EY[i]);
                    const double phQ = (qxd - ccx) * (qxd - ccx) + (qyd - ccy) * (qyd - ccy) - R2;
                    if ((phQ < 0.0) != inP) cut |= 1u << i;
                }
                while (cut != 0u) {
                    const int i = __builtin_ctz(cut);
                    cut &= cut - 1u;
                    double q, th;
                    int k;
                    rigid_cut(I, ccx, ccy, th0, x, y, i, inP, q, th, k);
                    const double jpc =
                        (1.0 - th) * P.jp[I.mk_off + k] + th * P.jp[I.mk_off + (k + 1) % N];
                    add_jump(S, tid, i, inP ? 1 : -1, jpc, P.err + I.inst, jscale);
                    if constexpr (REC) stage_record(S, tid, i, 0);
                }
            }
        }
        __syncthreads();

        // Corrections of this node's outgoing populations: the simple force
        // term of the spread force plus the jumps of the links it sends; the
        // sweep adds them before its single store.  Under Guo's term the
        // populations take the jumps alone and the force itself follows.
        // Only nodes with a non-zero correction are written; the slot's mask
        // tells the readers which.
        {
            float* cr = P.corr[parity] + (long long)(I.act_off + a) * kCorrPlanes * kTileNodes + tid;
            const double fs = I.guo ? 0.0 : 3.0;
            float dl[8];
            bool nz = false;
#pragma unroll
            for (int i = 1; i < 9; i++) {
                const double delta =
                    valid ? fs * WD[i] * ((double)EX[i] * gx + (double)EY[i] * gy) +
                                jump_sum(S.acc[i - 1][tid], jinv)
                          : 0.0;
                dl[i - 1] = (float)delta;
                nz = nz || dl[i - 1] != 0.f;
            }
            const float fgx = valid ? (float)gx : 0.f, fgy = valid ? (float)gy : 0.f;
            if (I.guo) nz = nz || fgx != 0.f || fgy != 0.f;
            const unsigned long long m = __ballot(nz);
            if (lane == 0) P.cmask[parity][(long long)(I.act_off + a) * 4 + wid] = m;
            if (nz) {
#pragma unroll
                for (int i = 0; i < 8; i++) cr[i * kTileNodes] = dl[i];
                if (I.guo) {
                    cr[8 * kTileNodes] = fgx;
                    cr[9 * kTileNodes] = fgy;
                }
            }
        }
        // Records of this tile: one global slice for the block; each is
        // expanded from its packed form by recomputing the crossing.
        if constexpr (REC) {
            const int nr = min(S.nrec, kTileRec);
            if (tid == 0) {
                S.base = nr > 0 ? atomicAdd(&P.rec_count[2 * I.inst + parity], nr) : 0;
                if (S.nrec > kTileRec) atomicOr(&P.err[I.inst], (int)kErrRecords);
            }
            __syncthreads();
            const int base = S.base;
            for (int rr = tid; rr < nr; rr += blockDim.x) {
                if (base + rr >= I.rec_cap) {
                    atomicOr(&P.err[I.inst], (int)kErrRecords);
                    continue;
                }
                const unsigned pk = S.rec[rr];
                const int node = pk & 255, i = 1 + ((pk >> 8) & 7), j = pk >> 11;
                const int x = x0 + (node & (kTile - 1)), y = y0 + node / kTile;
                ii_lbm_link L;
                L.x = x; L.y = y; L.dir = i; L.inst = I.inst;
                if (IFACE == II_LBM_IF_MEMBRANE) {
                    const Chord ch = S.ch[j];
                    const long long dx = ch.bx - ch.ax, dy = ch.by - ch.ay;
                    const long long oP = dx * (((long long)y << 16) - ch.ay) - dy * (((long long)x << 16) - ch.ax);
                    int sg = 0;
                    double qq = 0.0, th = 0.0;
                    (void)link_crossing<true>(x, y, i, ch, oP, node_sign(oP, dx, dy), sg, qq, th);
                    L.sigma = sg; L.seg = S.key[j]; L.q = qq; L.theta = th;
                    L.jp = (1.0 - th) * S.jpa[j] + th * S.jpb[j];
                } else {
                    double ccx = I.cx, ccy = I.cy, th0 = 0.0;
                    if (I.moving) {
                        ccx = P.body[I.inst].c[0];
                        ccy = P.body[I.inst].c[1];
                        th0 = P.body[I.inst].theta_mod;
                    }
                    const double dx = (double)x - ccx, dy = (double)y - ccy;
                    const bool inP = dx * dx + dy * dy - I.radius * I.radius < 0.0;
                    double q, th;
                    int k;
                    rigid_cut(I, ccx, ccy, th0, x, y, i, inP, q, th, k);
                    L.sigma = inP ? 1 : -1; L.seg = k; L.q = q; L.theta = th;
                    L.jp = (1.0 - th) * P.jp[I.mk_off + k] + th * P.jp[I.mk_off + (k + 1) % N];
                }
                P.rec[I.rec_off + base + rr] = L;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Cubic-spline membranes.
//   k_spline  M_k of the periodic cubic spline through the markers, from the
//             closed-form inverse of the cyclic system M_{k-1} + 4 M_k +
//             M_{k+1} = r_k, r_k = 6 (X_{k+1} - 2 X_k + X_{k-1}): M_k =
//             sum_j g_j r_{k+j} with g_j = lambda^|j| / (2 sqrt 3), lambda =
//             sqrt 3 - 2, truncated at |j| <= 32 (|lambda|^33 < 1e-18), or, for
//             N <= 64 markers, its periodic sum over every j (taps from the host).
//   k_tiles_spline  the tile pass on the spline: the crossings of each link
//             with each segment are the roots of the cubic e x (S(t) - P),
//             split at its critical points and bisected 64 times; [[p]] at a
//             crossing is dX (G x T) / |T|^2 with T = S'(t), G linear between
//             the markers.
// ---------------------------------------------------------------------------
// One 64-lane wave per marker, one or two taps per lane, summed by shuffles.
__global__ __launch_bounds__(256) void k_spline(InstDev I, DevPtrs P, int par)
{
    const int N = I.n_markers;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= N) return;   // whole waves leave together
    const double2* X = P.X[par] + I.mk_off;
    const double* g = P.spline_taps + I.tap_off;
    const int j0 = I.spl_periodic ? 0 : -32, ntap = I.spl_periodic ? N : 65;
    double mx = 0.0, my = 0.0;
    for (int u = lane; u < ntap; u += 64) {
        const int j = j0 + u;
        const int q = ((k + j) % N + N) % N;
        const int qm = q == 0 ? N - 1 : q - 1, qp = q == N - 1 ? 0 : q + 1;
        const double2 a = X[qm], b = X[q], c = X[qp];
        const double gj = g[u];
        mx += gj * (6.0 * (c.x - 2.0 * b.x + a.x));
        my += gj * (6.0 * (c.y - 2.0 * b.y + a.y));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mx += __shfl_xor(mx, off, 64);
        my += __shfl_xor(my, off, 64);
    }
    if (lane == 0) P.M[I.mk_off + k] = make_double2(mx, my);
}

hipError_t launch_spline(const InstDev& I, const DevPtrs& P, int par, hipStream_t s)
{
    hipLaunchKernelGGL(k_spline, dim3((I.n_markers + 3) / 4), dim3(256), 0, s, I, P, par);
    return hipGetLastError();
}

__device__ __forceinline__ double spl_cubic(const double F[4], double t)
{
    return ((F[3] * t + F[2]) * t + F[1]) * t + F[0];
}

// Crossings of link (px, py) -> + (ex, ey) with a segment: cf = (ax, ay, bx,
// by, cx, cy, dx, dy, X_{k+1}x, X_{k+1}y, B1x, B1y, B2x, B2y) with the inner
// Bezier control points B1 = a + b/3, B2 = a + (2b + c)/3.  Writes up to 3
// (t, q, sigma).
__device__ int spl_crossings(const double* cf, double px, double py, int ex, int ey, double* ts,
                             double* qs, int* sg)
{
    // control-point hull test: B0 = a, B1, B2, B3 = X_{k+1}
    const double b0 = ex * (cf[1] - py) - ey * (cf[0] - px);
    const double b1 = ex * (cf[11] - py) - ey * (cf[10] - px);
    const double b2 = ex * (cf[13] - py) - ey * (cf[12] - px);
    const double b3 = ex * (cf[9] - py) - ey * (cf[8] - px);
    if ((b0 > 0.0 && b1 > 0.0 && b2 > 0.0 && b3 > 0.0) ||
        (b0 < 0.0 && b1 < 0.0 && b2 < 0.0 && b3 < 0.0))
        return 0;
    double F[4];
    F[0] = ex * (cf[1] - py) - ey * (cf[0] - px);
    F[1] = ex * cf[3] - ey * cf[2];
    F[2] = ex * cf[5] - ey * cf[4];
    F[3] = ex * cf[7] - ey * cf[6];
    const double f1 = ex * (cf[9] - py) - ey * (cf[8] - px);
    double br[4];
    int nb = 0;
    br[nb++] = 0.0;
    const double A = 3.0 * F[3], Bq = 2.0 * F[2], Cq = F[1];
    double r1 = -1.0, r2 = -1.0;
    if (A == 0.0) {
        if (Bq != 0.0) r1 = -Cq / Bq;
    } else {
        const double disc = Bq * Bq - 4.0 * A * Cq;
        if (disc > 0.0) {
            const double sq = sqrt(disc);
            const double qq = Bq >= 0.0 ? -0.5 * (Bq + sq) : -0.5 * (Bq - sq);
            r1 = qq / A;
            r2 = qq != 0.0 ? Cq / qq : -1.0;
            if (r2 < r1) { const double tt = r1; r1 = r2; r2 = tt; }
        }
    }
    if (r1 > 0.0 && r1 < 1.0) br[nb++] = r1;
    if (r2 > 0.0 && r2 < 1.0 && r2 != r1) br[nb++] = r2;
    br[nb] = 1.0;
    int n = 0;
    const double ee = (double)(ex * ex + ey * ey);
    for (int j = 0; j < nb; j++) {
        double lo = br[j], hi = br[j + 1];
        const double flo = spl_cubic(F, lo), fhi = (j == nb - 1) ? f1 : spl_cubic(F, hi);
        const bool slo = flo >= 0.0, shi = fhi >= 0.0;
        if (slo == shi) continue;
        for (int it = 0; it < 64; it++) {
            const double mid = 0.5 * (lo + hi);
            if ((spl_cubic(F, mid) >= 0.0) == slo) lo = mid; else hi = mid;
        }
        const double t = 0.5 * (lo + hi);
        const double sx = ((cf[6] * t + cf[4]) * t + cf[2]) * t + cf[0];
        const double sy = ((cf[7] * t + cf[5]) * t + cf[3]) * t + cf[1];
        const double q = ((sx - px) * ex + (sy - py) * ey) / ee;
        if (!(q >= 0.0 && q < 1.0)) continue;
        ts[n] = t;
        qs[n] = q;
        sg[n] = slo ? -1 : 1;
        n++;
    }
    return n;
}

__device__ __forceinline__ double spl_jump(const double* cf, const double* gk, double dX, double t)
{
    const double Gx = (1.0 - t) * gk[0] + t * gk[2], Gy = (1.0 - t) * gk[1] + t * gk[3];
    const double Tx = (3.0 * cf[6] * t + 2.0 * cf[4]) * t + cf[2];
    const double Ty = (3.0 * cf[7] * t + 2.0 * cf[5]) * t + cf[3];
    return dX * (Gx * Ty - Gy * Tx) / (Tx * Tx + Ty * Ty);
}

template <bool REC>
struct TileSharedSpl {
    int raw[kTileCap];
    int start[kTileCap];
    int key[kTileCap];
    double cf[kTileCap][14];     // segment coefficients, X_{k+1}, inner control points
    double gk[kTileCap][4];      // G_k, G_{k+1}
    short box[kTileCap][4];
    float wx[kTileCap][4], wy[kTileCap][4];
    int2 f0[kTileCap];
    double gtx[kTileCap], gty[kTileCap];
    long long acc[8][kTileNodes];
    unsigned rec[REC ? kTileRec : 1];   // (node, direction, chord, root)
    int cnt, total, nrec, base;
};

template <bool REC>
__device__ void tiles_spline_body(const InstDev& I, const DevPtrs& P, int parity, int blk, int nblk)
{
    __shared__ TileSharedSpl<REC> S;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int N = I.n_markers;
    const double2* X = P.X[parity] + I.mk_off;
    const int nact = min(P.act_count[2 * I.inst + parity], I.act_cap);
    for (int a = blk; a < nact; a += nblk) {
        const int t = P.act_list[parity][I.act_off + a].y;
        const int gt = I.tile_off + t;
        const int tx = t % I.tiles_x, ty = t / I.tiles_x;
        const int x0 = tx * kTile, y0 = ty * kTile;
        if (tid < kTileCap) S.raw[tid] = P.tile_list[I.list_off + (long long)t * kTileCap + tid];
        if (tid == 0) {
            S.cnt = min(P.tile_count[gt], kTileCap);
            S.nrec = 0;
        }
#pragma unroll
        for (int i = 0; i < 8; i++) S.acc[i][tid] = 0;
        __syncthreads();
        const int c = S.cnt;
        if (tid == 0) {
            P.tile_count[gt] = 0;
            P.tile_slot[parity][gt] = I.act_off + a;
        }
        if (tid < c) {
            const int k = S.raw[tid];
            int r = 0;
            for (int m = 0; m < c; m++) r += (S.raw[m] < k) ? 1 : 0;
            const int kp = (k + 1) % N, mk = I.mk_off + k, mp = I.mk_off + kp;
            const double2 Xk = X[k], Xp = X[kp], Mk = P.M[mk], Mp = P.M[mp];
            const double2 Gk = P.G[mk], Gp = P.G[mp];
            double* cf = S.cf[r];
            cf[0] = Xk.x;
            cf[1] = Xk.y;
            cf[2] = Xp.x - Xk.x - (2.0 * Mk.x + Mp.x) / 6.0;
            cf[3] = Xp.y - Xk.y - (2.0 * Mk.y + Mp.y) / 6.0;
            cf[4] = 0.5 * Mk.x;
            cf[5] = 0.5 * Mk.y;
            cf[6] = (Mp.x - Mk.x) / 6.0;
            cf[7] = (Mp.y - Mk.y) / 6.0;
            cf[8] = Xp.x;
            cf[9] = Xp.y;
            cf[10] = cf[0] + cf[2] / 3.0;
            cf[11] = cf[1] + cf[3] / 3.0;
            cf[12] = cf[0] + (2.0 * cf[2] + cf[4]) / 3.0;
            cf[13] = cf[1] + (2.0 * cf[3] + cf[5]) / 3.0;
            S.gk[r][0] = Gk.x; S.gk[r][1] = Gk.y; S.gk[r][2] = Gp.x; S.gk[r][3] = Gp.y;
            S.key[r] = k;
            // candidate source nodes: within one spacing of the control-point hull
            const double t1x = cf[2] + 2.0 * cf[4] + 3.0 * cf[6], t1y = cf[3] + 2.0 * cf[5] + 3.0 * cf[7];
            const double hx1 = cf[0] + cf[2] / 3.0, hy1 = cf[1] + cf[3] / 3.0;
            const double hx2 = Xp.x - t1x / 3.0, hy2 = Xp.y - t1y / 3.0;
            const double xmn = fmin(fmin(Xk.x, Xp.x), fmin(hx1, hx2));
            const double xmx = fmax(fmax(Xk.x, Xp.x), fmax(hx1, hx2));
            const double ymn = fmin(fmin(Xk.y, Xp.y), fmin(hy1, hy2));
            const double ymx = fmax(fmax(Xk.y, Xp.y), fmax(hy1, hy2));
            const int bx0 = max((int)floor(xmn) - 1, x0);
            const int bx1 = min((int)ceil(xmx) + 1, min(x0 + kTile, I.nx) - 1);
            const int by0 = max((int)floor(ymn) - 1, y0);
            const int by1 = min((int)ceil(ymx) + 1, min(y0 + kTile, I.ny) - 1);
            S.box[r][0] = (short)bx0; S.box[r][1] = (short)bx1;
            S.box[r][2] = (short)by0; S.box[r][3] = (short)by1;
            S.start[r] = (bx0 <= bx1 && by0 <= by1) ? (bx1 - bx0 + 1) * (by1 - by0 + 1) : 0;
            S.f0[r] = P.f0[mk];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                S.wx[r][q] = (float)P.wx[4 * mk + q];
                S.wy[r][q] = (float)P.wy[4 * mk + q];
            }
            const double2 gtk = P.Gt[mk];
            S.gtx[r] = gtk.x;
            S.gty[r] = gtk.y;
        }
        __syncthreads();
        if (wid == 0) {
            const int v0 = 2 * lane < c ? S.start[2 * lane] : 0;
            const int v1 = 2 * lane + 1 < c ? S.start[2 * lane + 1] : 0;
            int sc = v0 + v1;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int u = __shfl_up(sc, off);
                if (lane >= off) sc += u;
            }
            if (2 * lane < c) S.start[2 * lane] = sc - v0 - v1;
            if (2 * lane + 1 < c) S.start[2 * lane + 1] = sc - v1;
            if (lane == 63) S.total = sc;
        }
        __syncthreads();
        const int total = S.total;
        for (int g = tid; g < total; g += blockDim.x) {
            int lo = 0, hi = c - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (S.start[mid] <= g) lo = mid; else hi = mid - 1;
            }
            const int j = lo, q = g - S.start[j];
            const int bx0 = S.box[j][0], by0 = S.box[j][2];
            const int w = S.box[j][1] - bx0 + 1;
            const int x = bx0 + q % w, y = by0 + q / w;
            const int node = (y - y0) * kTile + (x - x0);
            for (int i = 1; i < 9; i++) {
                double ts[3], qs[3];
                int sg[3];
                const int nr = spl_crossings(S.cf[j], (double)x, (double)y, EX[i], EY[i], ts, qs, sg);
                for (int rr = 0; rr < nr; rr++) {
                    add_jump(S, node, i, sg[rr], spl_jump(S.cf[j], S.gk[j], I.dX, ts[rr]), P.err + I.inst);
                    if constexpr (REC) {
                        const int e = atomicAdd(&S.nrec, 1);
                        if (e < kTileRec)
                            S.rec[e] = (unsigned)node | ((unsigned)(i - 1) << 8) | ((unsigned)j << 11) |
                                       ((unsigned)rr << 18);
                    }
                }
            }
        }
        const int lx = tid & (kTile - 1), ly = tid / kTile;
        const int x = x0 + lx, y = y0 + ly;
        const bool valid = x < I.nx && y < I.ny;
        double gx = 0.0, gy = 0.0;
        if (valid) {
#pragma unroll 4
            for (int j = 0; j < c; j++) {
                const int2 f = S.f0[j];
                const int ix = x - f.x, iy = y - f.y;
                const bool in = (unsigned)ix <= 3u && (unsigned)iy <= 3u;
                const double wgt = in ? (double)S.wx[j][ix & 3] * (double)S.wy[j][iy & 3] : 0.0;
                gx += S.gtx[j] * wgt * I.dX;
                gy += S.gty[j] * wgt * I.dX;
            }
        }
        __syncthreads();
        {
            // every node written (the mask marks all of them)
            float* cr = P.corr[parity] + (long long)(I.act_off + a) * kCorrPlanes * kTileNodes + tid;
            if (lane == 0) P.cmask[parity][(long long)(I.act_off + a) * 4 + wid] = ~0ull;
            const double fs = I.guo ? 0.0 : 3.0;
#pragma unroll
            for (int i = 1; i < 9; i++) {
                const double delta =
                    valid ? fs * WD[i] * ((double)EX[i] * gx + (double)EY[i] * gy) +
                                jump_sum(S.acc[i - 1][tid])
                          : 0.0;
                cr[(i - 1) * kTileNodes] = (float)delta;
            }
            if (I.guo) {
                cr[8 * kTileNodes] = valid ? (float)gx : 0.f;
                cr[9 * kTileNodes] = valid ? (float)gy : 0.f;
            }
        }
        if constexpr (REC) {
            const int nr = min(S.nrec, kTileRec);
            if (tid == 0) {
                S.base = nr > 0 ? atomicAdd(&P.rec_count[2 * I.inst + parity], nr) : 0;
                if (S.nrec > kTileRec) atomicOr(&P.err[I.inst], (int)kErrRecords);
            }
            __syncthreads();
            const int base = S.base;
            for (int e = tid; e < nr; e += blockDim.x) {
                if (base + e >= I.rec_cap) {
                    atomicOr(&P.err[I.inst], (int)kErrRecords);
                    continue;
                }
                const unsigned pk = S.rec[e];
                const int node = pk & 255, i = 1 + ((pk >> 8) & 7), j = (pk >> 11) & 127,
                          rr = (pk >> 18) & 3;
                const int x = x0 + (node & (kTile - 1)), y = y0 + node / kTile;
                double ts[3], qs[3];
                int sg[3];
                (void)spl_crossings(S.cf[j], (double)x, (double)y, EX[i], EY[i], ts, qs, sg);
                ii_lbm_link L;
                L.x = x; L.y = y; L.dir = i; L.inst = I.inst;
                L.sigma = sg[rr]; L.seg = S.key[j]; L.q = qs[rr]; L.theta = ts[rr];
                L.jp = spl_jump(S.cf[j], S.gk[j], I.dX, ts[rr]);
                P.rec[I.rec_off + base + e] = L;
            }
        }
        __syncthreads();
    }
}

template <bool REC>
__global__ __launch_bounds__(256) void k_tiles_spline(InstDev I, DevPtrs P, int parity)
{
    tiles_spline_body<REC>(I, P, parity, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// IB-LBM tile pass: no cut links, so a tile only gathers the force of the
// markers binned to it, G spread with the delta weights of the marker pass
// (Sec. 2.2.2), summed in increasing marker order.  The comparison method
// places markers 1/3 lu apart, so a tile lists up to kTileCapIB of them.
// ---------------------------------------------------------------------------
struct TileSharedIB {
    int raw[kTileCapIB];         // marker ids as binned
    int2 f0[kTileCapIB];         // in increasing id order: first stencil node,
    float wx[kTileCapIB][4], wy[kTileCapIB][4];   // delta weights,
    double gx[kTileCapIB], gy[kTileCapIB];        // and force
    int cnt;
};

__device__ __forceinline__ void tiles_ib_body(const InstDev& I, const DevPtrs& P, int parity,
                                              int blk, int nblk)
{
    __shared__ TileSharedIB S;
    const int tid = threadIdx.x;
    const int nact = min(P.act_count[2 * I.inst + parity], I.act_cap);
    for (int a = blk; a < nact; a += nblk) {
        const int t = P.act_list[parity][I.act_off + a].y;
        const int gt = I.tile_off + t;
        const int tx = t % I.tiles_x, ty = t / I.tiles_x;
        const int* list = P.tile_list + I.list_off + (long long)t * I.tile_cap;
        if (tid == 0) S.cnt = min(P.tile_count[gt], min(I.tile_cap, kTileCapIB));
        __syncthreads();
        const int c = S.cnt;
        for (int q = tid; q < c; q += blockDim.x) S.raw[q] = list[q];
        __syncthreads();
        if (tid == 0) {
            P.tile_count[gt] = 0;  // ready for the next step
            P.tile_slot[parity][gt] = I.act_off + a;
        }
        for (int q = tid; q < c; q += blockDim.x) {
            const int k = S.raw[q];
            int r = 0;
            for (int m = 0; m < c; m++) r += (S.raw[m] < k) ? 1 : 0;
            const int mk = I.mk_off + k;
            S.f0[r] = P.f0[mk];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                S.wx[r][j] = (float)P.wx[4 * mk + j];
                S.wy[r][j] = (float)P.wy[4 * mk + j];
            }
            const double2 G = P.G[mk];
            S.gx[r] = G.x;
            S.gy[r] = G.y;
        }
        __syncthreads();
        const int x = tx * kTile + (tid & (kTile - 1)), y = ty * kTile + tid / kTile;
        const bool valid = x < I.nx && y < I.ny;
        double gx = 0.0, gy = 0.0;
        if (valid) {
            // g(x) = sum_k G_k delta_h(x - X_k) dX (Sec. 2.2.2)
            for (int j = 0; j < c; j++) {
                const int2 f = S.f0[j];
                const int ix = x - f.x, iy = y - f.y;
                const bool in = (unsigned)ix <= 3u && (unsigned)iy <= 3u;
                const double wgt = in ? (double)S.wx[j][ix & 3] * (double)S.wy[j][iy & 3] : 0.0;
                gx += S.gx[j] * wgt * I.dX;
                gy += S.gy[j] * wgt * I.dX;
            }
        }
        // the simple force term of g for the sweep (none under Guo's term,
        // whose sweep reads g itself), and g for the marker velocity; every
        // node written (the mask marks all of them)
        float* cr = P.corr[parity] + (long long)(I.act_off + a) * kCorrPlanes * kTileNodes + tid;
        if ((tid & 63) == 0) P.cmask[parity][(long long)(I.act_off + a) * 4 + (tid >> 6)] = ~0ull;
        const double fs = I.guo ? 0.0 : 3.0;
#pragma unroll
        for (int i = 1; i < 9; i++)
            cr[(i - 1) * kTileNodes] =
                valid ? (float)(fs * WD[i] * ((double)EX[i] * gx + (double)EY[i] * gy)) : 0.f;
        cr[8 * kTileNodes] = valid ? (float)gx : 0.f;
        cr[9 * kTileNodes] = valid ? (float)gy : 0.f;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_tiles_ib(InstDev I, DevPtrs P, int parity)
{
    tiles_ib_body(I, P, parity, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_tiles_ib_batch(const InstDev* __restrict__ insts,
                                                        const int2* __restrict__ units, DevPtrs P,
                                                        int parity)
{
    const int2 u = units[blockIdx.x];
    const InstDev I = insts[u.x];
    tiles_ib_body(I, P, parity, u.y, I.tile_blocks);
}

// Membrane tile blocks (without records) are held to 80 registers (six waves
// per SIMD), so that beside the tile pass the sweep keeps wave slots and
// registers on every CU: 4 tile blocks per CU at 96 registers left it three
// waves per SIMD, at 80 four.
constexpr int tile_waves(int iface, bool rec)
{
    return iface == II_LBM_IF_MEMBRANE && !rec ? 6 : 1;
}

template <int IFACE, bool REC>
__global__ __launch_bounds__(256, tile_waves(IFACE, REC)) void k_tiles(InstDev I, DevPtrs P,
                                                                       int parity)
{
    tiles_body<IFACE, REC>(I, P, parity, blockIdx.x, gridDim.x);
}

template <int IFACE, bool REC>
__global__ __launch_bounds__(256, tile_waves(IFACE, REC)) void k_tiles_batch(
    const InstDev* __restrict__ insts, const int2* __restrict__ units, DevPtrs P, int parity)
{
    const int2 u = units[blockIdx.x];
    const InstDev I = insts[u.x];
    tiles_body<IFACE, REC>(I, P, parity, u.y, I.tile_blocks);
}

template <int IFACE>
static hipError_t tiles_i(const InstDev& I, const DevPtrs& P, int parity, bool records,
                          hipStream_t s)
{
    const int nb = I.tile_blocks;
    if (records)
        hipLaunchKernelGGL((k_tiles<IFACE, true>), dim3(nb), dim3(256), 0, s, I, P, parity);
    else
        hipLaunchKernelGGL((k_tiles<IFACE, false>), dim3(nb), dim3(256), 0, s, I, P, parity);
    return hipGetLastError();
}

hipError_t launch_tiles(const InstDev& I, const DevPtrs& P, int parity, bool records, hipStream_t s)
{
    if (I.jumps && I.iface == II_LBM_IF_MEMBRANE && I.geometry == 1) {
        if (records)
            hipLaunchKernelGGL(k_tiles_spline<true>, dim3(I.tile_blocks), dim3(256), 0, s, I, P, parity);
        else
            hipLaunchKernelGGL(k_tiles_spline<false>, dim3(I.tile_blocks), dim3(256), 0, s, I, P, parity);
        return hipGetLastError();
    }
    if (!I.jumps) {
        hipLaunchKernelGGL(k_tiles_ib, dim3(I.tile_blocks), dim3(256), 0, s, I, P, parity);
        return hipGetLastError();
    }
    return I.iface == II_LBM_IF_MEMBRANE ? tiles_i<II_LBM_IF_MEMBRANE>(I, P, parity, records, s)
                                         : tiles_i<II_LBM_IF_RIGID>(I, P, parity, records, s);
}

template <int IFACE>
static hipError_t tiles_batch_i(const Batch& b, const DevPtrs& P, int parity, bool records,
                                hipStream_t s)
{
    const dim3 g(b.tile_units);
    if (records)
        hipLaunchKernelGGL((k_tiles_batch<IFACE, true>), g, dim3(256), 0, s, b.insts,
                           b.tile_table, P, parity);
    else
        hipLaunchKernelGGL((k_tiles_batch<IFACE, false>), g, dim3(256), 0, s, b.insts,
                           b.tile_table, P, parity);
    return hipGetLastError();
}

hipError_t launch_tiles_batch(const Batch& b, const DevPtrs& P, int parity, bool records,
                              hipStream_t s)
{
    if (b.tile_units == 0) return hipSuccess;
    if (!b.jumps) {
        hipLaunchKernelGGL(k_tiles_ib_batch, dim3(b.tile_units), dim3(256), 0, s, b.insts,
                           b.tile_table, P, parity);
        return hipGetLastError();
    }
    return b.iface == II_LBM_IF_MEMBRANE
               ? tiles_batch_i<II_LBM_IF_MEMBRANE>(b, P, parity, records, s)
               : tiles_batch_i<II_LBM_IF_RIGID>(b, P, parity, records, s);
}

// ---------------------------------------------------------------------------
// Moving rigid circle: the body update that ends step m (Sec. 2.3).
//   F^ext = -sum_k G_k dX + rho_f V_s (U_c^m - U_c^{m-1}),
//   T^ext = -sum_k (X_k - X_c) x G_k dX + (rho_f / rho_s) I_s (W^m - W^{m-1}),
// rho_f = 1, V_s = pi R^2, m = rho* V_s, I_s = m R^2 / 2; on a free axis
// m a^{m+1} = F (+ spring and damper), U^{m+1} = U^m + a^{m+1},
// X_c^{m+1} = X_c^m + U^m + (a^m + a^{m+1}) / 2, and the same for the angle; a
// prescribed axis takes U_c and X_c of step m+1 from its harmonic motion.
// The sums run in marker order on one lane; then every lane places the
// markers of step m+1 rigidly at X_c + R (cos, sin)(theta + 2 pi k / N).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_body(InstDev I, DevPtrs P, int par)
{
    BodyDev& b = P.body[I.inst];
    const int N = I.n_markers;
    const double2* X = P.X[par] + I.mk_off;
    if (threadIdx.x == 0) {
        double Fx = 0.0, Fy = 0.0, T = 0.0;
        for (int k = 0; k < N; k++) {
            const double2 G = P.G[I.mk_off + k];
            const double rx = X[k].x - b.c[0], ry = X[k].y - b.c[1];
            Fx -= G.x * I.dX;
            Fy -= G.y * I.dX;
            T -= (rx * G.y - ry * G.x) * I.dX;
        }
        const double R = I.radius, Vs = M_PI * R * R;
        const double m = I.rho_star * Vs, Is = 0.5 * m * R * R;
        Fx += Vs * (b.U[0] - b.Uprev[0]);
        Fy += Vs * (b.U[1] - b.Uprev[1]);
        T += Is / I.rho_star * (b.W - b.Wprev);
        b.F[0] = Fx;
        b.F[1] = Fy;
        b.T = T;
        const double Fa[2] = {Fx, Fy};
        double Unew[2] = {b.U[0], b.U[1]};
        const double tn = (double)(b.n + 1);
        for (int ax = 0; ax < 2; ax++) {
            b.Uprev[ax] = b.U[ax];
            if (I.presc_umax[ax] != 0.0) {
                const double A = I.presc_amp[ax], Um = I.presc_umax[ax];
                Unew[ax] = -Um * cos(Um * tn / A);
                b.c[ax] = b.c0[ax] - A * sin(Um * tn / A);
                continue;
            }
            if (!(I.body_free & (1 << ax))) continue;
            const double Fe = Fa[ax] - I.spring[ax] * (b.c[ax] - b.c0[ax]) - I.damping[ax] * b.U[ax];
            const double an = Fe / m;
            Unew[ax] = b.U[ax] + an;
            b.c[ax] = b.c[ax] + b.U[ax] + 0.5 * (b.a[ax] + an);
            b.a[ax] = an;
        }
        b.U[0] = Unew[0];
        b.U[1] = Unew[1];
        b.Wprev = b.W;
        if (I.body_free & 4) {
            const double wn = T / Is;
            const double Wn = b.W + wn;
            b.theta = b.theta + b.W + 0.5 * (b.wdot + wn);
            b.wdot = wn;
            b.W = Wn;
        }
        b.theta_mod = b.theta - 2.0 * M_PI * floor(b.theta / (2.0 * M_PI));
        b.n += 1;
    }
    __syncthreads();
    double2* Xn = P.X[par ^ 1] + I.mk_off;
    const double cx = b.c[0], cy = b.c[1], th = b.theta;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const double ang = th + 2.0 * M_PI * k / N;
        Xn[k] = make_double2(cx + I.radius * cos(ang), cy + I.radius * sin(ang));
    }
}

hipError_t launch_body(const InstDev& I, const DevPtrs& P, int par, hipStream_t s)
{
    hipLaunchKernelGGL(k_body, dim3(1), dim3(256), 0, s, I, P, par);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pressure on either side of the interface: the mean of p = rho c_s^2 over the
// nodes farther than `margin` lu from the marker polygon, inside and outside
// (the pressure jump of Sec. 3.1, whose equilibrium value across a tensioned
// circle is Laplace's T / R).  One block per row (grid stride): the block
// walks the chords in batches of 256; a node's inside parity counts the
// chords that cross its row to the right of it (half-open in y), and a node
// is left out when some chord lies within `margin` of it.  Nodes that far
// from the curve are classified the same by every correct even-odd rule.
// Per block: (sum p inside, count inside, sum p outside, count outside).
// ---------------------------------------------------------------------------
constexpr int kPjRow = 8192 / 256;   // nodes per thread of a row (nx <= 8192)

template <typename T, typename M>
__global__ __launch_bounds__(256) void k_pjump(InstDev I, const T* __restrict__ A,
                                               const double2* __restrict__ X, double margin,
                                               double* __restrict__ part)
{
    __shared__ double xc[256];
    __shared__ int near[256];
    __shared__ int ncross, nnear;
    __shared__ double sh[4][256];
    const int t = threadIdx.x, N = I.n_markers;
    double s_in = 0.0, c_in = 0.0, s_out = 0.0, c_out = 0.0;
    for (int y = blockIdx.x; y < I.ny; y += gridDim.x) {
        unsigned par_bits = 0u, near_bits = 0u;
        const double yd = (double)y;
        for (int base = 0; base < N; base += 256) {
            if (t == 0) { ncross = 0; nnear = 0; }
            __syncthreads();
            const int k = base + t;
            if (k < N) {
                const double2 a = X[k], b = X[k + 1 < N ? k + 1 : 0];
                if ((a.y > yd) != (b.y > yd))
                    xc[atomicAdd(&ncross, 1)] = a.x + (yd - a.y) * (b.x - a.x) / (b.y - a.y);
                if (fmin(a.y, b.y) - margin < yd && yd < fmax(a.y, b.y) + margin)
                    near[atomicAdd(&nnear, 1)] = k;
            }
            __syncthreads();
            const int nc = ncross, nn = nnear;
            for (int j = 0; j < kPjRow; j++) {
                const int x = t + 256 * j;
                if (x >= I.nx) break;
                const double xd = (double)x;
                for (int c = 0; c < nc; c++)
                    if (xc[c] > xd) par_bits ^= 1u << j;
                if (near_bits & (1u << j)) continue;
                for (int c = 0; c < nn; c++) {
                    const int q = near[c];
                    const double2 a = X[q], b = X[q + 1 < N ? q + 1 : 0];
                    if (xd <= fmin(a.x, b.x) - margin || xd >= fmax(a.x, b.x) + margin) continue;
                    const double vx = b.x - a.x, vy = b.y - a.y, wx = xd - a.x, wy = yd - a.y;
                    double u = (vx * wx + vy * wy) / (vx * vx + vy * vy);
                    if (u < 0.0) u = 0.0;
                    if (u > 1.0) u = 1.0;
                    const double dx = xd - (a.x + u * vx), dy = yd - (a.y + u * vy);
                    if (sqrt(dx * dx + dy * dy) < margin) {
                        near_bits |= 1u << j;
                        break;
                    }
                }
            }
            __syncthreads();
        }
        for (int j = 0; j < kPjRow; j++) {
            const int x = t + 256 * j;
            if (x >= I.nx) break;
            if (near_bits & (1u << j)) continue;
            M d[9];
            gather<T, M>(I, A, x, y, d);
            double r = 0.0;
#pragma unroll
            for (int i = 0; i < 9; i++) r += (double)d[i];
            const double pr = (1.0 + r) * kCs2;
            if (par_bits & (1u << j)) { s_in += pr; c_in += 1.0; }
            else { s_out += pr; c_out += 1.0; }
        }
    }
    sh[0][t] = s_in; sh[1][t] = c_in; sh[2][t] = s_out; sh[3][t] = c_out;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int c = 0; c < 4; c++) sh[c][t] += sh[c][t + w];
        __syncthreads();
    }
    if (t == 0)
        for (int c = 0; c < 4; c++) part[4 * blockIdx.x + c] = sh[c][0];
}

template <typename T, typename M>
static hipError_t pjump_t(const InstDev& I, const void* A, const double2* X, double margin,
                          double* part, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_pjump<T, M>), dim3(nblocks), dim3(256), 0, s, I, (const T*)A, X, margin,
                       part);
    return hipGetLastError();
}

hipError_t launch_pjump(const InstDev& I, const void* A, const double2* X, double margin,
                        double* part, int nblocks, hipStream_t s)
{
    if (I.n_markers < 3 || I.nx > kPjRow * 256) return hipErrorInvalidValue;
    if (I.storage == II_LBM_FP16)
        return I.math == II_LBM_MATH_FP64 ? pjump_t<_Float16, double>(I, A, X, margin, part, nblocks, s)
                                          : pjump_t<_Float16, float>(I, A, X, margin, part, nblocks, s);
    return I.math == II_LBM_MATH_FP64 ? pjump_t<float, double>(I, A, X, margin, part, nblocks, s)
                                      : pjump_t<float, float>(I, A, X, margin, part, nblocks, s);
}

}  // namespace iilbm
