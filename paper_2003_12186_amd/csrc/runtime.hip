// Host runtime of the II-LBM library: problem validation, workspace layout,
// the per-step launch sequence, readout, checkpoint/restart and the C ABI
// declared in include/ii_lbm.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "common.hpp"

using namespace iilbm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDiagBlocks = 1024;
constexpr int kEventPool = 16384;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    std::vector<InstDev> inst;
    size_t lat_bytes = 0;  // one lattice buffer (all instances)
    size_t off_lat[2] = {0, 0};
    size_t off_X[2] = {0, 0}, off_U = 0, off_G = 0, off_Gt = 0, off_jp = 0, off_wx = 0, off_wy = 0, off_f0 = 0;
    size_t off_tile_count = 0, off_tile_list = 0, off_tile_slot = 0, off_corr = 0;
    size_t off_act_list[2] = {0, 0}, off_act_count = 0;
    size_t off_rec = 0, off_rec_count = 0, off_err = 0, off_diag = 0;
    size_t total = 0;
    int n_markers_total = 0, tiles_total = 0, act_total = 0, rec_total = 0;
};

int validate(const ii_lbm_problem& p, const double* X0)
{
    if (p.nx < 8 || p.ny < 8 || p.nx > 8192 || p.ny > 8192) return II_LBM_EINVAL;
    if (!(p.tau > 0.5) || !isfinite(p.tau)) return II_LBM_EINVAL;
    if (p.collision != II_LBM_SRT && p.collision != II_LBM_MRT) return II_LBM_EINVAL;
    for (int i = 0; i < 4; i++)
        if (p.bc[i] < II_LBM_BC_PERIODIC || p.bc[i] > II_LBM_BC_OUTLET) return II_LBM_EINVAL;
    if ((p.bc[0] == II_LBM_BC_PERIODIC) != (p.bc[1] == II_LBM_BC_PERIODIC)) return II_LBM_EINVAL;
    if ((p.bc[2] == II_LBM_BC_PERIODIC) != (p.bc[3] == II_LBM_BC_PERIODIC)) return II_LBM_EINVAL;
    if (p.bc[1] == II_LBM_BC_INLET || p.bc[2] == II_LBM_BC_INLET || p.bc[3] == II_LBM_BC_INLET)
        return II_LBM_EINVAL;
    if (p.bc[0] == II_LBM_BC_OUTLET || p.bc[2] == II_LBM_BC_OUTLET || p.bc[3] == II_LBM_BC_OUTLET)
        return II_LBM_EINVAL;
    if (p.storage != II_LBM_FP32 && p.storage != II_LBM_FP16) return II_LBM_EINVAL;
    if (p.math != II_LBM_MATH_FP32 && p.math != II_LBM_MATH_FP64) return II_LBM_EINVAL;
    if (p.force_mode != II_LBM_FORCE_II) return II_LBM_EINVAL;
    if (p.interface_kind == II_LBM_IF_NONE) return II_LBM_OK;
    if (p.interface_kind != II_LBM_IF_MEMBRANE && p.interface_kind != II_LBM_IF_RIGID)
        return II_LBM_EINVAL;
    if (p.n_markers < 3 || p.n_markers > (1 << 20)) return II_LBM_EINVAL;
    if (!(p.dX > 0.0) || p.dX > 2.0 || !(p.kappa >= 0.0)) return II_LBM_EINVAL;
    if (p.interface_kind == II_LBM_IF_RIGID && !(p.radius > 0.0)) return II_LBM_EINVAL;
    if (!X0) return II_LBM_EINVAL;
    double area = 0.0;
    const int N = p.n_markers;
    for (int k = 0; k < N; k++) {
        const double x = X0[2 * k], y = X0[2 * k + 1];
        if (!isfinite(x) || !isfinite(y)) return II_LBM_EINVAL;
        if (x < 3.0 || x > p.nx - 4 || y < 3.0 || y > p.ny - 4) return II_LBM_EGEOMETRY;
        const int kp = (k + 1) % N;
        area += X0[2 * k] * X0[2 * kp + 1] - X0[2 * kp] * X0[2 * k + 1];
        const double l = hypot(X0[2 * kp] - x, X0[2 * kp + 1] - y);
        if (l > 2.0 || l == 0.0) return II_LBM_EGEOMETRY;
    }
    if (!(area > 0.0)) return II_LBM_EGEOMETRY;  // must be counter-clockwise
    return II_LBM_OK;
}

int storage_bytes(int storage) { return storage == II_LBM_FP16 ? 2 : 4; }

// FP16 storage scale: 2^e with the largest expected deviation (three times
// the initial [[p]] or the inlet speed) near 2^12 of the half range.
int auto_fp16_exp(const ii_lbm_problem& p, const double* X0)
{
    double est = 3.0 * fabs(p.u_max);
    const int N = p.n_markers;
    if (p.interface_kind == II_LBM_IF_MEMBRANE && X0) {
        for (int k = 0; k < N; k++) {
            const int km = (k + N - 1) % N, kp = (k + 1) % N;
            const double gx = p.kappa * (X0[2 * kp] - 2.0 * X0[2 * k] + X0[2 * km]) / (p.dX * p.dX);
            const double gy =
                p.kappa * (X0[2 * kp + 1] - 2.0 * X0[2 * k + 1] + X0[2 * km + 1]) / (p.dX * p.dX);
            est = std::max(est, 3.0 * hypot(gx, gy));
        }
    }
    est = std::max(est, 1e-7);
    return (int)floor(log2(est)) - 12;
}

int build_layout(const ii_lbm_problem* p, int n_inst, Layout& L)
{
    L.inst.resize(n_inst);
    size_t lat = 0;
    int mk = 0, tiles = 0, act = 0, rec = 0;
    for (int j = 0; j < n_inst; j++) {
        const ii_lbm_problem& q = p[j];
        InstDev I;
        memset(&I, 0, sizeof I);
        I.nx = q.nx;
        I.ny = q.ny;
        I.pitch = (q.nx + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
        I.px = q.bc[0] == II_LBM_BC_PERIODIC;
        I.py = q.bc[2] == II_LBM_BC_PERIODIC;
        I.bounded = !(I.px && I.py);
        for (int s = 0; s < 4; s++) {
            I.bc[s] = q.bc[s];
            I.u_wall[s] = (float)q.u_wall[s];
        }
        I.collision = q.collision;
        I.storage = q.storage;
        I.math = q.math;
        I.iface = q.interface_kind;
        I.n_markers = q.interface_kind == II_LBM_IF_NONE ? 0 : q.n_markers;
        I.inst = j;
        I.plane = (long long)I.pitch * q.ny;
        const int eb = storage_bytes(q.storage);
        lat = align_up(lat);
        I.lat_off = (long long)(lat / eb);
        lat += (size_t)9 * I.plane * eb;
        I.omega = (float)(1.0 / q.tau);
        I.omega_d = 1.0 / q.tau;
        bool all_zero = true;
        for (int a = 0; a < 9; a++) all_zero = all_zero && q.mrt_s[a] == 0.0;
        const double defaults[9] = {0.0, 1.63, 1.14, 0.0, 1.92, 0.0, 1.92, 1.0 / q.tau, 1.0 / q.tau};
        for (int a = 0; a < 9; a++) I.s[a] = (float)(all_zero ? defaults[a] : q.mrt_s[a]);
        I.u_max = (float)q.u_max;
        I.body[0] = (float)q.body_force[0];
        I.body[1] = (float)q.body_force[1];
        I.scale = 1.f;
        I.inv_scale = 1.f;
        I.kappa = q.kappa;
        I.dX = q.dX;
        I.cx = q.center[0];
        I.cy = q.center[1];
        I.radius = q.radius;
        I.mk_off = mk;
        mk += I.n_markers;
        I.tiles_x = (q.nx + kTile - 1) / kTile;
        I.tiles_y = (q.ny + kTile - 1) / kTile;
        I.tile_off = tiles;
        tiles += I.tiles_x * I.tiles_y;
        I.act_off = act;
        // tiles within 2.5 lu of a closed curve of N chords; the bound leaves
        // room for chords of up to 2 lu (longer curves report ECAPACITY)
        I.act_cap = std::min(I.tiles_x * I.tiles_y, I.n_markers / 2 + 256);
        act += I.act_cap;
        I.rec_off = rec;
        I.rec_cap = 48 * I.n_markers + 1024;
        rec += I.rec_cap;
        L.inst[j] = I;
    }
    L.lat_bytes = align_up(lat);
    L.n_markers_total = mk;
    L.tiles_total = tiles;
    L.act_total = act;
    L.rec_total = rec;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t nm = std::max(mk, 1);
    L.off_lat[0] = take(L.lat_bytes);
    L.off_lat[1] = take(L.lat_bytes);
    L.off_X[0] = take(nm * sizeof(double2));
    L.off_X[1] = take(nm * sizeof(double2));
    L.off_U = take(nm * sizeof(double2));
    L.off_G = take(nm * sizeof(double2));
    L.off_Gt = take(nm * sizeof(double2));
    L.off_jp = take(nm * sizeof(double));
    L.off_wx = take(4 * nm * sizeof(double));
    L.off_wy = take(4 * nm * sizeof(double));
    L.off_f0 = take(nm * sizeof(int2));
    L.off_tile_count = take((size_t)tiles * sizeof(int));
    L.off_tile_list = take((size_t)tiles * kTileCap * sizeof(int));
    L.off_tile_slot = take((size_t)tiles * sizeof(int));
    L.off_corr = take((size_t)std::max(act, 1) * 8 * kTileNodes * sizeof(float));
    L.off_act_list[0] = take((size_t)std::max(act, 1) * sizeof(int2));
    L.off_act_list[1] = take((size_t)std::max(act, 1) * sizeof(int2));
    L.off_act_count = take((size_t)2 * n_inst * sizeof(int));
    L.off_rec = take((size_t)std::max(rec, 1) * sizeof(ii_lbm_link));
    L.off_rec_count = take((size_t)2 * n_inst * sizeof(int));
    L.off_err = take((size_t)n_inst * sizeof(int));
    L.off_diag = take((size_t)4 * kDiagBlocks * sizeof(double));
    L.total = o;
    return II_LBM_OK;
}

}  // namespace

struct ii_lbm_handle {
    Layout L;
    std::vector<ii_lbm_problem> prob;
    char* ws = nullptr;
    bool owns_ws = false;
    hipStream_t stream = nullptr;
    DevPtrs P;
    int parity = 0;        // which lattice / marker buffer is current
    int64_t steps = 0;
    int failed = 0;        // sticky error code
    int records = 1;
    bool timing = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs
    int ev_used = 0;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
};

static int hip_fail(ii_lbm_handle* h, hipError_t e)
{
    if (e == hipSuccess) return II_LBM_OK;
    if (h) h->failed = II_LBM_EDEVICE;
    return II_LBM_EDEVICE;
}

static int check_device_errors(ii_lbm_handle* h)
{
    const int n = (int)h->prob.size();
    std::vector<int> err(n);
    hipError_t e = hipMemcpyAsync(err.data(), h->P.err, n * sizeof(int), hipMemcpyDeviceToHost,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    int bits = 0;
    for (int v : err) bits |= v;
    if (bits & kErrUnstable) h->failed = II_LBM_EUNSTABLE;
    else if (bits & kErrGeometry) h->failed = II_LBM_EGEOMETRY;
    else if (bits & kErrCapacity) h->failed = II_LBM_ECAPACITY;
    return h->failed;
}

static int sync_and_check(ii_lbm_handle* h)
{
    if (!h) return II_LBM_EINVAL;
    const hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    if (h->failed) return h->failed;
    return check_device_errors(h);
}

extern "C" {

int ii_lbm_workspace_size(const ii_lbm_problem* p, int32_t n_inst, size_t* bytes)
{
    if (!p || n_inst < 1 || !bytes) return II_LBM_EINVAL;
    Layout L;
    build_layout(p, n_inst, L);
    *bytes = L.total;
    return II_LBM_OK;
}

int ii_lbm_init(const ii_lbm_problem* p, int32_t n_inst, const double* const* X0,
                void* d_workspace, size_t ws_bytes, void* hip_stream, ii_lbm_handle** out)
{
    if (!p || n_inst < 1 || !out) return II_LBM_EINVAL;
    *out = nullptr;
    for (int j = 0; j < n_inst; j++) {
        const double* x0 = (X0 && p[j].interface_kind != II_LBM_IF_NONE) ? X0[j] : nullptr;
        const int rc = validate(p[j], x0);
        if (rc) return rc;
    }
    ii_lbm_handle* h = new (std::nothrow) ii_lbm_handle();
    if (!h) return II_LBM_EINVAL;
    h->prob.assign(p, p + n_inst);
    build_layout(p, n_inst, h->L);
    for (int j = 0; j < n_inst; j++) {
        InstDev& I = h->L.inst[j];
        if (p[j].storage == II_LBM_FP16) {
            const double* x0 = (X0 && p[j].interface_kind != II_LBM_IF_NONE) ? X0[j] : nullptr;
            const int e = p[j].fp16_log2_scale != 0 ? p[j].fp16_log2_scale : auto_fp16_exp(p[j], x0);
            I.scale = ldexpf(1.f, e);
            I.inv_scale = ldexpf(1.f, -e);
        }
    }
    h->stream = (hipStream_t)hip_stream;
    if (d_workspace) {
        if (ws_bytes < h->L.total || ((uintptr_t)d_workspace % kAlign) != 0) {
            delete h;
            return II_LBM_EWORKSPACE;
        }
        h->ws = (char*)d_workspace;
    } else {
        if (hipMalloc((void**)&h->ws, h->L.total) != hipSuccess) {
            delete h;
            return II_LBM_EDEVICE;
        }
        h->owns_ws = true;
    }
    const Layout& L = h->L;
    DevPtrs& P = h->P;
    P.lat[0] = h->ws + L.off_lat[0];
    P.lat[1] = h->ws + L.off_lat[1];
    P.X[0] = (double2*)(h->ws + L.off_X[0]);
    P.X[1] = (double2*)(h->ws + L.off_X[1]);
    P.U = (double2*)(h->ws + L.off_U);
    P.G = (double2*)(h->ws + L.off_G);
    P.Gt = (double2*)(h->ws + L.off_Gt);
    P.jp = (double*)(h->ws + L.off_jp);
    P.wx = (double*)(h->ws + L.off_wx);
    P.wy = (double*)(h->ws + L.off_wy);
    P.f0 = (int2*)(h->ws + L.off_f0);
    P.tile_count = (int*)(h->ws + L.off_tile_count);
    P.tile_list = (int*)(h->ws + L.off_tile_list);
    P.tile_slot = (int*)(h->ws + L.off_tile_slot);
    P.corr = (float*)(h->ws + L.off_corr);
    P.act_list[0] = (int2*)(h->ws + L.off_act_list[0]);
    P.act_list[1] = (int2*)(h->ws + L.off_act_list[1]);
    P.act_count = (int*)(h->ws + L.off_act_count);
    P.rec = (ii_lbm_link*)(h->ws + L.off_rec);
    P.rec_count = (int*)(h->ws + L.off_rec_count);
    P.err = (int*)(h->ws + L.off_err);
    P.diag = (double*)(h->ws + L.off_diag);

    hipError_t e = hipSuccess;
    for (int j = 0; j < n_inst && e == hipSuccess; j++) {
        e = launch_fill_zero(L.inst[j], P.lat[0], h->stream);
        if (e == hipSuccess) e = launch_fill_zero(L.inst[j], P.lat[1], h->stream);
    }
    if (e == hipSuccess) e = launch_fill_ints(P.tile_count, L.tiles_total, 0, h->stream);
    if (e == hipSuccess) e = launch_fill_ints(P.tile_slot, L.tiles_total, -1, h->stream);
    if (e == hipSuccess) e = launch_fill_ints(P.act_count, 2 * n_inst, 0, h->stream);
    if (e == hipSuccess) e = launch_fill_ints(P.rec_count, 2 * n_inst, 0, h->stream);
    if (e == hipSuccess) e = launch_fill_ints(P.err, n_inst, 0, h->stream);
    for (int j = 0; j < n_inst && e == hipSuccess; j++) {
        const InstDev& I = L.inst[j];
        if (I.n_markers == 0) continue;
        e = hipMemcpyAsync(P.X[0] + I.mk_off, X0[j], (size_t)I.n_markers * sizeof(double2),
                           hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(P.X[1] + I.mk_off, X0[j], (size_t)I.n_markers * sizeof(double2),
                               hipMemcpyHostToDevice, h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        if (h->owns_ws) hipFree(h->ws);
        delete h;
        return II_LBM_EDEVICE;
    }
    *out = h;
    return II_LBM_OK;
}

int ii_lbm_step(ii_lbm_handle* h, int64_t n_steps)
{
    if (!h || n_steps < 0) return II_LBM_EINVAL;
    if (h->failed) return II_LBM_ESTATE;
    const int n_inst = (int)h->prob.size();
    for (int64_t s = 0; s < n_steps; s++) {
        const int par = h->parity;
        void* A = h->P.lat[par];
        void* B = h->P.lat[par ^ 1];
        for (int j = 0; j < n_inst; j++) {
            const InstDev& I = h->L.inst[j];
            hipError_t e = hipSuccess;
            if (I.n_markers > 0) {
                e = launch_markers(I, h->P, A, par, h->stream);
                if (e == hipSuccess) e = launch_tiles(I, h->P, par, h->records, h->stream);
            }
            if (e != hipSuccess) return hip_fail(h, e);
            const bool timed = h->timing && h->ev_used + 2 <= (int)h->ev.size();
            if (timed) hipEventRecord(h->ev[h->ev_used], h->stream);
            e = launch_sweep(I, h->P, A, B, h->stream);
            if (e != hipSuccess) return hip_fail(h, e);
            if (timed) {
                hipEventRecord(h->ev[h->ev_used + 1], h->stream);
                h->ev_used += 2;
            }
        }
        h->parity ^= 1;
        h->steps++;
    }
    return II_LBM_OK;
}

int ii_lbm_sync(ii_lbm_handle* h) { return sync_and_check(h); }

int ii_lbm_markers(ii_lbm_handle* h, int32_t inst, double* X, double* U, double* G)
{
    if (!h || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    const InstDev& I = h->L.inst[inst];
    const size_t nb = (size_t)I.n_markers * sizeof(double2);
    hipError_t e = hipSuccess;
    if (X && nb) e = hipMemcpyAsync(X, h->P.X[h->parity] + I.mk_off, nb, hipMemcpyDeviceToHost, h->stream);
    if (U && nb && e == hipSuccess)
        e = hipMemcpyAsync(U, h->P.U + I.mk_off, nb, hipMemcpyDeviceToHost, h->stream);
    if (G && nb && e == hipSuccess)
        e = hipMemcpyAsync(G, h->P.G + I.mk_off, nb, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    return sync_and_check(h);
}

int ii_lbm_set_markers(ii_lbm_handle* h, int32_t inst, const double* X)
{
    if (!h || !X || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    if (h->failed) return II_LBM_ESTATE;
    const InstDev& I = h->L.inst[inst];
    const int rc = validate(h->prob[inst], X);
    if (rc) return rc;
    const hipError_t e = hipMemcpyAsync(h->P.X[h->parity] + I.mk_off, X,
                                        (size_t)I.n_markers * sizeof(double2),
                                        hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    return hip_fail(h, hipStreamSynchronize(h->stream));
}

int ii_lbm_fields(ii_lbm_handle* h, int32_t inst, uint32_t what, void* out, int32_t dtype,
                  int32_t on_device)
{
    if (!h || !out || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    if (dtype != II_LBM_DT_F32 && dtype != II_LBM_DT_F64) return II_LBM_EINVAL;
    if (what == 0 || (what & ~31u)) return II_LBM_EINVAL;
    const int rc = sync_and_check(h);
    if (rc) return rc;
    const InstDev& I = h->L.inst[inst];
    int planes = 0;
    for (int b = 0; b < 4; b++) planes += (what >> b) & 1;
    if (what & II_LBM_F_DISTRIB) planes += 9;
    const size_t bytes = (size_t)planes * I.nx * I.ny * (dtype == II_LBM_DT_F64 ? 8 : 4);
    void* dst = out;
    if (!on_device) {
        if (hipMalloc(&dst, bytes) != hipSuccess) return II_LBM_EDEVICE;
    }
    hipError_t e = launch_fields(I, h->P.lat[h->parity], what, dst, dtype, h->stream);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (!on_device) hipFree(dst);
    return hip_fail(h, e);
}

int ii_lbm_set_distrib(ii_lbm_handle* h, int32_t inst, const double* f)
{
    if (!h || !f || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    if (h->failed) return II_LBM_ESTATE;
    const InstDev& I = h->L.inst[inst];
    const size_t bytes = (size_t)9 * I.nx * I.ny * sizeof(double);
    double* d = nullptr;
    if (hipMalloc((void**)&d, bytes) != hipSuccess) return II_LBM_EDEVICE;
    hipError_t e = hipMemcpyAsync(d, f, bytes, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = launch_set_distrib(I, d, h->P.lat[h->parity], h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    hipFree(d);
    return hip_fail(h, e);
}

int ii_lbm_state_size(ii_lbm_handle* h, int32_t inst, size_t* bytes)
{
    if (!h || !bytes || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    const InstDev& I = h->L.inst[inst];
    *bytes = sizeof(int64_t) + (size_t)I.n_markers * sizeof(double2) +
             (size_t)9 * I.plane * storage_bytes(I.storage);
    return II_LBM_OK;
}

int ii_lbm_save_state(ii_lbm_handle* h, int32_t inst, void* host_buf, size_t bytes)
{
    size_t need = 0;
    int rc = ii_lbm_state_size(h, inst, &need);
    if (rc) return rc;
    if (!host_buf || bytes < need) return II_LBM_EINVAL;
    rc = sync_and_check(h);
    if (rc) return rc;
    const InstDev& I = h->L.inst[inst];
    char* b = (char*)host_buf;
    memcpy(b, &h->steps, sizeof(int64_t));
    b += sizeof(int64_t);
    const size_t mb = (size_t)I.n_markers * sizeof(double2);
    hipError_t e = hipSuccess;
    if (mb) e = hipMemcpy(b, h->P.X[h->parity] + I.mk_off, mb, hipMemcpyDeviceToHost);
    b += mb;
    const size_t eb = storage_bytes(I.storage);
    if (e == hipSuccess)
        e = hipMemcpy(b, (char*)h->P.lat[h->parity] + I.lat_off * eb, (size_t)9 * I.plane * eb,
                      hipMemcpyDeviceToHost);
    return hip_fail(h, e);
}

int ii_lbm_load_state(ii_lbm_handle* h, int32_t inst, const void* host_buf, size_t bytes)
{
    size_t need = 0;
    int rc = ii_lbm_state_size(h, inst, &need);
    if (rc) return rc;
    if (!host_buf || bytes < need) return II_LBM_EINVAL;
    if (h->failed) return II_LBM_ESTATE;
    rc = hip_fail(h, hipStreamSynchronize(h->stream));
    if (rc) return rc;
    const InstDev& I = h->L.inst[inst];
    const char* b = (const char*)host_buf;
    memcpy(&h->steps, b, sizeof(int64_t));
    b += sizeof(int64_t);
    const size_t mb = (size_t)I.n_markers * sizeof(double2);
    hipError_t e = hipSuccess;
    if (mb) e = hipMemcpy(h->P.X[h->parity] + I.mk_off, b, mb, hipMemcpyHostToDevice);
    b += mb;
    const size_t eb = storage_bytes(I.storage);
    if (e == hipSuccess)
        e = hipMemcpy((char*)h->P.lat[h->parity] + I.lat_off * eb, b, (size_t)9 * I.plane * eb,
                      hipMemcpyHostToDevice);
    return hip_fail(h, e);
}

int ii_lbm_cutlinks(ii_lbm_handle* h, int32_t inst, ii_lbm_link* out, int32_t cap, int32_t* count)
{
    if (!h || !count || cap < 0 || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    const int rc = sync_and_check(h);
    if (rc) return rc;
    const InstDev& I = h->L.inst[inst];
    // records of the last step live under the parity that step used
    const int par = h->parity ^ 1;
    int n = 0;
    hipError_t e = hipMemcpy(&n, h->P.rec_count + 2 * inst + par, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e);
    if (h->steps == 0) n = 0;
    *count = n;
    const int m = std::min(std::min(n, I.rec_cap), (int)cap);
    if (m > 0 && out)
        e = hipMemcpy(out, h->P.rec + I.rec_off, (size_t)m * sizeof(ii_lbm_link), hipMemcpyDeviceToHost);
    return hip_fail(h, e);
}

int ii_lbm_diag(ii_lbm_handle* h, int32_t inst, ii_lbm_diag_t* out)
{
    if (!h || !out || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    memset(out, 0, sizeof *out);
    int rc = sync_and_check(h);
    const InstDev& I = h->L.inst[inst];
    int errbits = 0;
    hipMemcpy(&errbits, h->P.err + inst, sizeof(int), hipMemcpyDeviceToHost);
    out->error_bits = errbits;
    out->step = h->steps;
    if (rc && rc != II_LBM_EUNSTABLE) return rc;
    hipError_t e = launch_diag(I, h->P.lat[h->parity], h->P.diag, kDiagBlocks, h->stream);
    std::vector<double> part(4 * kDiagBlocks);
    if (e == hipSuccess)
        e = hipMemcpyAsync(part.data(), h->P.diag, part.size() * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    double s[4] = {0, 0, 0, 0};
    for (int b = 0; b < kDiagBlocks; b++)
        for (int c = 0; c < 4; c++) s[c] += part[4 * b + c];
    out->mass = (double)I.nx * I.ny + s[0];
    out->momentum[0] = s[1];
    out->momentum[1] = s[2];
    if (s[3] > 0.0) {
        h->failed = II_LBM_EUNSTABLE;
        out->error_bits |= kErrUnstable;
    }
    const int N = I.n_markers;
    if (N > 0) {
        std::vector<double2> X(N), G(N);
        e = hipMemcpy(X.data(), h->P.X[h->parity] + I.mk_off, N * sizeof(double2), hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(G.data(), h->P.G + I.mk_off, N * sizeof(double2), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(h, e);
        double a = 0.0, fx = 0.0, fy = 0.0;
        for (int k = 0; k < N; k++) {
            const int kp = (k + 1) % N;
            a += X[k].x * X[kp].y - X[kp].x * X[k].y;
            fx -= G[k].x * I.dX;
            fy -= G[k].y * I.dX;
        }
        out->area = 0.5 * a;
        out->force[0] = h->steps > 0 ? fx : 0.0;
        out->force[1] = h->steps > 0 ? fy : 0.0;
        int n = 0;
        if (h->steps > 0)
            hipMemcpy(&n, h->P.rec_count + 2 * inst + (h->parity ^ 1), sizeof(int), hipMemcpyDeviceToHost);
        out->n_cut_links = n;
    }
    return h->failed;
}

int ii_lbm_set_timing(ii_lbm_handle* h, int32_t enable)
{
    if (!h) return II_LBM_EINVAL;
    if (enable && h->ev.empty()) {
        h->ev.resize(kEventPool);
        for (auto& ev : h->ev)
            if (hipEventCreate(&ev) != hipSuccess) return hip_fail(h, hipErrorUnknown);
    }
    h->timing = enable != 0;
    return II_LBM_OK;
}

int ii_lbm_get_timing(ii_lbm_handle* h, double* sweep_ms, int64_t* launches)
{
    if (!h || !sweep_ms || !launches) return II_LBM_EINVAL;
    const hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    double tot = 0.0;
    for (int i = 0; i + 1 < h->ev_used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) != hipSuccess) return hip_fail(h, hipErrorUnknown);
        tot += ms;
    }
    *sweep_ms = tot;
    *launches = h->ev_used / 2;
    h->ev_used = 0;
    return II_LBM_OK;
}

int ii_lbm_sweep_bytes(ii_lbm_handle* h, int32_t inst, double* bytes)
{
    if (!h || !bytes || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    const InstDev& I = h->L.inst[inst];
    *bytes = 18.0 * storage_bytes(I.storage) * (double)I.nx * (double)I.ny;
    return II_LBM_OK;
}

int ii_lbm_destroy(ii_lbm_handle* h)
{
    if (!h) return II_LBM_EINVAL;
    hipStreamSynchronize(h->stream);
    for (auto& ev : h->ev) hipEventDestroy(ev);
    if (h->owns_ws) hipFree(h->ws);
    delete h;
    return II_LBM_OK;
}

const char* ii_lbm_strerror(int code)
{
    switch (code) {
    case II_LBM_OK: return "ok";
    case II_LBM_EINVAL: return "invalid problem or argument";
    case II_LBM_EWORKSPACE: return "workspace missing, misaligned or too small";
    case II_LBM_EDEVICE: return "HIP call failed";
    case II_LBM_EUNSTABLE: return "non-finite state";
    case II_LBM_EGEOMETRY: return "markers outside the supported region or not counter-clockwise";
    case II_LBM_ESTATE: return "handle already failed";
    case II_LBM_ECAPACITY: return "interface too dense for a tile chord list";
    default: return "unknown error";
    }
}

}  // extern "C"
