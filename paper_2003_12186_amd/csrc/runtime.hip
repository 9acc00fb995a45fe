// Host runtime of the II-LBM library: problem validation, workspace layout,
// the per-step launch sequence, readout, checkpoint/restart and the C ABI
// declared in include/ii_lbm.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"

using namespace iilbm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDiagBlocks = 1024;
constexpr int kEventPool = 16384;
constexpr int kXcds = 8;   // MI355X: eight accelerator complex dies, one L2 each

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

// Staging array of ii_lbm_fields_noalloc: one copy per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not a
// device address: its address on each device comes from
// hipGetSymbolAddress, taken once per device at ii_lbm_init and kept in the
// handle.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (the current device).
hipError_t scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

struct Layout {
    std::vector<InstDev> inst;
    size_t lat_bytes = 0;  // one lattice buffer (all instances)
    size_t off_lat[2] = {0, 0};
    size_t off_X[2] = {0, 0}, off_U = 0, off_G = 0, off_Gt = 0, off_jp = 0, off_wx = 0, off_wy = 0, off_f0 = 0;
    size_t off_tile_count = 0, off_tile_list = 0, off_tile_slot[2] = {0, 0}, off_corr[2] = {0, 0};
    size_t off_cmask[2] = {0, 0};
    size_t off_act_list[2] = {0, 0}, off_act_count = 0;
    size_t off_rec = 0, off_rec_count = 0, off_err = 0, off_diag = 0, off_body = 0;
    size_t off_M = 0, off_taps = 0;
    int taps_total = 0;
    size_t off_insts = 0, off_mk_table = 0, off_tile_table = 0, off_sweep_table = 0;
    size_t off_geo_table = 0;
    int mk_units = 0, tile_units = 0, sweep_units_max = 0, geo_units = 0;
    size_t total = 0;
    int n_markers_total = 0, tiles_total = 0, act_total = 0, rec_total = 0;
};

int validate(const ii_lbm_problem& p, const double* X0)
{
    if (p.nx < 8 || p.ny < 8 || p.nx > 8192 || p.ny > 8192) return II_LBM_EINVAL;
    if (!(p.tau > 0.5) || !isfinite(p.tau)) return II_LBM_EINVAL;
    if (p.collision != II_LBM_SRT && p.collision != II_LBM_MRT) return II_LBM_EINVAL;
    for (int i = 0; i < 4; i++)
        if (p.bc[i] < II_LBM_BC_PERIODIC || p.bc[i] > II_LBM_BC_INLET_UNIFORM) return II_LBM_EINVAL;
    if ((p.bc[0] == II_LBM_BC_PERIODIC) != (p.bc[1] == II_LBM_BC_PERIODIC)) return II_LBM_EINVAL;
    if ((p.bc[2] == II_LBM_BC_PERIODIC) != (p.bc[3] == II_LBM_BC_PERIODIC)) return II_LBM_EINVAL;
    for (int q = 1; q < 4; q++)
        if (p.bc[q] == II_LBM_BC_INLET || p.bc[q] == II_LBM_BC_INLET_UNIFORM) return II_LBM_EINVAL;
    if (p.storage != II_LBM_FP32 && p.storage != II_LBM_FP16) return II_LBM_EINVAL;
    if (p.math != II_LBM_MATH_FP32 && p.math != II_LBM_MATH_FP64) return II_LBM_EINVAL;
    if (p.force_mode < II_LBM_FORCE_II || p.force_mode > II_LBM_FORCE_II_GUO) return II_LBM_EINVAL;
    if (p.interface_kind == II_LBM_IF_NONE) return II_LBM_OK;
    if (p.interface_kind != II_LBM_IF_MEMBRANE && p.interface_kind != II_LBM_IF_RIGID &&
        p.interface_kind != II_LBM_IF_NORMAL)
        return II_LBM_EINVAL;
    if (p.n_markers < 3 || p.n_markers > (1 << 20)) return II_LBM_EINVAL;
    if (!(p.dX > 0.0) || p.dX > 2.0 || !(p.kappa >= 0.0)) return II_LBM_EINVAL;
    if ((p.interface_kind == II_LBM_IF_RIGID || p.interface_kind == II_LBM_IF_NORMAL) &&
        !(p.radius > 0.0))
        return II_LBM_EINVAL;
    if (p.interface_kind == II_LBM_IF_NORMAL && !isfinite(p.f_normal)) return II_LBM_EINVAL;
    if (p.geometry != 0 && p.geometry != 1) return II_LBM_EINVAL;
    if (p.geometry == 1 && p.interface_kind != II_LBM_IF_MEMBRANE) return II_LBM_EINVAL;
    const bool moving = p.body_free != 0 || p.presc_umax[0] != 0.0 || p.presc_umax[1] != 0.0;
    if (moving) {
        if (p.interface_kind != II_LBM_IF_RIGID || (p.body_free & ~7)) return II_LBM_EINVAL;
        if (p.body_free && !(p.rho_star > 0.0 && isfinite(p.rho_star))) return II_LBM_EINVAL;
        for (int a = 0; a < 2; a++) {
            if (!isfinite(p.spring[a]) || !isfinite(p.damping[a])) return II_LBM_EINVAL;
            if (p.presc_umax[a] != 0.0 && !(fabs(p.presc_amp[a]) > 0.0)) return II_LBM_EINVAL;
        }
    }
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
        if (l > 4.0 || l == 0.0) return II_LBM_EGEOMETRY;
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
    if (p.interface_kind == II_LBM_IF_NORMAL) est = std::max(est, 3.0 * fabs(p.f_normal));
    est = std::max(est, 3.0 * std::max(fabs(p.presc_umax[0]), fabs(p.presc_umax[1])));
    est = std::max(est, 1e-7);
    return (int)floor(log2(est)) - 12;
}

int build_layout(const ii_lbm_problem* p, int n_inst, Layout& L)
{
    L.inst.resize(n_inst);
    size_t lat = 0;
    int mk = 0, tiles = 0, act = 0, rec = 0, taps = 0;
    long long list = 0;
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
        I.jumps = q.force_mode == II_LBM_FORCE_II || q.force_mode == II_LBM_FORCE_II_GUO;
        I.guo = q.force_mode == II_LBM_FORCE_IB_GUO || q.force_mode == II_LBM_FORCE_II_GUO;
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
        I.f_normal = q.f_normal;
        I.geometry = q.interface_kind == II_LBM_IF_MEMBRANE ? q.geometry : 0;
        I.spl_periodic = I.n_markers <= 64;
        I.tap_off = taps;
        if (I.geometry == 1) taps += I.spl_periodic ? I.n_markers : 65;
        I.moving = q.interface_kind == II_LBM_IF_RIGID &&
                   (q.body_free != 0 || q.presc_umax[0] != 0.0 || q.presc_umax[1] != 0.0);
        I.body_free = q.body_free;
        I.rho_star = q.rho_star;
        for (int a = 0; a < 2; a++) {
            I.spring[a] = q.spring[a];
            I.damping[a] = q.damping[a];
            I.presc_amp[a] = q.presc_amp[a];
            I.presc_umax[a] = q.presc_umax[a];
        }
        I.mk_off = mk;
        mk += I.n_markers;
        I.tiles_x = (q.nx + kTile - 1) / kTile;
        I.tiles_y = (q.ny + kTile - 1) / kTile;
        I.tile_off = tiles;
        tiles += I.tiles_x * I.tiles_y;
        I.tile_cap = I.jumps ? kTileCap : kTileCapIB;
        I.list_off = list;
        list += (long long)I.tiles_x * I.tiles_y * I.tile_cap;
        I.act_off = act;
        // tiles within 2.5 lu of a closed curve of N chords; the bound leaves
        // room for chords of up to 4 lu (longer curves report ECAPACITY), and
        // the record buffer for the links such chords cut
        I.act_cap = std::min(I.tiles_x * I.tiles_y, I.n_markers + 256);
        act += I.act_cap;
        I.rec_off = rec;
        I.rec_cap = 32 * I.n_markers + 1024;
        rec += I.rec_cap;
        I.mk_blocks = (16 * I.n_markers + 255) / 256;
        I.tile_blocks = std::max(1, std::min(I.act_cap, 2048));
        L.mk_units += I.n_markers > 0 ? I.mk_blocks : 0;
        L.geo_units += (I.n_markers + 255) / 256;
        L.sweep_units_max += (int)(((long long)q.nx * q.ny + 127) / 128);
        if (j == n_inst - 1) L.sweep_units_max += kXcds;   // padding of the XCD interleave
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
    L.off_tile_list = take((size_t)std::max(list, 1LL) * sizeof(int));
    for (int q = 0; q < 2; q++) {
        L.off_tile_slot[q] = take((size_t)tiles * sizeof(int));
        L.off_corr[q] = take((size_t)std::max(act, 1) * kCorrPlanes * kTileNodes * sizeof(float));
        L.off_cmask[q] = take((size_t)std::max(act, 1) * 4 * sizeof(unsigned long long));
    }
    L.off_act_list[0] = take((size_t)std::max(act, 1) * sizeof(int2));
    L.off_act_list[1] = take((size_t)std::max(act, 1) * sizeof(int2));
    L.off_act_count = take((size_t)2 * n_inst * sizeof(int));
    L.off_rec = take((size_t)std::max(rec, 1) * sizeof(ii_lbm_link));
    L.off_rec_count = take((size_t)2 * n_inst * sizeof(int));
    L.off_err = take((size_t)n_inst * sizeof(int));
    L.off_diag = take((size_t)8 * kDiagBlocks * sizeof(double));
    L.off_body = take((size_t)n_inst * sizeof(BodyDev));
    L.off_M = take(nm * sizeof(double2));
    L.taps_total = taps;
    L.off_taps = take((size_t)std::max(taps, 1) * sizeof(double));
    // batched launches: descriptors and work tables (tile table sized for the
    // largest per-instance block count)
    int tile_units = 0;
    for (const InstDev& I : L.inst) tile_units += I.n_markers > 0 ? I.act_cap : 0;
    L.off_insts = take((size_t)n_inst * sizeof(InstDev));
    L.off_mk_table = take((size_t)std::max(L.mk_units, 1) * sizeof(int2));
    L.off_geo_table = take((size_t)std::max(L.geo_units, 1) * sizeof(int2));
    L.off_tile_table = take((size_t)std::max(tile_units, 1) * sizeof(int2));
    L.off_sweep_table = take((size_t)std::max(L.sweep_units_max, 1) * sizeof(int2));
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
    // Membranes' steps build no cut-link records; rec_fresh: those of the
    // current markers have been built since (ensure_records)
    bool rec_fresh = false;
    // isolation (ii_lbm_set_isolation): an instance's own errors are kept in
    // its error bits and do not stop the handle
    bool isolate = false;
    bool timing = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs
    int ev_used = 0;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
    // batched mode (several instances): one launch per phase for all of them
    bool batched = false;
    Batch batch;
    int sweep_order = 0;           // 0: instance order, 1: largest instances first
    double tuned_us = 0.0;
    std::vector<int> tile_est;     // estimated active tiles per instance (batched)
    int tile_per_cu = 0;           // tile-pass blocks per CU (0: one per estimated tile)
    double tuned_step_us = 0.0;    // the autotuner's fastest whole step
    // hipGraph replay: graphs of two steps and a ladder of longer ones (the
    // longest of graph_steps steps, then the powers of two below it down to
    // four), one per length and starting parity
    bool use_graph = false;
    int graph_steps = 64;          // steps of the longest graph (even; 2: the pair only)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};       // two steps, per starting parity
    static constexpr int kLadder = 7;                   // 256, 128, ..., 4 at most
    int ladder[kLadder] = {};                           // lengths, longest first (0: unused)
    hipGraphExec_t gexec_long[kLadder][2] = {};
    // Membranes: the interface work of step m+1 runs on `aux` while the
    // sweep of step m runs on the main stream (fork/join through events).
    bool lookahead = false;
    int overlap = 1;           // II_LBM_OVERLAP_* (membranes only)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool rec_valid = false;  // rigid bodies: a step has built cut-link records
    int n_cu = 256;
    // learned correction after every step (ii_lbm_set_learned): its marker-
    // only phases run on `lrn` as soon as the step's interpolation has moved
    // the markers (ev_x); ev_b / ev_g mark its band tiles / patch geometry
    LearnedCfg learned;
    hipStream_t lrn = nullptr;
    hipEvent_t ev_x = nullptr, ev_b = nullptr, ev_g = nullptr;
    // this device's static staging array (ii_lbm_fields_noalloc)
    void* scratch = nullptr;
};

static int hip_fail(ii_lbm_handle* h, hipError_t e)
{
    if (e == hipSuccess) return II_LBM_OK;
    if (h) h->failed = II_LBM_EDEVICE;
    return II_LBM_EDEVICE;
}

static int check_device_errors(ii_lbm_handle* h)
{
    // the instances' error words in chunks through a stack buffer (no
    // allocation, so the allocation-free readout can use this too)
    const int n = (int)h->prob.size();
    int bits = 0;
    for (int j0 = 0; j0 < n; j0 += 64) {
        int err[64];
        const int m = std::min(64, n - j0);
        hipError_t e = hipMemcpyAsync(err, h->P.err + j0, m * sizeof(int), hipMemcpyDeviceToHost,
                                      h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e);
        for (int q = 0; q < m; q++) bits |= err[q];
    }
    if (h->isolate) return h->failed;
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

// Tiles within 2.5 lu of the initial chords: the tile kernel's blocks per
// instance (they stride over whatever the active count turns out to be).
static int estimate_active_tiles(const ii_lbm_problem& p, const double* X0)
{
    const int N = p.n_markers, tx = (p.nx + kTile - 1) / kTile, ty = (p.ny + kTile - 1) / kTile;
    std::vector<unsigned char> hit((size_t)tx * ty, 0);
    int n = 0;
    for (int k = 0; k < N; k++) {
        const int kp = (k + 1) % N;
        const double x0 = std::min(X0[2 * k], X0[2 * kp]) - 2.5, x1 = std::max(X0[2 * k], X0[2 * kp]) + 2.5;
        const double y0 = std::min(X0[2 * k + 1], X0[2 * kp + 1]) - 2.5,
                     y1 = std::max(X0[2 * k + 1], X0[2 * kp + 1]) + 2.5;
        for (int b = std::max(0, (int)floor(y0 / kTile)); b <= std::min(ty - 1, (int)floor(y1 / kTile)); b++)
            for (int a = std::max(0, (int)floor(x0 / kTile)); a <= std::min(tx - 1, (int)floor(x1 / kTile)); a++)
                if (!hit[(size_t)b * tx + a]) { hit[(size_t)b * tx + a] = 1; n++; }
    }
    return n;
}

// Sweep work table: slices of `unit` nodes, instances in the given order.
static std::vector<int2> sweep_table(const Layout& L, int unit, int order)
{
    std::vector<int> idx(L.inst.size());
    for (size_t j = 0; j < idx.size(); j++) idx[j] = (int)j;
    if (order == 1)
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return (long long)L.inst[a].nx * L.inst[a].ny > (long long)L.inst[b].nx * L.inst[b].ny;
        });
    std::vector<int2> t;
    for (int j : idx) {
        const long long n = (long long)L.inst[j].nx * L.inst[j].ny;
        for (long long r = 0; r < n; r += unit) t.push_back(make_int2(j, (int)r));
    }
    // Workgroups go to the XCDs round-robin by index, each XCD with its own
    // L2.  Cut the slice sequence into one contiguous run per XCD and
    // interleave the runs, so that an XCD sweeps neighbouring rows and reads
    // their y +- 1 neighbours from its own L2; (-1, 0) pads the last round.
    const size_t per = (t.size() + kXcds - 1) / kXcds;
    std::vector<int2> out(per * kXcds, make_int2(-1, 0));
    for (size_t q = 0; q < t.size(); q++) out[(q % per) * kXcds + q / per] = t[q];
    return out;
}

static hipError_t upload_sweep_table(ii_lbm_handle* h, int unit, int order)
{
    const std::vector<int2> t = sweep_table(h->L, unit, order);
    hipError_t e = hipMemcpy((void*)h->batch.sweep_table, t.data(), t.size() * sizeof(int2),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        h->batch.sweep_units = (int)t.size();
        h->batch.sweep_unit = unit;
        h->sweep_order = order;
    }
    return e;
}

// Interface phases of one step on stream s: slot/count reset of plane `par`
// (unless the interpolation just before did it: `reset` false), the marker
// pass (`mode`), then the tile pass (with the cut-link records when
// `records`).
static hipError_t enqueue_interface(ii_lbm_handle* h, int par, int mode, hipStream_t s,
                                    bool records, bool reset = true)
{
    void* A = h->P.lat[par];
    hipError_t e = hipSuccess;
    if (h->batched) {
        if (reset) e = launch_slot_reset_batch(h->batch, (int)h->L.inst.size(), h->P, par, s);
        if (e == hipSuccess) e = launch_markers_batch(h->batch, h->P, A, par, mode, s);
        if (e == hipSuccess) e = launch_tiles_batch(h->batch, h->P, par, records, s);
        return e;
    }
    for (size_t j = 0; j < h->L.inst.size() && e == hipSuccess; j++) {
        const InstDev& I = h->L.inst[j];
        if (I.n_markers == 0) continue;
        if (reset) e = launch_slot_reset(I, h->P, par, s);
        if (e == hipSuccess && I.geometry == 1) e = launch_spline(I, h->P, par, s);
        if (e == hipSuccess) e = launch_markers(I, h->P, A, par, mode, s);
        if (e == hipSuccess) e = launch_tiles(I, h->P, par, records, s);
    }
    return e;
}

static hipError_t enqueue_sweep(ii_lbm_handle* h, int par, hipStream_t s, bool timed)
{
    void* A = h->P.lat[par];
    void* B = h->P.lat[par ^ 1];
    hipError_t e = hipSuccess;
    if (h->batched) {
        if (timed) (void)hipEventRecord(h->ev[h->ev_used], s);
        e = launch_sweep_batch(h->batch, h->P, A, B, par, s);
        if (timed) {
            (void)hipEventRecord(h->ev[h->ev_used + 1], s);
            h->ev_used += 2;
        }
        return e;
    }
    for (size_t j = 0; j < h->L.inst.size() && e == hipSuccess; j++) {
        const bool t = timed && h->ev_used + 2 <= (int)h->ev.size();
        if (t) (void)hipEventRecord(h->ev[h->ev_used], s);
        e = launch_sweep(h->L.inst[j], h->P, A, B, par, s);
        if (t) {
            (void)hipEventRecord(h->ev[h->ev_used + 1], s);
            h->ev_used += 2;
        }
    }
    return e;
}

// Interpolation of step m on plane `par` from f^m (U^m, X^{m+1}).
static hipError_t enqueue_interp(ii_lbm_handle* h, int par, hipStream_t s)
{
    void* A = h->P.lat[par];
    if (h->batched) return launch_markers_batch(h->batch, h->P, A, par, kModeInterp, s);
    hipError_t e = hipSuccess;
    for (size_t j = 0; j < h->L.inst.size() && e == hipSuccess; j++)
        e = launch_markers(h->L.inst[j], h->P, A, par, kModeInterp, s);
    return e;
}

// Enqueue one time step of every instance on stream s (no host work besides
// launches and event operations, so it can be captured into a graph).
//   membranes, by overlap mode (the sweep of step m and the interface pass of
//   step m+1 touch disjoint buffers):
//     SERIAL:  sweep(m), interp(m), reset/geom/tiles(m+1), all on s
//     FULL:    fork -> aux: interp(m), reset/geom/tiles(m+1); s: sweep(m) -> join
//     INTERP_FIRST: interp(m) on s, fork -> aux: reset/geom/tiles(m+1);
//              s: sweep(m) -> join
//   rigid bodies: full markers (resetting the slot plane of m+1)/tiles(m) ->
//     sweep(m), in order on s
// The learned correction's phases for the state of plane `par` on stream s.
static hipError_t enqueue_learned(ii_lbm_handle* h, int par, hipStream_t s,
                                  hipError_t (*phase)(const HandleView&, const LearnedCfg&))
{
    HandleView v;
    handle_view(h, &v);
    v.parity = par;
    v.stream = s;
    return phase(v, h->learned);
}

// `records`: a rigid body's tile pass also writes the cut-link records.  Only
// the newest step's are ever reported, so a graph builds them on its last step.
static hipError_t enqueue_step(ii_lbm_handle* h, int par, hipStream_t s, bool timed,
                               bool records = true)
{
    hipError_t e = hipSuccess;
    const bool lrn = h->learned.on;
    if (h->lookahead && h->overlap == II_LBM_OVERLAP_SERIAL) {
        e = enqueue_sweep(h, par, s, timed);
        if (e == hipSuccess) e = enqueue_interp(h, par, s);
        if (e == hipSuccess) e = enqueue_interface(h, par ^ 1, kModeGeom, s, false, false);
        if (lrn) {
            if (e == hipSuccess) e = enqueue_learned(h, par ^ 1, s, learned_band);
            if (e == hipSuccess) e = enqueue_learned(h, par ^ 1, s, learned_geom);
            if (e == hipSuccess) e = enqueue_learned(h, par ^ 1, s, learned_flow);
            if (e == hipSuccess) e = enqueue_learned(h, par ^ 1, s, learned_infer);
        }
        return e;
    }
    if (h->lookahead) {
        const bool first = h->overlap == II_LBM_OVERLAP_INTERP_FIRST;
        if (first) e = enqueue_interp(h, par, s);
        if (e == hipSuccess) e = hipEventRecord(h->ev_fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->aux, h->ev_fork, 0);
        if (e == hipSuccess && !first) e = enqueue_interp(h, par, h->aux);
        if (lrn) {
            // band tiles and patch geometry of the next state need only the
            // moved markers X^{m+1}; they run beside the sweep and the
            // interface pass
            if (e == hipSuccess) e = hipEventRecord(h->ev_x, first ? s : h->aux);
            if (e == hipSuccess) e = hipStreamWaitEvent(h->lrn, h->ev_x, 0);
            if (e == hipSuccess) e = enqueue_learned(h, par ^ 1, h->lrn, learned_band);
            if (e == hipSuccess) e = hipEventRecord(h->ev_b, h->lrn);
            if (e == hipSuccess) e = enqueue_learned(h, par ^ 1, h->lrn, learned_geom);
            if (e == hipSuccess) e = hipEventRecord(h->ev_g, h->lrn);
        }
        if (e == hipSuccess) e = enqueue_interface(h, par ^ 1, kModeGeom, h->aux, false, false);
        if (e == hipSuccess) e = enqueue_sweep(h, par, s, timed);
        if (lrn) {
            // patch flow and the network need the swept lattice; the interface
            // pass of the next step does not read it, so they overlap it too
            if (e == hipSuccess) e = hipStreamWaitEvent(s, h->ev_b, 0);
            if (e == hipSuccess) e = enqueue_learned(h, par ^ 1, s, learned_flow);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, h->ev_g, 0);
            if (e == hipSuccess) e = enqueue_learned(h, par ^ 1, s, learned_infer);
        }
        if (e == hipSuccess) e = hipEventRecord(h->ev_join, h->aux);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, h->ev_join, 0);
        return e;
    }
    // the plane of this step was reset by the previous step's marker pass
    // (or is still as the set-up left it)
    e = enqueue_interface(h, par, kModeFull, s, records, false);
    if (e == hipSuccess) e = enqueue_sweep(h, par, s, timed);
    for (size_t j = 0; j < h->L.inst.size() && e == hipSuccess; j++)
        if (h->L.inst[j].moving) e = launch_body(h->L.inst[j], h->P, par, s);
    return e;
}

// Membranes: build the interface data of the current step from the current
// markers (after init, set_markers or load_state).
static hipError_t prime(ii_lbm_handle* h)
{
    if (!h->lookahead) return hipSuccess;
    h->rec_fresh = false;
    const hipError_t e = enqueue_interface(h, h->parity, kModeGeom, h->stream, false);
    return e == hipSuccess ? hipStreamSynchronize(h->stream) : e;
}

// Membranes: the cut-link records of the current markers, for the calls that
// report them.  The interface pass of the current plane runs again with the
// records on; it is a deterministic function of the markers and rewrites the
// same forces, tile lists and corrections that the next sweep reads.
static int ensure_records(ii_lbm_handle* h)
{
    if (!h->lookahead || h->rec_fresh) return II_LBM_OK;
    hipError_t e = enqueue_interface(h, h->parity, kModeGeom, h->stream, true);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e);
    h->rec_fresh = true;
    return check_device_errors(h);
}

static void drop_graphs(ii_lbm_handle* h)
{
    // replays run on the handle's stream: let any in flight finish first
    bool any = h->gexec[0] || h->gexec[1];
    for (auto& pair : h->gexec_long) any = any || pair[0] || pair[1];
    if (any) (void)hipStreamSynchronize(h->stream);
    for (auto& g : h->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    for (auto& pair : h->gexec_long)
        for (auto& g : pair)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

// Lengths of the long graphs for the longest L: L, then the powers of two
// below it down to four (a call of n steps replays them greedily, so that
// few launches cover it: 20 steps of the default ladder take 16 + 4).
static void set_ladder(ii_lbm_handle* h, int L)
{
    for (int& v : h->ladder) v = 0;
    if (L <= 2) return;
    int q = 0;
    h->ladder[q++] = L;
    int p = 1;
    while (p * 2 < L) p *= 2;
    for (; p >= 4 && q < ii_lbm_handle::kLadder; p /= 2) h->ladder[q++] = p;
}

// Blocks of the batched tile pass.  per_cu = 0: one block per estimated
// active tile of each instance (plus a quarter), the fastest pass on its own;
// per_cu > 0: about per_cu blocks per CU in all, shared in proportion to the
// instances' estimates (at least one each), every block walking several of
// its instance's tiles.  Beside the sweep a smaller footprint leaves the
// sweep's waves more of each CU.  The caller has synchronised the handle.
static hipError_t upload_tile_table(ii_lbm_handle* h, int per_cu)
{
    long long tot = 0;
    for (size_t j = 0; j < h->L.inst.size(); j++)
        if (h->L.inst[j].n_markers > 0) tot += h->tile_est[j];
    std::vector<int2> tl;
    for (size_t j = 0; j < h->L.inst.size(); j++) {
        InstDev& I = h->L.inst[j];
        if (I.n_markers == 0) continue;
        const long long est = h->tile_est[j];
        long long nb = est + est / 4 + 1;
        if (per_cu > 0)
            nb = std::min(nb, (long long)per_cu * h->n_cu * est / std::max(tot, 1LL));
        I.tile_blocks = (int)std::max(1LL, std::min((long long)I.act_cap, nb));
        for (int q = 0; q < I.tile_blocks; q++) tl.push_back(make_int2((int)j, q));
    }
    hipError_t e = hipSuccess;
    if (!tl.empty())
        e = hipMemcpy((void*)h->batch.tile_table, tl.data(), tl.size() * sizeof(int2),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy((void*)h->batch.insts, h->L.inst.data(), h->L.inst.size() * sizeof(InstDev),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        h->batch.tile_units = (int)tl.size();
        h->tile_per_cu = per_cu;
    }
    drop_graphs(h);
    return e;
}

// n (even) steps starting at parity `par`, captured on the handle's own
// stream into *out; the last step builds the cut-link records.
static hipError_t build_graph(ii_lbm_handle* h, int par, int n, hipGraphExec_t* out)
{
    if (!h->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e1 = hipSuccess;
    for (int k = 0; k < n && e1 == hipSuccess; k++)
        e1 = enqueue_step(h, par ^ (k & 1), h->cap_stream, false, k == n - 1);
    e = hipStreamEndCapture(h->cap_stream, &g);
    if (e1 != hipSuccess) e = e1;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

// Every graph (the pair and each long length, one of each per starting
// parity) at once: an odd number of direct steps between replays flips the
// parity, and no graph may be captured and instantiated in the middle of a
// caller's timed loop.
static hipError_t ensure_graphs(ii_lbm_handle* h)
{
    if (h->ladder[0] != (h->graph_steps > 2 ? h->graph_steps : 0)) set_ladder(h, h->graph_steps);
    for (int par = 0; par < 2; par++) {
        if (!h->gexec[par]) {
            const hipError_t e = build_graph(h, par, 2, &h->gexec[par]);
            if (e != hipSuccess) return e;
        }
        for (int q = 0; q < ii_lbm_handle::kLadder && h->ladder[q] > 0; q++)
            if (!h->gexec_long[q][par]) {
                const hipError_t e = build_graph(h, par, h->ladder[q], &h->gexec_long[q][par]);
                if (e != hipSuccess) return e;
            }
    }
    return hipSuccess;
}

// Plane of the newest cut-link records: membranes hold those of the current
// markers, rigid bodies those built by the last step (-1: none yet).
static int record_parity(const ii_lbm_handle* h)
{
    if (h->lookahead) return h->parity;
    return h->rec_valid ? (h->parity ^ 1) : -1;
}

// Blocks of the tile kernel of a single instance.  Beside the sweep it runs
// with one block per CU (each block walks several tiles), which leaves the
// sweep more room; on the critical path it runs with up to 2048 blocks.
static void size_tile_blocks(ii_lbm_handle* h)
{
    if (h->batched) return;
    const bool beside = h->lookahead && h->overlap != II_LBM_OVERLAP_SERIAL;
    const int per_cu = h->tile_per_cu > 0 ? h->tile_per_cu : 1;
    // the spline's tile pass carries root finding and is the step's critical
    // path even beside the sweep: it keeps every block
    for (InstDev& I : h->L.inst)
        if (I.n_markers > 0)
            I.tile_blocks =
                std::max(1, std::min(I.act_cap, beside && I.geometry != 1 ? per_cu * h->n_cu : 2048));
}

static void release(ii_lbm_handle* h)
{
    drop_graphs(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->aux) (void)hipStreamDestroy(h->aux);
    if (h->lrn) (void)hipStreamDestroy(h->lrn);
    for (hipEvent_t ev : {h->ev_x, h->ev_b, h->ev_g})
        if (ev) (void)hipEventDestroy(ev);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    for (auto& ev : h->ev) (void)hipEventDestroy(ev);
    if (h->owns_ws) (void)hipFree(h->ws);
    delete h;
}

namespace iilbm {
int handle_view(ii_lbm_handle* h, HandleView* v)
{
    if (!h || !v) return II_LBM_EINVAL;
    v->n_inst = (int)h->prob.size();
    v->inst = h->L.inst.data();
    v->d_inst = (const InstDev*)(h->ws + h->L.off_insts);
    v->P = h->P;
    v->parity = h->parity;
    v->stream = h->stream;
    v->failed = h->failed;
    v->n_cu = h->n_cu;
    return II_LBM_OK;
}
}  // namespace iilbm

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
    for (int q = 0; q < 2; q++) {
        P.tile_slot[q] = (int*)(h->ws + L.off_tile_slot[q]);
        P.corr[q] = (float*)(h->ws + L.off_corr[q]);
        P.cmask[q] = (unsigned long long*)(h->ws + L.off_cmask[q]);
    }
    P.act_list[0] = (int2*)(h->ws + L.off_act_list[0]);
    P.act_list[1] = (int2*)(h->ws + L.off_act_list[1]);
    P.act_count = (int*)(h->ws + L.off_act_count);
    P.rec = (ii_lbm_link*)(h->ws + L.off_rec);
    P.rec_count = (int*)(h->ws + L.off_rec_count);
    P.err = (int*)(h->ws + L.off_err);
    P.diag = (double*)(h->ws + L.off_diag);
    P.body = (BodyDev*)(h->ws + L.off_body);
    P.M = (double2*)(h->ws + L.off_M);
    P.spline_taps = (const double*)(h->ws + L.off_taps);

    hipError_t e = hipSuccess;
    for (int j = 0; j < n_inst && e == hipSuccess; j++) {
        e = launch_fill_zero(L.inst[j], P.lat[0], h->stream);
        if (e == hipSuccess) e = launch_fill_zero(L.inst[j], P.lat[1], h->stream);
    }
    if (e == hipSuccess) e = launch_fill_ints(P.tile_count, L.tiles_total, 0, h->stream);
    for (int q = 0; q < 2 && e == hipSuccess; q++)
        e = launch_fill_ints(P.tile_slot[q], L.tiles_total, -1, h->stream);
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
    // Spline taps: the inverse of the cyclic system M_{k-1} + 4 M_k + M_{k+1},
    // g_j = lambda^|j| / (2 sqrt 3) with lambda = sqrt 3 - 2 for |j| <= 32, or
    // its periodic sum (lambda^j + lambda^(N-j)) / (2 sqrt 3 (1 - lambda^N)),
    // j = 0 .. N-1, for N <= 64 markers.
    if (e == hipSuccess && L.taps_total > 0) {
        std::vector<double> taps(L.taps_total);
        const double lam = sqrt(3.0) - 2.0, c0 = 1.0 / (2.0 * sqrt(3.0));
        for (int j = 0; j < n_inst; j++) {
            const InstDev& I = L.inst[j];
            if (I.geometry != 1) continue;
            const int N = I.n_markers;
            if (I.spl_periodic) {
                const double lN = pow(lam, N);
                for (int q = 0; q < N; q++)
                    taps[I.tap_off + q] = (pow(lam, q) + pow(lam, N - q)) * c0 / (1.0 - lN);
            } else {
                for (int q = -32; q <= 32; q++) taps[I.tap_off + q + 32] = pow(lam, abs(q)) * c0;
            }
        }
        e = hipMemcpyAsync((void*)P.spline_taps, taps.data(), taps.size() * sizeof(double),
                           hipMemcpyHostToDevice, h->stream);
    }
    // Moving bodies start at their initial centre, at rest (a prescribed axis
    // at its velocity of t = 0), in orientation 0.
    {
        std::vector<BodyDev> bodies(n_inst);
        for (int j = 0; j < n_inst; j++) {
            BodyDev& b = bodies[j];
            memset(&b, 0, sizeof b);
            b.c[0] = b.c0[0] = p[j].center[0];
            b.c[1] = b.c0[1] = p[j].center[1];
            for (int a = 0; a < 2; a++)
                if (p[j].presc_umax[a] != 0.0) b.U[a] = b.Uprev[a] = -p[j].presc_umax[a];
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(P.body, bodies.data(), n_inst * sizeof(BodyDev),
                               hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    // Several instances advance together through the batched launches; they
    // share storage precision, collision arithmetic, force mode and interface
    // kind; a moving body has a handle of its own.
    if (e == hipSuccess && n_inst > 1) {
        int iface = II_LBM_IF_NONE;
        for (int j = 0; j < n_inst; j++) {
            if (p[j].storage != p[0].storage || p[j].math != p[0].math ||
                p[j].force_mode != p[0].force_mode || h->L.inst[j].moving ||
                h->L.inst[j].geometry != 0) {
                e = hipErrorInvalidValue;
                break;
            }
            if (p[j].interface_kind != II_LBM_IF_NONE) {
                if (iface != II_LBM_IF_NONE && iface != p[j].interface_kind) {
                    e = hipErrorInvalidValue;
                    break;
                }
                iface = p[j].interface_kind;
            }
        }
        if (e != hipSuccess) {
            if (h->owns_ws) (void)hipFree(h->ws);
            delete h;
            return II_LBM_EINVAL;
        }
        h->batched = true;
        Batch& b = h->batch;
        b.insts = (const InstDev*)(h->ws + L.off_insts);
        b.mk_table = (const int2*)(h->ws + L.off_mk_table);
        b.geo_table = (const int2*)(h->ws + L.off_geo_table);
        b.tile_table = (const int2*)(h->ws + L.off_tile_table);
        b.sweep_table = (const int2*)(h->ws + L.off_sweep_table);
        b.storage = p[0].storage;
        b.math = p[0].math;
        b.iface = iface;
        b.guo = h->L.inst[0].guo;
        b.jumps = h->L.inst[0].jumps;
        std::vector<int2> mk, tl, geo;
        h->tile_est.assign(n_inst, 0);
        for (int j = 0; j < n_inst; j++) {
            InstDev& I = h->L.inst[j];
            if (I.n_markers == 0) continue;
            const int est = estimate_active_tiles(p[j], X0[j]);
            h->tile_est[j] = est;
            I.tile_blocks = std::max(1, std::min(I.act_cap, est + est / 4 + 1));
            for (int q = 0; q < I.mk_blocks; q++) mk.push_back(make_int2(j, q));
            for (int q = 0; q < (I.n_markers + 255) / 256; q++) geo.push_back(make_int2(j, q));
            for (int q = 0; q < I.tile_blocks; q++) tl.push_back(make_int2(j, q));
        }
        b.mk_units = (int)mk.size();
        b.geo_units = (int)geo.size();
        b.tile_units = (int)tl.size();
        e = hipMemcpy((void*)b.insts, h->L.inst.data(), n_inst * sizeof(InstDev), hipMemcpyHostToDevice);
        if (e == hipSuccess && !mk.empty())
            e = hipMemcpy((void*)b.mk_table, mk.data(), mk.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess && !geo.empty())
            e = hipMemcpy((void*)b.geo_table, geo.data(), geo.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess && !tl.empty())
            e = hipMemcpy((void*)b.tile_table, tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = upload_sweep_table(h, 256, 1);
    }
    // every handle keeps a device copy of its descriptors
    if (e == hipSuccess)
        e = hipMemcpy(h->ws + L.off_insts, h->L.inst.data(), n_inst * sizeof(InstDev),
                      hipMemcpyHostToDevice);
    // membranes (no direct forcing) take the overlapped schedule
    bool any = false, all_membrane = true;
    for (int j = 0; j < n_inst; j++)
        if (p[j].interface_kind != II_LBM_IF_NONE) {
            any = true;
            all_membrane = all_membrane && p[j].interface_kind == II_LBM_IF_MEMBRANE;
        }
    h->lookahead = any && all_membrane;
    h->overlap = II_LBM_OVERLAP_FULL;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            h->n_cu = cus;
    }
    size_tile_blocks(h);
    if (e == hipSuccess) e = scratch_address(&h->scratch);
    if (e == hipSuccess && h->lookahead) {
        e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = prime(h);
    if (e != hipSuccess) {
        release(h);
        return II_LBM_EDEVICE;
    }
    *out = h;
    return II_LBM_OK;
}

int ii_lbm_step(ii_lbm_handle* h, int64_t n_steps)
{
    if (!h || n_steps < 0) return II_LBM_EINVAL;
    if (h->failed) return II_LBM_ESTATE;
    int64_t left = n_steps;
    if (h->use_graph && !h->timing) {
        if (left >= 2) {
            const hipError_t e = ensure_graphs(h);
            if (e != hipSuccess) return hip_fail(h, e);
        }
        // an even number of steps leaves the parity unchanged
        for (int q = 0; q < ii_lbm_handle::kLadder && h->ladder[q] > 0; q++)
            while (left >= h->ladder[q]) {
                const hipError_t e = hipGraphLaunch(h->gexec_long[q][h->parity], h->stream);
                if (e != hipSuccess) return hip_fail(h, e);
                h->steps += h->ladder[q];
                left -= h->ladder[q];
            }
        while (left >= 2) {
            const hipError_t e = hipGraphLaunch(h->gexec[h->parity], h->stream);
            if (e != hipSuccess) return hip_fail(h, e);
            h->steps += 2;
            left -= 2;
        }
    }
    for (; left > 0; left--) {
        const bool timed = h->timing && h->ev_used + 2 <= (int)h->ev.size();
        const hipError_t e = enqueue_step(h, h->parity, h->stream, timed);
        if (e != hipSuccess) return hip_fail(h, e);
        h->parity ^= 1;
        h->steps++;
    }
    if (n_steps > 0) {
        h->rec_valid = true;
        h->rec_fresh = false;
    }
    return II_LBM_OK;
}

int ii_lbm_set_overlap(ii_lbm_handle* h, int32_t mode)
{
    if (!h || mode < II_LBM_OVERLAP_SERIAL || mode > II_LBM_OVERLAP_INTERP_FIRST) return II_LBM_EINVAL;
    if (h->overlap != mode) drop_graphs(h);
    h->overlap = mode;
    size_tile_blocks(h);
    return II_LBM_OK;
}

int ii_lbm_set_learned(ii_lbm_handle* h, const float* params, const void* packed,
                       const ii_cnn_scales* sc, int32_t cap, int32_t* tiles, int32_t* count,
                       uint16_t* in, uint8_t* flags, float* pscale)
{
    if (!h) return II_LBM_EINVAL;
    if (!params) {
        if (h->learned.on) drop_graphs(h);
        h->learned = LearnedCfg();
        return II_LBM_OK;
    }
    HandleView v;
    handle_view(h, &v);
    int rc = learned_validate(v, cap);
    if (rc) return rc;
    if (!packed || !sc || !tiles || !count || !in || !flags || !pscale) return II_LBM_EINVAL;
    if (!h->lrn) {
        hipError_t e = hipStreamCreateWithFlags(&h->lrn, hipStreamNonBlocking);
        for (hipEvent_t* ev : {&h->ev_x, &h->ev_b, &h->ev_g})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(h, e);
    }
    LearnedCfg c;
    c.on = true;
    c.params = params;
    c.packed = packed;
    c.sc = *sc;
    c.cap = cap;
    c.tiles = tiles;
    c.count = count;
    c.in = in;
    c.flags = flags;
    c.pscale = pscale;
    drop_graphs(h);
    h->learned = c;
    return II_LBM_OK;
}

int ii_lbm_set_isolation(ii_lbm_handle* h, int32_t enable)
{
    if (!h) return II_LBM_EINVAL;
    h->isolate = enable != 0;
    return II_LBM_OK;
}

int ii_lbm_instance_errors(ii_lbm_handle* h, int32_t* bits, int32_t n)
{
    if (!h || !bits || n < 0) return II_LBM_EINVAL;
    const int rc = sync_and_check(h);
    if (rc == II_LBM_EDEVICE) return rc;
    const int m = std::min(n, (int)h->prob.size());
    if (m > 0) {
        const hipError_t e = hipMemcpy(bits, h->P.err, (size_t)m * sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(h, e);
    }
    return rc;
}

int ii_lbm_set_graph(ii_lbm_handle* h, int32_t enable)
{
    if (!h || enable < 0 || enable > 256 || (enable > 1 && enable % 2 != 0)) return II_LBM_EINVAL;
    const int steps = enable <= 1 ? 64 : enable;
    if (steps != h->graph_steps) drop_graphs(h);
    h->graph_steps = steps;
    h->use_graph = enable != 0;
    if (!h->use_graph) {
        drop_graphs(h);
        return II_LBM_OK;
    }
    if (h->failed) return II_LBM_ESTATE;
    return hip_fail(h, ensure_graphs(h));
}

int ii_lbm_autotune(ii_lbm_handle* h, int32_t trials, int32_t* unit, int32_t* order, double* best_us)
{
    if (!h || trials < 1) return II_LBM_EINVAL;
    if (h->failed) return II_LBM_ESTATE;
    if (!h->batched) {
        if (unit) *unit = 0;
        if (order) *order = 0;
        if (best_us) *best_us = 0.0;
        return II_LBM_OK;
    }
    // The sweep is a pure function of the current lattice: time each
    // candidate on it writing the other buffer, which the next step rewrites.
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return hip_fail(h, hipErrorUnknown);
    const int units[3] = {128, 256, 512};
    double best = 1e300, alone[2][3] = {{0.0}};
    int bu = 256, bo = 1;
    hipError_t e = hipSuccess;
    for (int o = 0; o < 2 && e == hipSuccess; o++)
        for (int ui = 0; ui < 3 && e == hipSuccess; ui++) {
            e = upload_sweep_table(h, units[ui], o);
            void* A = h->P.lat[h->parity];
            void* B = h->P.lat[h->parity ^ 1];
            const int par = h->parity;
            if (e == hipSuccess) e = launch_sweep_batch(h->batch, h->P, A, B, par, h->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
            for (int t = 0; t < trials && e == hipSuccess; t++)
                e = launch_sweep_batch(h->batch, h->P, A, B, par, h->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const double us = 1e3 * ms / trials;
            alone[o][ui] = us;
            if (e == hipSuccess && us < best) {
                best = us;
                bu = units[ui];
                bo = o;
            }
        }
    if (e == hipSuccess) e = upload_sweep_table(h, bu, bo);
    // Membranes whose interface pass runs beside the sweep: the slice width
    // (in the chosen order) and the footprint of the tile pass together,
    // timed on whole steps, since the sweep's slices and the tile blocks share
    // the CUs (widths within a microsecond of each other alone differ by a
    // tenth of a step beside the interface pass).  A step that starts again
    // from the same parity recomputes the same results (each phase reads one
    // plane and writes the other), so repeating it leaves the state as it was.
    double best_step = 0.0;
    if (e == hipSuccess && h->lookahead && h->overlap != II_LBM_OVERLAP_SERIAL) {
        const int cands[8] = {0, 24, 16, 12, 8, 4, 2, 1};
        int bc = 0, bw = bu;
        best_step = 1e300;
        for (int ui = 0; ui < 3 && e == hipSuccess; ui++) {
            e = upload_sweep_table(h, units[ui], bo);
            for (int ci = 0; ci < 8 && e == hipSuccess; ci++) {
                e = upload_tile_table(h, cands[ci]);
                if (e == hipSuccess) e = enqueue_step(h, h->parity, h->stream, false);
                if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
                for (int t = 0; t < trials && e == hipSuccess; t++)
                    e = enqueue_step(h, h->parity, h->stream, false);
                if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                const double us = 1e3 * ms / trials;
                if (e == hipSuccess && us < best_step) {
                    best_step = us;
                    bc = cands[ci];
                    bw = units[ui];
                }
            }
        }
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess) e = upload_sweep_table(h, bw, bo);
        if (e == hipSuccess) e = upload_tile_table(h, bc);
        bu = bw;
        best = alone[bo][bw == 128 ? 0 : bw == 256 ? 1 : 2];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(h, e);
    drop_graphs(h);
    h->tuned_us = best;
    h->tuned_step_us = best_step;
    if (unit) *unit = bu;
    if (order) *order = bo;
    if (best_us) *best_us = best;
    return II_LBM_OK;
}

int ii_lbm_set_tile_blocks(ii_lbm_handle* h, int32_t per_cu)
{
    if (!h || per_cu < 0 || per_cu > 64) return II_LBM_EINVAL;
    if (h->failed) return II_LBM_ESTATE;
    if (!h->batched) {
        // single instance: per_cu blocks per CU beside the sweep (0: one)
        h->tile_per_cu = per_cu;
        drop_graphs(h);
        size_tile_blocks(h);
        return II_LBM_OK;
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess && h->aux) e = hipStreamSynchronize(h->aux);
    if (e == hipSuccess) e = upload_tile_table(h, per_cu);
    return e == hipSuccess ? II_LBM_OK : hip_fail(h, e);
}

int ii_lbm_get_schedule(ii_lbm_handle* h, int32_t* unit, int32_t* order, int32_t* tile_per_cu,
                        double* step_us)
{
    if (!h) return II_LBM_EINVAL;
    if (unit) *unit = h->batched ? h->batch.sweep_unit : 0;
    if (order) *order = h->batched ? h->sweep_order : 0;
    if (tile_per_cu) *tile_per_cu = h->tile_per_cu;
    if (step_us) *step_us = h->tuned_step_us;
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
    hipError_t e = hipMemcpyAsync(h->P.X[h->parity] + I.mk_off, X,
                                  (size_t)I.n_markers * sizeof(double2), hipMemcpyHostToDevice,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = prime(h);
    return hip_fail(h, e);
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
    if (!on_device) (void)hipFree(dst);
    return hip_fail(h, e);
}

int ii_lbm_fields_noalloc(ii_lbm_handle* h, int32_t inst, uint32_t what, void* out, int32_t dtype)
{
    if (!h || !out || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    if (dtype != II_LBM_DT_F32 && dtype != II_LBM_DT_F64) return II_LBM_EINVAL;
    if (what == 0 || (what & ~31u)) return II_LBM_EINVAL;
    const InstDev& I = h->L.inst[inst];
    int planes = 0;
    for (int b = 0; b < 4; b++) planes += (what >> b) & 1;
    if (what & II_LBM_F_DISTRIB) planes += 9;
    const size_t bytes = (size_t)planes * I.nx * I.ny * (dtype == II_LBM_DT_F64 ? 8 : 4);
    if (bytes > kScratchBytes) return II_LBM_ECAPACITY;
    if (!h->scratch) return II_LBM_EDEVICE;
    const int rc = sync_and_check(h);
    if (rc) return rc;
    hipError_t e = launch_fields(I, h->P.lat[h->parity], what, h->scratch, dtype, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, h->scratch, bytes, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
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
    (void)hipFree(d);
    return hip_fail(h, e);
}

int ii_lbm_state_size(ii_lbm_handle* h, int32_t inst, size_t* bytes)
{
    if (!h || !bytes || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    const InstDev& I = h->L.inst[inst];
    *bytes = sizeof(int64_t) + (size_t)I.n_markers * sizeof(double2) +
             (size_t)9 * I.plane * storage_bytes(I.storage) + (I.moving ? sizeof(BodyDev) : 0);
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
    b += (size_t)9 * I.plane * eb;
    if (e == hipSuccess && I.moving)
        e = hipMemcpy(b, h->P.body + I.inst, sizeof(BodyDev), hipMemcpyDeviceToHost);
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
    b += (size_t)9 * I.plane * eb;
    if (e == hipSuccess && I.moving)
        e = hipMemcpy(h->P.body + I.inst, b, sizeof(BodyDev), hipMemcpyHostToDevice);
    h->rec_valid = false;
    if (e == hipSuccess) e = prime(h);
    return hip_fail(h, e);
}

int ii_lbm_body(ii_lbm_handle* h, int32_t inst, double* out)
{
    if (!h || !out || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    const InstDev& I = h->L.inst[inst];
    if (!I.moving) return II_LBM_EINVAL;
    const int rc = sync_and_check(h);
    if (rc) return rc;
    BodyDev b;
    const hipError_t e = hipMemcpy(&b, h->P.body + I.inst, sizeof b, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e);
    const double v[14] = {b.c[0], b.c[1], b.U[0], b.U[1], b.theta, b.W, b.F[0], b.F[1],
                          b.T, b.a[0], b.a[1], b.wdot, (double)b.n, 0.0};
    memcpy(out, v, sizeof v);
    return II_LBM_OK;
}

int ii_lbm_cutlinks(ii_lbm_handle* h, int32_t inst, ii_lbm_link* out, int32_t cap, int32_t* count)
{
    if (!h || !count || cap < 0 || inst < 0 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    int rc = sync_and_check(h);
    if (rc) return rc;
    if ((rc = ensure_records(h))) return rc;
    const InstDev& I = h->L.inst[inst];
    int n = 0;
    hipError_t e = hipSuccess;
    const int par = record_parity(h);
    if (par >= 0) e = hipMemcpy(&n, h->P.rec_count + 2 * inst + par, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(h, e);
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
    (void)hipMemcpy(&errbits, h->P.err + inst, sizeof(int), hipMemcpyDeviceToHost);
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
        if (!h->isolate) h->failed = II_LBM_EUNSTABLE;
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
        const bool have_g = h->lookahead || h->rec_valid;
        out->force[0] = have_g ? fx : 0.0;
        out->force[1] = have_g ? fy : 0.0;
        // a failed membrane handle reports no links unless its records are current
        int n = 0;
        const bool current =
            !h->lookahead || h->rec_fresh || (!h->failed && ensure_records(h) == II_LBM_OK);
        const int par = record_parity(h);
        if (current && par >= 0)
            (void)hipMemcpy(&n, h->P.rec_count + 2 * inst + par, sizeof(int), hipMemcpyDeviceToHost);
        out->n_cut_links = n;
        // pressure on either side, 3 lu away from the polygon
        const int nb = std::min(I.ny, kDiagBlocks);
        double* pp = h->P.diag + 4 * kDiagBlocks;
        e = launch_pjump(I, h->P.lat[h->parity], h->P.X[h->parity] + I.mk_off, 3.0, pp, nb, h->stream);
        std::vector<double> pj(4 * (size_t)nb);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pj.data(), pp, pj.size() * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(h, e);
        double q[4] = {0, 0, 0, 0};
        for (int b = 0; b < nb; b++)
            for (int c = 0; c < 4; c++) q[c] += pj[4 * b + c];
        out->n_in = (int64_t)q[1];
        out->n_out = (int64_t)q[3];
        out->p_in = q[1] > 0.0 ? q[0] / q[1] : NAN;
        out->p_out = q[3] > 0.0 ? q[2] / q[3] : NAN;
    } else {
        out->p_in = out->p_out = NAN;
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
    if (!h || !bytes || inst < -1 || inst >= (int)h->prob.size()) return II_LBM_EINVAL;
    double b = 0.0;
    for (int j = 0; j < (int)h->prob.size(); j++) {
        if (inst >= 0 && j != inst) continue;
        const InstDev& I = h->L.inst[j];
        b += 18.0 * storage_bytes(I.storage) * (double)I.nx * (double)I.ny;
    }
    *bytes = b;
    return II_LBM_OK;
}

int ii_lbm_destroy(ii_lbm_handle* h)
{
    if (!h) return II_LBM_EINVAL;
    (void)hipStreamSynchronize(h->stream);
    if (h->aux) (void)hipStreamSynchronize(h->aux);
    if (h->lrn) (void)hipStreamSynchronize(h->lrn);
    release(h);
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
