// Host-side sanitizer driver of the II-LBM library (test infrastructure):
// tests/test_sanitized.py builds the library's host code with
// AddressSanitizer and UndefinedBehaviorSanitizer and links this driver to it.
// It exercises every path that runs without a GPU: problem validation and
// workspace layout (ii_lbm_workspace_size, and ii_lbm_init on problems that
// fail validation), the D3Q19 mesh checks, the CNN size queries, the error
// strings, and the NULL-handle guards of every call.  One valid init with a
// library-allocated workspace fails at its first device call (no GPU) and
// must clean up without leaking.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "../include/ii_lbm.h"
#include "../include/ii_lbm3.h"
#include "../include/ii_learned.h"

static int failures = 0;

#define EXPECT(cond)                                                      \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond);   \
            failures++;                                                   \
        }                                                                 \
    } while (0)

static ii_lbm_problem membrane(int nx, int ny, int n)
{
    ii_lbm_problem p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.tau = 0.8;
    p.interface_kind = II_LBM_IF_MEMBRANE;
    p.n_markers = n;
    p.kappa = 0.05;
    p.dX = 2.0 * M_PI * sqrt(0.09 * nx * ny / 4.0 * 0.6667) / n;
    return p;
}

static std::vector<double> ellipse(double cx, double cy, double a, double b, int n, bool ccw = true)
{
    std::vector<double> X(2 * n);
    for (int k = 0; k < n; k++) {
        const double t = (ccw ? 1.0 : -1.0) * 2.0 * M_PI * k / n;
        X[2 * k] = cx + a * cos(t);
        X[2 * k + 1] = cy + b * sin(t);
    }
    return X;
}

int main()
{
    size_t bytes = 0;
    // workspace layouts of valid problems
    ii_lbm_problem m = membrane(64, 64, 96);
    EXPECT(ii_lbm_workspace_size(&m, 1, &bytes) == II_LBM_OK && bytes > 2 * 9 * 64 * 64 * 4);
    ii_lbm_problem batch[3] = {membrane(64, 64, 96), membrane(96, 160, 300), membrane(512, 256, 900)};
    batch[2].storage = II_LBM_FP16;
    EXPECT(ii_lbm_workspace_size(batch, 3, &bytes) == II_LBM_OK);
    ii_lbm_problem big;
    memset(&big, 0, sizeof big);
    big.nx = big.ny = 8192;
    big.tau = 0.6;
    EXPECT(ii_lbm_workspace_size(&big, 1, &bytes) == II_LBM_OK && bytes > (size_t)2 * 9 * 8192 * 8192 * 4);
    ii_lbm_problem cyl;
    memset(&cyl, 0, sizeof cyl);
    cyl.nx = 1024;
    cyl.ny = 512;
    cyl.tau = 0.66;
    cyl.collision = II_LBM_MRT;
    cyl.bc[0] = II_LBM_BC_INLET;
    cyl.bc[1] = II_LBM_BC_OUTLET;
    cyl.bc[2] = cyl.bc[3] = II_LBM_BC_WALL;
    cyl.u_max = 0.05;
    cyl.interface_kind = II_LBM_IF_RIGID;
    cyl.n_markers = 101;
    cyl.dX = M_PI * 32 / 101;
    cyl.center[0] = 256;
    cyl.center[1] = 256;
    cyl.radius = 16;
    EXPECT(ii_lbm_workspace_size(&cyl, 1, &bytes) == II_LBM_OK);
    ii_lbm_problem spl = membrane(64, 64, 96);
    spl.geometry = 1;
    spl.force_mode = II_LBM_FORCE_IB_GUO;
    EXPECT(ii_lbm_workspace_size(&spl, 1, &bytes) == II_LBM_OK);
    EXPECT(ii_lbm_workspace_size(nullptr, 1, &bytes) == II_LBM_EINVAL);
    EXPECT(ii_lbm_workspace_size(&m, 0, &bytes) == II_LBM_EINVAL);

    // init: every invalid problem is refused before any device work
    std::vector<double> X = ellipse(32, 32, 12, 8, 96);
    const double* X0[1] = {X.data()};
    ii_lbm_handle* h = nullptr;
    struct Case {
        void (*edit)(ii_lbm_problem&);
        int want;
    };
    const Case cases[] = {
        {[](ii_lbm_problem& p) { p.nx = 8193; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.ny = 7; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.tau = 0.5; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.tau = NAN; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.collision = 2; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.bc[0] = II_LBM_BC_WALL; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.bc[0] = p.bc[1] = p.bc[2] = p.bc[3] = II_LBM_BC_WALL; p.bc[3] = II_LBM_BC_INLET; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.bc[0] = 9; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.storage = 3; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.math = 5; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.force_mode = 4; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.interface_kind = 7; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.n_markers = 2; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.dX = 2.5; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.kappa = -1.0; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.geometry = 2; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.body_free = 1; }, II_LBM_EINVAL},
        {[](ii_lbm_problem& p) { p.nx = 40; }, II_LBM_EGEOMETRY},   // markers beyond x = 36
    };
    for (const Case& c : cases) {
        ii_lbm_problem p = m;
        c.edit(p);
        EXPECT(ii_lbm_init(&p, 1, X0, nullptr, 0, nullptr, &h) == c.want && h == nullptr);
    }
    std::vector<double> cw = ellipse(32, 32, 12, 8, 96, false);
    const double* Xcw[1] = {cw.data()};
    EXPECT(ii_lbm_init(&m, 1, Xcw, nullptr, 0, nullptr, &h) == II_LBM_EGEOMETRY);
    std::vector<double> sparse = ellipse(32, 32, 12, 8, 12);   // chords over 4 lu
    const double* Xsp[1] = {sparse.data()};
    ii_lbm_problem m12 = m;
    m12.n_markers = 12;
    m12.dX = 1.9;
    EXPECT(ii_lbm_init(&m12, 1, Xsp, nullptr, 0, nullptr, &h) == II_LBM_EGEOMETRY);
    std::vector<double> bad = X;
    bad[10] = NAN;
    const double* Xnan[1] = {bad.data()};
    EXPECT(ii_lbm_init(&m, 1, Xnan, nullptr, 0, nullptr, &h) == II_LBM_EINVAL);
    EXPECT(ii_lbm_init(&m, 1, nullptr, nullptr, 0, nullptr, &h) == II_LBM_EINVAL);
    // a valid problem with a library workspace: without a GPU the first
    // device call fails and the handle is released
    const int rc = ii_lbm_init(&m, 1, X0, nullptr, 0, nullptr, &h);
    EXPECT(rc == II_LBM_EDEVICE || rc == II_LBM_OK);
    if (rc == II_LBM_OK) ii_lbm_destroy(h);

    // NULL-handle guards
    double d2[2];
    int32_t i1 = 0;
    int64_t l1 = 0;
    ii_lbm_diag_t dg;
    EXPECT(ii_lbm_step(nullptr, 1) == II_LBM_EINVAL);
    EXPECT(ii_lbm_sync(nullptr) == II_LBM_EINVAL);
    EXPECT(ii_lbm_markers(nullptr, 0, d2, nullptr, nullptr) == II_LBM_EINVAL);
    EXPECT(ii_lbm_fields(nullptr, 0, II_LBM_F_RHO, d2, II_LBM_DT_F64, 0) == II_LBM_EINVAL);
    EXPECT(ii_lbm_fields_noalloc(nullptr, 0, II_LBM_F_RHO, d2, II_LBM_DT_F64) == II_LBM_EINVAL);
    EXPECT(ii_lbm_diag(nullptr, 0, &dg) == II_LBM_EINVAL);
    EXPECT(ii_lbm_cutlinks(nullptr, 0, nullptr, 0, &i1) == II_LBM_EINVAL);
    EXPECT(ii_lbm_get_timing(nullptr, d2, &l1) == II_LBM_EINVAL);
    EXPECT(ii_lbm_set_graph(nullptr, 1) == II_LBM_EINVAL);
    EXPECT(ii_lbm_autotune(nullptr, 1, nullptr, nullptr, nullptr) == II_LBM_EINVAL);
    EXPECT(ii_lbm_set_tile_blocks(nullptr, 4) == II_LBM_EINVAL);
    EXPECT(ii_lbm_get_schedule(nullptr, nullptr, nullptr, nullptr, nullptr) == II_LBM_EINVAL);
    EXPECT(ii_lbm_destroy(nullptr) == II_LBM_EINVAL);
    for (int code = 1; code >= -8; code--) EXPECT(ii_lbm_strerror(code) != nullptr);

    // CNN sizes
    EXPECT(ii_cnn_packed_bytes() > 0 && ii_cnn_save_bytes() > 0 && ii_cnn_work_bytes(64) > 0);

    // D3Q19: the host-only mesh check on a tetrahedron-free closed octahedron
    ii_lbm3_problem p3;
    memset(&p3, 0, sizeof p3);
    p3.nx = p3.ny = p3.nz = 16;
    p3.tau = 0.8;
    const double oct[18] = {10, 8, 8, 6, 8, 8, 8, 10, 8, 8, 6, 8, 8, 8, 10, 8, 8, 6};
    const int32_t tri[24] = {0, 2, 4, 2, 1, 4, 1, 3, 4, 3, 0, 4, 2, 0, 5, 1, 2, 5, 3, 1, 5, 0, 3, 5};
    EXPECT(ii_lbm3_check_mesh(&p3, 6, oct, 8, tri) == II_LBM_OK);
    int32_t flipped[24];
    memcpy(flipped, tri, sizeof tri);
    std::swap(flipped[0], flipped[1]);
    EXPECT(ii_lbm3_check_mesh(&p3, 6, oct, 8, flipped) == II_LBM_EGEOMETRY);
    int32_t oob[24];
    memcpy(oob, tri, sizeof tri);
    oob[5] = 6;
    EXPECT(ii_lbm3_check_mesh(&p3, 6, oct, 8, oob) == II_LBM_EINVAL);
    ii_lbm3_handle* h3 = nullptr;
    ii_lbm3_problem bad3 = p3;
    bad3.nx = 4;
    EXPECT(ii_lbm3_init(&bad3, nullptr, nullptr, &h3) == II_LBM_EINVAL && h3 == nullptr);
    ii_lbm3_allocator half = {nullptr, nullptr, nullptr};
    EXPECT(ii_lbm3_init_with(&p3, nullptr, nullptr, &half, &h3) == II_LBM_EINVAL && h3 == nullptr);
    EXPECT(ii_lbm3_init_with(&bad3, nullptr, nullptr, nullptr, &h3) == II_LBM_EINVAL && h3 == nullptr);

    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("sanitize-host-check ok\n");
    return 0;
}
