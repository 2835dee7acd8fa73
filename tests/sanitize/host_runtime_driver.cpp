// Sanitizer driver for the library's host runtime (paper_2504_20169_amd/csrc/lbm_capi.hip):
// built with AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
// (tests/test_sanitizers.py), it drives every entry point that runs without a device --
// descriptor validation, the setters, the geometry and tile classification behind lbm_grid,
// lbm_footprint and lbm_node_classes over a sweep of sizes, PML widths, side masks, boundary
// kinds, stencils, storages and layouts, the launch settings, the error paths, and the check
// that rejects device buffers that overlap -- so an out-of-bounds access, a use after free, a
// leak or undefined arithmetic in that code ends the run with a report.  Also checks the
// documented invariants of the node classes.  Exit status 0 when every call behaved as
// documented.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lbm.h"

static int failures = 0;

#define EXPECT(cond, what)                                                           \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "FAIL line %d: %s (%s)\n", __LINE__, what, lbm_last_error()); \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

static lbm_desc make_desc(int nx, int ny, int storage, int lattice, int layout, int row_pad) {
    lbm_desc d;
    std::memset(&d, 0, sizeof d);
    d.nx = nx; d.ny = ny; d.tau = 0.8;
    d.rho0 = 1.0; d.ux0 = 0.05; d.uy0 = 0.0; d.T0 = 1.0;
    d.storage = storage; d.lattice = lattice; d.layout = layout; d.row_pad = row_pad;
    return d;
}

// An allocator that hands out the same host block every time: every buffer aliases.
struct Aliasing {
    std::vector<unsigned char> block = std::vector<unsigned char>(64 << 20);
    int allocs = 0, frees = 0;
};
static void *alias_alloc(size_t bytes, void *ctx) {
    Aliasing *a = (Aliasing *)ctx;
    if (bytes > a->block.size()) return nullptr;
    ++a->allocs;
    return a->block.data();
}
static void alias_free(void *, void *ctx) { ++((Aliasing *)ctx)->frees; }

int main() {
    // stencils
    for (int q : {37, 17, 9}) {
        std::vector<int32_t> e(2 * q);
        std::vector<double> w(q);
        double r = 0;
        EXPECT(lbm_velocities(q, e.data(), w.data(), &r) == LBM_OK, "velocities");
        double sw = 0;
        for (double v : w) sw += v;
        EXPECT(sw > 0.999999 && sw < 1.000001 && r > 1.0, "weights sum to one");
    }
    EXPECT(lbm_velocities(5, nullptr, nullptr, nullptr) == LBM_ERR_ARG, "unknown stencil");

    // geometry sweep
    long configs = 0;
    const int sizes[][2] = {{1, 1}, {3, 3}, {7, 5}, {9, 13}, {40, 33}, {130, 70}, {257, 64}};
    const int widths[] = {0, 1, 2, 3, 6, 17};
    for (auto &sz : sizes)
        for (int W : widths)
            for (unsigned mask = 0; mask < 16; mask += (W ? 1 : 16))
                for (int bcx = 0; bcx < 4; ++bcx)
                    for (int bcy = 0; bcy < 4; ++bcy)
                        for (int q : {37, 17, 9})
                            for (int storage = 0; storage < 3; ++storage)
                                for (int layout = 0; layout < 2; ++layout) {
                                    if (q != 37 && (storage != 0 || layout != 0)) continue;
                                    lbm_desc d = make_desc(sz[0], sz[1], storage, q, layout,
                                                           layout ? 0 : (bcx == 2 ? -1 : 0));
                                    lbm_handle h = nullptr;
                                    EXPECT(lbm_create(&d, &h) == LBM_OK && h, "create");
                                    if (!h) continue;
                                    EXPECT(lbm_set_bc(h, LBM_XMIN | LBM_XMAX, (lbm_bc)bcx) == LBM_OK, "bc x");
                                    EXPECT(lbm_set_bc(h, LBM_YMIN | LBM_YMAX, (lbm_bc)bcy) == LBM_OK, "bc y");
                                    EXPECT(lbm_set_pml(h, mask, W, 0.05) == LBM_OK, "pml");
                                    EXPECT(lbm_set_nrbc_pml_terms(h, (unsigned)(bcx & 7)) == LBM_OK, "terms");
                                    EXPECT(lbm_set_debug(h, (unsigned)(bcy & 1)) == LBM_OK, "debug");
                                    int32_t Nx = 0, Ny = 0;
                                    EXPECT(lbm_grid(h, &Nx, &Ny) == LBM_OK, "grid");
                                    int64_t cls[4] = {-1, -1, -1, -1};
                                    size_t fp = 0;
                                    lbm_status s1 = lbm_node_classes(h, cls);
                                    lbm_status s2 = lbm_footprint(h, &fp);
                                    EXPECT(s1 == s2, "classes and footprint agree on validity");
                                    if (s1 == LBM_OK) {
                                        EXPECT(cls[0] >= 0 && cls[1] >= 0 && cls[2] >= 0 && cls[3] >= 0, "counts");
                                        EXPECT(cls[0] + cls[1] == (int64_t)Nx * Ny, "bulk + frame = grid");
                                        EXPECT(cls[3] <= cls[1], "ring inside the frame");
                                        EXPECT(cls[2] <= (int64_t)Nx * Ny, "Q region inside the grid");
                                        EXPECT(fp > 2 * (size_t)Nx * Ny, "footprint holds two buffers");
                                    } else {
                                        EXPECT(s1 == LBM_ERR_ARG, "invalid geometry is an argument error");
                                    }
                                    lbm_launch L = {128, 2, 16, 1};
                                    EXPECT(lbm_set_launch(h, &L) == LBM_OK, "set launch");
                                    lbm_launch G{};
                                    EXPECT(lbm_get_launch(h, &G) == LBM_OK && G.bulk_tx == 128 &&
                                               G.graph_steps == 16, "get launch");
                                    lbm_destroy(h);
                                    ++configs;
                                }

    // descriptor and setter validation
    lbm_handle h = nullptr;
    lbm_desc d = make_desc(16, 16, 0, 37, 0, 0);
    EXPECT(lbm_create(nullptr, &h) == LBM_ERR_ARG, "NULL descriptor");
    d.tau = 0.5;
    EXPECT(lbm_create(&d, &h) == LBM_ERR_ARG && !h, "tau 0.5");
    d = make_desc(0, 16, 0, 37, 0, 0);
    EXPECT(lbm_create(&d, &h) == LBM_ERR_ARG, "zero size");
    d = make_desc(16, 16, 7, 37, 0, 0);
    EXPECT(lbm_create(&d, &h) == LBM_ERR_ARG, "unknown storage");
    d = make_desc(16, 16, 0, 11, 0, 0);
    EXPECT(lbm_create(&d, &h) == LBM_ERR_ARG, "unknown stencil");
    d = make_desc(16, 16, 0, 37, 0, 5000);
    EXPECT(lbm_create(&d, &h) == LBM_ERR_ARG, "row_pad out of range");
    d = make_desc(16, 16, 2, 37, 0, 0);
    d.f16_scale = 3.0;
    EXPECT(lbm_create(&d, &h) == LBM_ERR_ARG, "f16 scale not a power of two");
    d = make_desc(16, 16, 0, 37, 0, 0);
    d.T0 = -1.0;
    EXPECT(lbm_create(&d, &h) == LBM_ERR_ARG, "T0 <= 0");
    d = make_desc(16, 16, 0, 37, 0, 0);
    EXPECT(lbm_create(&d, &h) == LBM_OK, "create");
    EXPECT(lbm_set_bc(h, 16, LBM_BC_ZG) == LBM_ERR_ARG, "bad side mask");
    EXPECT(lbm_set_bc(h, 1, (lbm_bc)9) == LBM_ERR_ARG, "unknown boundary");
    EXPECT(lbm_set_pml(h, 15, -2, 0.1) == LBM_ERR_ARG, "negative W");
    EXPECT(lbm_set_nrbc_pml_terms(h, 8) == LBM_ERR_ARG, "unknown term");
    EXPECT(lbm_set_debug(h, LBM_DEBUG_POISON | LBM_DEBUG_RANGES) == LBM_OK, "debug flags");
    EXPECT(lbm_set_debug(h, 4) == LBM_ERR_ARG, "unknown debug flag");
    EXPECT(lbm_set_debug(h, 0) == LBM_OK, "debug flags cleared");
    EXPECT(lbm_set_check_interval(h, -1) == LBM_ERR_ARG, "negative check interval");
    EXPECT(lbm_set_check_interval(h, 64) == LBM_OK, "check interval");
    EXPECT(lbm_set_check_interval(h, 0) == LBM_OK, "check interval off");
    lbm_launch bad = {96, 2, 32, 0};
    EXPECT(lbm_set_launch(h, &bad) == LBM_ERR_ARG, "bad tile width");
    bad = {64, 4, 3, 0};
    EXPECT(lbm_set_launch(h, &bad) == LBM_ERR_ARG, "odd graph steps");
    EXPECT(lbm_step(h, 1) == LBM_ERR_STATE, "step before init");
    EXPECT(lbm_set_bc(h, LBM_XMIN, LBM_BC_ZG) == LBM_OK, "one side open");
    int64_t cls[4];
    EXPECT(lbm_node_classes(h, cls) == LBM_ERR_ARG, "periodic on one side only");
    std::vector<double> F(4 * 16 * 16, 1.0);
    EXPECT(lbm_init_fields(h, F.data(), F.data(), F.data(), F.data()) == LBM_ERR_ARG,
           "init with an inconsistent configuration");
    lbm_destroy(h);
    lbm_destroy(nullptr);

    // buffers that overlap are refused before any device work (a stream is supplied, so the
    // call makes no device call before the check)
    Aliasing alias;
    lbm_allocator A = {alias_alloc, alias_free, &alias};
    d = make_desc(20, 20, 0, 37, 0, 0);
    d.allocator = &A;
    d.stream = (void *)&alias;   // never used: the check fails first
    h = nullptr;
    EXPECT(lbm_create(&d, &h) == LBM_OK, "create with allocator");
    EXPECT(lbm_set_bc(h, LBM_ALL, LBM_BC_NRBC) == LBM_OK, "bc");
    EXPECT(lbm_set_pml(h, LBM_ALL, 4, 0.05) == LBM_OK, "pml");
    std::vector<double> G(4 * 28 * 28, 1.0);
    lbm_status st = lbm_init_fields(h, G.data(), G.data(), G.data(), G.data());
    EXPECT(st == LBM_ERR_ARG && std::strstr(lbm_last_error(), "overlap"), "aliasing buffers refused");
    EXPECT(alias.allocs > 1 && alias.allocs == alias.frees, "every buffer returned to the allocator");
    lbm_destroy(h);

    std::printf("host runtime: %ld configurations, %d failures\n", configs, failures);
    return failures ? 1 : 0;
}
