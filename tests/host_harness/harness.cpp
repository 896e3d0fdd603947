// harness.cpp -- the C-ABI layer's host logic on the CPU, built with
// AddressSanitizer and UndefinedBehaviorSanitizer against the HIP stand-in
// (hip_stub.cpp) and the oracle (oracle.c).  Sweep kernels are replaced by
// launchers that add the pass's step count to the time level each buffer
// carries in its first 8 bytes, so a run's buffer choreography (ping-pong
// order, remainder pass, aliasing, in-place passes, graph replay) is checked
// by reading the level of the output.  Usage: harness <scenario> [args];
// prints one line per check and exits nonzero on the first failure.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/stencil.h"
#include "../../paper_2103_08825_amd/csrc/launch.hpp"
#include "../../paper_2103_08825_amd/csrc/registry.hpp"
#include "hip_stub.h"

extern "C" int oracle_run(int dim, const int64_t *shape, int r, int kind, const double *coef, int bc,
                          int64_t T, const double *u0, double *uT, int nthreads, double *seconds);
extern "C" int oracle_adjoint(int dim, const int64_t *shape, int r, int kind, const double *coef, int bc,
                              int64_t T, int64_t ckpt, const double *u0, const double *gT, double *grad_u0,
                              double *grad_c, int nthreads);

#define CHECK(cond, ...)                                                    \
    do {                                                                    \
        if (!(cond)) {                                                      \
            printf("FAIL %s:%d: %s -- ", __FILE__, __LINE__, #cond);        \
            printf(__VA_ARGS__);                                            \
            printf(" [%s]\n", stencil_last_error());                        \
            exit(1);                                                        \
        }                                                                   \
    } while (0)

static int64_t level_of(const void *p) { return *static_cast<const int64_t *>(p); }
static void set_level(void *p, int64_t v) { *static_cast<int64_t *>(p) = v; }

// launch log and the cost model the autotuner sees (ms per launch)
struct Launch {
    const void *src;
    void *dst;
    int k, mode;
};
static std::vector<Launch> g_log;
static int g_best_variant = 3, g_best_k = 4;

template <int V, int K, int MODE>
static hipError_t stub_sweep(const stn::SweepLaunch &L, hipStream_t st) {
    if (MODE == 2 ? L.src != L.dst : L.src == L.dst) return hipErrorInvalidValue;
    if (MODE == 2 && !L.aux) return hipErrorInvalidValue;
    const void *src = L.src;
    void *dst = L.dst;
    g_log.push_back({src, dst, K, MODE});
    const double cost = K * (1.0 + 0.1 * (V != g_best_variant) + 0.05 * (K != g_best_k));
    stub_enqueue(st, [=] {
        set_level(dst, level_of(src) + K);
        g_stub.clock_ms += cost;
    });
    return hipSuccess;
}

template <int V, int K> static void reg_one() {
    stn::register_launcher(stn::KernelKey{stn::kF32, 3, 1, 0, V, K, 0}, &stub_sweep<V, K, 0>);
    stn::register_launcher(stn::KernelKey{stn::kF32, 3, 1, 0, V, K, 2}, &stub_sweep<V, K, 2>);
}
template <int V> static void reg_variant() {
    reg_one<V, 1>();
    reg_one<V, 2>();
    reg_one<V, 3>();
    reg_one<V, 4>();
    reg_one<V, 5>();
    reg_one<V, 6>();
}

namespace stn {
hipError_t launch_generic(int, const void *src, void *dst, int64_t, int64_t, int64_t, int, int, const int *, const void *,
                          hipStream_t st) {
    g_log.push_back({src, dst, 1, 9});
    stub_enqueue(st, [=] { set_level(dst, level_of(src) + 1); });
    return hipSuccess;
}
hipError_t launch_reduce(int, const void *, const void *, int64_t, double *, double *out, hipStream_t) {
    for (int i = 0; i < 6; ++i) out[i] = 0.0;
    return hipSuccess;
}
int reduce_partials_bytes() { return 2048 * 6 * 8; }
}  // namespace stn

static stencil_plan *make_plan(const int64_t *shape, stencil_opts o, int *rc_out = nullptr) {
    double c[7] = {0.1, 0.1, 0.1, 0.4, 0.1, 0.1, 0.1};
    stencil_plan *p = nullptr;
    const int rc = stencil_plan_create(&p, 3, shape, 1, STENCIL_STAR, c, 7, STENCIL_BC_ZERO, STENCIL_F32, &o);
    if (rc_out) *rc_out = rc;
    return p;
}

static const int64_t kShape[3] = {40, 64, 64};

static void scenario_validation() {
    double c[7] = {0};
    stencil_plan *p = (stencil_plan *)1;
    int64_t sh[3] = {8, 8, 8};
    CHECK(stencil_plan_create(nullptr, 3, sh, 1, 0, c, 7, 0, 1, nullptr) == STENCIL_E_INVALID, "NULL out");
    CHECK(stencil_plan_create(&p, 4, sh, 1, 0, c, 7, 0, 1, nullptr) == STENCIL_E_INVALID && !p, "dim 4");
    CHECK(stencil_plan_create(&p, 3, sh, 0, 0, c, 7, 0, 1, nullptr) == STENCIL_E_INVALID, "radius 0");
    CHECK(stencil_plan_create(&p, 3, sh, 5, 0, c, 31, 0, 1, nullptr) == STENCIL_E_UNSUPPORTED, "radius 5");
    CHECK(stencil_plan_create(&p, 3, sh, 1, 0, c, 6, 0, 1, nullptr) == STENCIL_E_INVALID, "ncoeffs");
    CHECK(stencil_plan_create(&p, 3, sh, 1, 2, c, 7, 0, 1, nullptr) == STENCIL_E_INVALID, "kind");
    CHECK(stencil_plan_create(&p, 3, sh, 1, 0, c, 7, 2, 1, nullptr) == STENCIL_E_INVALID, "bc");
    CHECK(stencil_plan_create(&p, 3, sh, 1, 0, c, 7, 0, 7, nullptr) == STENCIL_E_INVALID, "dtype");
    CHECK(stencil_plan_create(&p, 3, sh, 1, 0, nullptr, 7, 0, 1, nullptr) == STENCIL_E_INVALID, "coeffs NULL");
    CHECK(stencil_plan_create(&p, 3, nullptr, 1, 0, c, 7, 0, 1, nullptr) == STENCIL_E_INVALID, "shape NULL");
    int64_t bad[3] = {8, 0, 8};
    CHECK(stencil_plan_create(&p, 3, bad, 1, 0, c, 7, 0, 1, nullptr) == STENCIL_E_INVALID, "extent 0");
    int64_t huge[3] = {(int64_t)1 << 30, (int64_t)1 << 30, 8};
    CHECK(stencil_plan_create(&p, 3, huge, 1, 0, c, 7, 0, 1, nullptr) == STENCIL_E_INVALID, "too large");
    stencil_opts o{};
    o.method = 5;
    CHECK(stencil_plan_create(&p, 3, sh, 1, 0, c, 7, 0, 1, &o) == STENCIL_E_INVALID, "method 5");
    o = stencil_opts{};
    o.fused_k = -1;
    CHECK(stencil_plan_create(&p, 3, sh, 1, 0, c, 7, 0, 1, &o) == STENCIL_E_INVALID, "fused_k -1");
    o = stencil_opts{};
    o.chunk = -2;
    CHECK(stencil_plan_create(&p, 3, sh, 1, 0, c, 7, 0, 1, &o) == STENCIL_E_INVALID, "chunk -2");
    o = stencil_opts{};
    o.method = STENCIL_METHOD_FUSED;
    o.fused_k = 9;
    CHECK(stencil_plan_create(&p, 3, sh, 1, 0, c, 7, 0, 1, &o) == STENCIL_E_UNSUPPORTED, "k beyond compiled");
    int32_t offs[3 * 27];
    CHECK(stencil_offsets(3, 1, STENCIL_BOX, offs) == 27 && offs[0] == -1 && offs[80] == 1, "offsets");
    CHECK(stencil_offsets(3, 1, STENCIL_BOX, nullptr) == STENCIL_E_INVALID, "offsets NULL");
    CHECK(stencil_num_points(2, 3, STENCIL_STAR) == 13, "npts");
    stencil_plan *q = make_plan(kShape, stencil_opts{});
    CHECK(q, "plan");
    float buf[4];
    CHECK(stencil_run(q, nullptr, buf, 1, nullptr) == STENCIL_E_INVALID, "run NULL in");
    CHECK(stencil_run(q, buf, buf, -1, nullptr) == STENCIL_E_INVALID, "run T<0");
    CHECK(stencil_run(nullptr, buf, buf, 1, nullptr) == STENCIL_E_INVALID, "run NULL plan");
    stencil_plan_desc d;
    CHECK(stencil_plan_info(q, nullptr) == STENCIL_E_INVALID, "info NULL");
    CHECK(stencil_plan_info(q, &d) == 0 && d.points == 40 * 64 * 64, "info");
    double out6[6];
    CHECK(stencil_reduce(9, buf, nullptr, 4, out6, nullptr) == STENCIL_E_INVALID, "reduce dtype");
    CHECK(stencil_reduce(1, buf, nullptr, -1, out6, nullptr) == STENCIL_E_INVALID, "reduce n");
    stencil_plan_destroy(q);
    stencil_plan_destroy(nullptr);
    printf("PASS validation\n");
}

static std::vector<char> field(const stencil_plan *p) {
    stencil_plan_desc d;
    stencil_plan_info(p, &d);
    return std::vector<char>((size_t)d.points * d.elem_bytes, 0);
}

static void scenario_passes(bool inplace) {
    g_stub.mallocs.clear();
    stencil_opts o{};
    o.method = STENCIL_METHOD_FUSED;
    o.fused_k = 5;
    o.inplace = inplace;
    stencil_plan *p = make_plan(kShape, o);
    CHECK(p, "plan");
    std::vector<char> in = field(p), out = field(p);
    for (int64_t T = 0; T <= 13; ++T) {
        for (int alias = 0; alias < 2; ++alias) {
            g_log.clear();
            set_level(in.data(), 100);
            set_level(out.data(), -7);
            void *dst = alias ? (void *)in.data() : (void *)out.data();
            CHECK(stencil_run(p, in.data(), dst, T, nullptr) == 0, "run T=%lld", (long long)T);
            CHECK(level_of(dst) == 100 + T, "T=%lld alias=%d level %lld", (long long)T, alias, (long long)level_of(dst));
            if (!alias) CHECK(level_of(in.data()) == 100, "input changed");
            const int64_t passes = T / 5 + (T % 5 ? 1 : 0);
            int in_place = 0;
            for (const Launch &l : g_log) in_place += l.mode == 2;
            if (inplace)
                CHECK(in_place == (alias ? passes : (passes > 0 ? passes - 1 : 0)), "in-place passes %d", in_place);
            else
                CHECK(in_place == 0, "a ping-pong plan ran in place");
        }
    }
    stencil_plan_desc d;
    stencil_plan_info(p, &d);
    const int64_t fieldb = d.points * d.elem_bytes;
    if (inplace) {
        CHECK(d.scratch_bytes > 0 && d.scratch_bytes != fieldb, "in-place plan holds %lld bytes", (long long)d.scratch_bytes);
        for (size_t n : g_stub.mallocs) CHECK((int64_t)n != fieldb, "a ping-pong field was allocated");
    } else {
        CHECK(d.scratch_bytes == 2 * fieldb, "ping-pong plan with an aliased run holds two fields");
    }
    stencil_plan_destroy(p);
    printf("PASS passes inplace=%d\n", (int)inplace);
}

static void scenario_graph(bool capture_fails) {
    g_stub.capture_fails = capture_fails;
    stencil_opts o{};
    o.method = STENCIL_METHOD_FUSED;
    o.fused_k = 4;
    o.graph = 1;
    stencil_plan *p = make_plan(kShape, o);
    std::vector<char> in = field(p), out = field(p);
    const int before = g_stub.graph_launches;
    for (int rep = 0; rep < 3; ++rep) {
        set_level(in.data(), 10 * rep);
        set_level(out.data(), -1);
        CHECK(stencil_run(p, in.data(), out.data(), 11, nullptr) == 0, "graph run");
        CHECK(level_of(out.data()) == 10 * rep + 11, "replay %d level %lld", rep, (long long)level_of(out.data()));
    }
    const int replays = g_stub.graph_launches - before;
    CHECK(capture_fails ? replays == 0 : replays == 3, "graph launches %d", replays);
    stencil_plan_destroy(p);
    g_stub.capture_fails = false;
    printf("PASS graph capture_fails=%d\n", (int)capture_fails);
}

// the tuned choice is cached per signature, which includes the requested
// depth: a plan asking for k = 2 never receives another plan's k
static void scenario_tune(const char *phase) {
    stencil_opts o{};
    o.method = STENCIL_METHOD_FUSED;
    o.autotune = 1;
    stencil_plan *a = make_plan(kShape, o);
    o.fused_k = 2;
    stencil_plan *b = make_plan(kShape, o);
    stencil_plan_desc da, db;
    if (!strcmp(phase, "corrupt")) g_best_variant = 2;
    if (!strcmp(phase, "load")) {
        // a different cost model: a loaded entry keeps the first process's choice
        g_best_variant = 1;
        g_best_k = 3;
    }
    CHECK(stencil_autotune(a, nullptr) == 0 && stencil_autotune(b, nullptr) == 0, "autotune");
    stencil_plan_info(a, &da);
    stencil_plan_info(b, &db);
    CHECK(db.fused_k == 2 && db.tuned == 1, "constrained plan got k=%d", db.fused_k);
    if (!strcmp(phase, "write") || !strcmp(phase, "load"))
        CHECK(da.variant == 3 && da.fused_k == 4, "tuned (variant %d, k %d)", da.variant, da.fused_k);
    if (!strcmp(phase, "corrupt")) CHECK(da.variant == 2, "tuned variant %d after a corrupt cache", da.variant);
    stencil_plan_destroy(a);
    stencil_plan_destroy(b);
    printf("PASS tune %s\n", phase);
}

static void scenario_oracle() {
    // small grids of every dimension, order and rule: constant fields are kept
    // under the periodic rule with weights summing to 1
    for (int dim = 1; dim <= 3; ++dim)
        for (int r = 1; r <= 3; ++r)
            for (int bc = 0; bc < 2; ++bc) {
                int64_t shape[3] = {5, 4, 3};
                int n = 1;
                for (int i = 0; i < dim; ++i) n *= (int)shape[i];
                const int npts = 2 * dim * r + 1;
                std::vector<double> c(npts, 0.5 / (npts - 1)), u(n, 2.0), out(n), g(n, 1.0), gu(n), gc(npts);
                c[npts / 2] = 0.5;
                CHECK(oracle_run(dim, shape, r, 0, c.data(), bc, 3, u.data(), out.data(), 1, nullptr) == 0, "oracle_run");
                if (bc == 1)
                    for (double v : out) CHECK(v > 2.0 - 1e-14 && v < 2.0 + 1e-14, "periodic constant field %.17g", v);
                CHECK(oracle_adjoint(dim, shape, r, 0, c.data(), bc, 4, 3, u.data(), g.data(), gu.data(), gc.data(), 1) == 0,
                      "oracle_adjoint");
            }
    int64_t sh[1] = {4};
    double c3[3] = {0.25, 0.5, 0.25}, u[4] = {0}, o[4];
    CHECK(oracle_run(1, sh, 1, 0, c3, 0, -1, u, o, 1, nullptr) == -1, "oracle T<0");
    CHECK(oracle_run(4, sh, 1, 0, c3, 0, 1, u, o, 1, nullptr) == -1, "oracle dim 4");
    printf("PASS oracle\n");
}

int main(int argc, char **argv) {
    reg_variant<1>();
    reg_variant<2>();
    reg_variant<3>();
    reg_variant<4>();
    reg_variant<5>();
    reg_variant<6>();
    const std::string s = argc > 1 ? argv[1] : "all";
    if (s == "all" || s == "validation") scenario_validation();
    if (s == "all" || s == "passes") {
        scenario_passes(false);
        scenario_passes(true);
    }
    if (s == "all" || s == "graph") {
        scenario_graph(false);
        scenario_graph(true);
    }
    if (s == "tune") scenario_tune(argc > 2 ? argv[2] : "write");
    if (s == "all" || s == "oracle") scenario_oracle();
    return 0;
}
