// api.cpp -- the C ABI: plans, sweeps, autotuning, reductions, errors.
#include <hip/hip_runtime.h>

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "plan.hpp"
#include "registry.hpp"
#include "variants.hpp"

namespace stn {

static thread_local std::string t_err;

int fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

void clear_error() { t_err.clear(); }

int elem_bytes(int dtype) {
    switch (dtype) {
    case STENCIL_F64: return 8;
    case STENCIL_F32: return 4;
    case STENCIL_BF16:
    case STENCIL_F16: return 2;
    default: return 0;
    }
}

// Canonical order: odometer over [-r, r]^dim with the last axis turning
// fastest, keeping the members of the star or the box.
int enumerate_offsets(int dim, int r, int kind, int32_t *out) {
    int o[STENCIL_MAX_DIM];
    for (int i = 0; i < dim; ++i) o[i] = -r;
    int n = 0;
    for (;;) {
        int nonzero = 0;
        for (int i = 0; i < dim; ++i) nonzero += (o[i] != 0);
        if (kind == STENCIL_BOX || nonzero <= 1) {
            if (out)
                for (int i = 0; i < dim; ++i) out[n * dim + i] = o[i];
            ++n;
        }
        int ax = dim - 1;
        while (ax >= 0 && ++o[ax] > r) {
            o[ax] = -r;
            --ax;
        }
        if (ax < 0) break;
    }
    return n;
}

static bool shape_of(int dim, int variant, VariantShape *v) {
    const int nv = dim == 3 ? kNumV3 : (dim == 2 ? kNumV2 : kNumV1);
    if (variant < 1 || variant > nv) return false;
    *v = dim == 3 ? kV3[variant] : (dim == 2 ? kV2[variant] : kV1[variant]);
    return true;
}

static int box_key(const stencil_plan *p) { return p->dim == 1 ? 0 : (p->kind == STENCIL_BOX ? 1 : 0); }

static int max_k_of(const stencil_plan *p, int variant) {
    return registered_max_k(p->dtype, p->dim, p->r, box_key(p), variant);
}

static int num_variants_of(int dim) { return dim == 3 ? kNumV3 : (dim == 2 ? kNumV2 : kNumV1); }

// 2D/3D fused kernels address one plane with 32-bit byte offsets (below
// 2^31, the out-of-range marker) and need the x extent to be a multiple of
// the lane width; the streamed extent must fit an int.
static bool variant_fits_shape(const stencil_plan *p, int variant) {
    VariantShape v;
    if (!shape_of(p->dim, variant, &v)) return false;
    if (p->dim == 1) return true;
    const int64_t plane_bytes = p->n1 * p->n2 * elem_bytes(p->dtype);
    if (plane_bytes >= ((int64_t)1 << 31) || p->n0 >= ((int64_t)1 << 31)) return false;
    return v.vx == 1 || p->n2 % v.vx == 0;
}

static bool variant_fits_ptr(const stencil_plan *p, int variant, const void *a, const void *b) {
    VariantShape v;
    if (!shape_of(p->dim, variant, &v)) return false;
    const uintptr_t al = (uintptr_t)v.vx * elem_bytes(p->dtype);
    return v.vx == 1 || (((uintptr_t)a % al) == 0 && ((uintptr_t)b % al) == 0);
}

SweepLauncher pass_launcher(const stencil_plan *p, const Exec &ex, int k, bool in_place) {
    if (ex.method == STENCIL_METHOD_GENERIC) return nullptr;
    const int mode = ex.method == STENCIL_METHOD_TESSELLATE ? 1 : (in_place ? 2 : 0);
    return find_launcher(KernelKey{p->dtype, p->dim, p->r, box_key(p), ex.variant, k, mode});
}

static int inplace_max_k(const stencil_plan *p, int variant) {
    return registered_max_k(p->dtype, p->dim, p->r, box_key(p), variant, 2);
}

// side-buffer bytes of an in-place plan: the largest over the depths its passes use
static int64_t inplace_side_bytes(const stencil_plan *p, const Exec &ex) {
    VariantShape v;
    if (!shape_of(p->dim, ex.variant, &v)) return 0;
    int64_t best = 0;
    for (int k = 1; k <= ex.k; ++k) {
        const InplaceSide s = inplace_side(p->dim, p->r, k, v, p->n0, p->n1, p->n2, ex.chunk);
        if (s.ok) best = std::max(best, s.total * elem_bytes(p->dtype));
    }
    return best;
}

// chunk 0 ("automatic") of a fused 2D/3D launch: balanced over the workgroups
// the device holds at once.  Stays 0 (the geometry's own rule: many short
// chunks) for one step per launch, whose workgroups wait on memory rather than
// compute (measured: the balanced rule loses 7% there), and when the
// residency cannot be queried.
static int auto_chunk(const stencil_plan *p, int variant, int k) {
    VariantShape v;
    if (p->dim < 2 || k < 2 || !shape_of(p->dim, variant, &v)) return 0;
    const int resident = resident_blocks(KernelKey{p->dtype, p->dim, p->r, box_key(p), variant, k});
    return balanced_chunk(p->dim, p->r, k, v, p->n0, p->n1, p->n2, resident);
}

// default variant: widest lanes that fit the shape, else the first registered
static int default_variant(const stencil_plan *p, int need_k) {
    int best = 0;
    for (int v = 1; v <= num_variants_of(p->dim); ++v) {
        if (!variant_fits_shape(p, v) || max_k_of(p, v) < need_k) continue;
        VariantShape s;
        shape_of(p->dim, v, &s);
        if (best == 0) {
            best = v;
        } else {
            VariantShape b;
            shape_of(p->dim, best, &b);
            // 1D/2D prefer wide lanes; 3D keeps the first listed (tuned default)
            if (p->dim < 3 && s.vx > b.vx) best = v;
        }
    }
    return best;
}

// 1D: a halo of k*r = 32 points per side of a 256-point (4 per lane) segment
// (measured, FP64 3-point: 262,144 points T = 200, k = 16 993 -> k = 32 1429
// GStencil/s, launch-bound; 10,240,000 points T = 1000, 4506 -> 4757, k = 24
// 4892; 5-point, k = 8 2671 -> k = 16 2896).
static int default_k(const stencil_plan *p, int variant) {
    const int kmax = max_k_of(p, variant);
    const int want = p->dim == 3 ? 4 : (p->dim == 2 ? 8 : 32 / p->r);
    return std::min(want, kmax);
}

// Measured defaults (MI355X, 512^3 3D and 8192^2 2D grids; each the fastest
// (variant, k, chunk) of a sweep over all compiled choices; chunk 0 = balanced
// over the resident workgroups for the plan's shape).  stencil_autotune
// refines them for a given plan.  The 3D 7-point FP32 depth is k = 6 since the
// zero halo goes through the weights (sustained T = 64 sweeps, alternating
// choices on one GPU: k = 6 2168, k = 5 2103, k = 4 1780 GStencil/s); the 2D
// 5-point depth is k = 10 (8192^2 periodic, T = 100: k = 8 3583, k = 10 4128,
// k = 12 4065), the 9-point stays at k = 8 (k = 10 the same, 12 slower).
// The 13-point FP32 star takes 48-plane chunks (T = 64 sweeps, medians of 8:
// 40 832, 48 831, 56 813, 64 783, 32 815, balanced 803 GStencil/s); its 16-bit
// form keeps 64 (1006 against 917 at 48).
struct Choice {
    int dim, r, kind, dclass;  // dclass: 0 FP64, 1 FP32, 2 16-bit
    int variant, k, chunk;     // fused
    int pvariant, pchunk;      // plain (k = 1)
};
static const Choice kChoices[] = {
    // 3D FP32: 7-point, 27-point, 13-point
    {3, 1, STENCIL_STAR, 1, 5, 6, 0, 3, 8}, {3, 1, STENCIL_BOX, 1, 5, 3, 0, 5, 0},
    {3, 2, STENCIL_STAR, 1, 4, 2, 48, 5, 0},
    // 3D 16-bit storage
    {3, 1, STENCIL_STAR, 2, 5, 6, 0, 5, 0}, {3, 1, STENCIL_BOX, 2, 5, 3, 0, 4, 0},
    {3, 2, STENCIL_STAR, 2, 4, 2, 64, 1, 64},
    // 3D FP64
    {3, 1, STENCIL_STAR, 0, 4, 4, 0, 1, 32}, {3, 1, STENCIL_BOX, 0, 4, 3, 0, 1, 32},
    {3, 2, STENCIL_STAR, 0, 4, 2, 0, 4, 0},
    // 2D FP32: 5-point, 9-point
    {2, 1, STENCIL_STAR, 1, 2, 10, 0, 2, 64}, {2, 1, STENCIL_BOX, 1, 2, 8, 0, 2, 64},
};

static const Choice *measured_choice(const stencil_plan *p) {
    const int dclass = p->dtype == STENCIL_F64 ? 0 : (p->dtype == STENCIL_F32 ? 1 : 2);
    for (const Choice &c : kChoices)
        if (c.dim == p->dim && c.r == p->r && c.kind == p->kind && c.dclass == dclass) return &c;
    return nullptr;
}

// The measured one-step (k = 1) choices were made on 512^3 grids.  One-step
// launches wait on memory and want many waves in flight, so a 3D grid of fewer
// than kPlainSmallGrid points (half of 512^3) takes the smallest tile (1,4,8)
// instead.  A measured one-step chunk above 8 planes (the 7-point stencils'
// 32) drops to 8; a choice that leaves the chunk to the automatic rule keeps
// that rule's shortest chunk, 4(2r+1) planes at k = 1 (12 for the 27-point box,
// 20 for the 13-point star).  Measured so at 256^3 FP32: 7-point 38 -> 29 us per
// step, 27-point 70 -> 46 us, 13-point 53 -> 40 us; BF16 7-point 39 -> 32 us; at
// 384^3 FP32 7-point 128 -> 115 us; at 128^3 FP64 7-point, chunks of 32 -> 8
// planes: 77 -> 118 GStencil/s.
constexpr int64_t kPlainSmallGrid = (int64_t)1 << 26;

static void plain_choice(const stencil_plan *p, const Choice *mc, int *variant, int *chunk) {
    *variant = mc->pvariant;
    *chunk = mc->pchunk;
    if (p->dim != 3 || p->points >= kPlainSmallGrid) return;
    if (!variant_fits_shape(p, 1) || max_k_of(p, 1) < 1) return;
    *variant = 1;
    if (*chunk > 8) *chunk = 8;
}

// rows of the stage-A frame of a tessellated pass with this variant
static int tess_tile_rows(const stencil_plan *p, int variant) {
    VariantShape v;
    return shape_of(p->dim, variant, &v) ? v.nw * v.rw : 0;
}

static int tess_max_k(const stencil_plan *p, int variant) {
    return registered_max_k(p->dtype, p->dim, p->r, box_key(p), variant, 1);
}

// The tessellated method: the fused choice's variant and depth where a
// tessellated kernel exists for them, the y extent permitting.
static int resolve_tess(stencil_plan *p, const Choice *mc, Exec *out) {
    const stencil_opts &o = p->opts;
    if (p->dim != 3) return fail(STENCIL_E_UNSUPPORTED, "the tessellated sweep is built for 3D grids");
    int variant = o.variant;
    if (variant == 0) {
        if (mc && tess_max_k(p, mc->variant) > 0) variant = mc->variant;
        for (int v = 1; v <= num_variants_of(p->dim) && variant == 0; ++v)
            if (tess_max_k(p, v) > 0) variant = v;
    }
    const int kmax = variant > 0 ? tess_max_k(p, variant) : 0;
    if (kmax == 0 || !variant_fits_shape(p, variant))
        return fail(STENCIL_E_UNSUPPORTED, "no tessellated kernel is compiled for this stencil (%dD r=%d %s dtype %d)",
                    p->dim, p->r, p->kind == STENCIL_BOX ? "box" : "star", p->dtype);
    int k = o.fused_k;
    if (k == 0) k = std::min(kmax, (mc && mc->variant == variant) ? mc->k : default_k(p, variant));
    if (k > kmax) return fail(STENCIL_E_UNSUPPORTED, "fused_k=%d exceeds the compiled tessellated maximum %d", k, kmax);
    const int rows = tess_tile_rows(p, variant);
    if (!tess_tiling(p->r, k, rows, p->n1, p->bc).ok)
        return fail(STENCIL_E_UNSUPPORTED, "the tessellated sweep needs a y extent of at least %d rows (got %lld)",
                    2 * (k + 1) * p->r, (long long)p->n1);
    int chunk = o.chunk;
    if (chunk == 0 && mc && mc->variant == variant) chunk = mc->chunk;
    *out = Exec{STENCIL_METHOD_TESSELLATE, variant, k, chunk > 0 ? chunk : auto_chunk(p, variant, k)};
    return STENCIL_OK;
}

// Resolve the requested method into an execution choice.  Returns a status.
static int resolve_exec(stencil_plan *p) {
    const stencil_opts &o = p->opts;
    Exec ex{STENCIL_METHOD_GENERIC, 0, 1, 0};
    int method = o.method;
    if (method == STENCIL_METHOD_TESSELLATE) {
        if (o.inplace) return fail(STENCIL_E_UNSUPPORTED, "the tessellated method has no in-place form");
        return resolve_tess(p, measured_choice(p), &p->exec);
    }
    if (o.inplace && (method == STENCIL_METHOD_GENERIC || p->dim == 1))
        return fail(STENCIL_E_UNSUPPORTED, "in-place passes need the 2D/3D fused kernels");
    if (method == STENCIL_METHOD_AUTO) {
        method = default_variant(p, 1) ? STENCIL_METHOD_FUSED : STENCIL_METHOD_GENERIC;
    }
    if (method == STENCIL_METHOD_GENERIC) {
        p->exec = ex;
        return STENCIL_OK;
    }
    int variant = o.variant;
    if (variant != 0) {
        VariantShape v;
        if (!shape_of(p->dim, variant, &v))
            return fail(STENCIL_E_INVALID, "variant %d does not exist for %dD", variant, p->dim);
        if (!variant_fits_shape(p, variant))
            return fail(STENCIL_E_INVALID, "variant %d needs the last extent to be a multiple of %d",
                        variant, v.vx);
    } else {
        // a requested depth narrows the choice to variants compiled that deep
        const int need_k = method == STENCIL_METHOD_FUSED && o.fused_k > 0 ? o.fused_k : 1;
        variant = default_variant(p, need_k);
        if (variant == 0) variant = default_variant(p, 1);  // reported as too deep below
    }
    const Choice *mc = measured_choice(p);
    int chunk = o.chunk;
    if (mc && o.variant == 0) {
        int mv = mc->variant, mchunk = mc->chunk;
        if (method == STENCIL_METHOD_PLAIN) plain_choice(p, mc, &mv, &mchunk);
        const int need_k = method == STENCIL_METHOD_FUSED && o.fused_k > 0 ? o.fused_k : 1;
        if (variant_fits_shape(p, mv) && max_k_of(p, mv) >= need_k) {
            variant = mv;
            if (o.chunk == 0) chunk = mchunk;
        }
    }
    if (variant == 0 || max_k_of(p, variant) < 1) {
        if (o.method == STENCIL_METHOD_AUTO) {
            p->exec = ex;
            return STENCIL_OK;
        }
        return fail(STENCIL_E_UNSUPPORTED,
                    "no fused kernel is compiled for this stencil (%dD r=%d %s dtype %d)", p->dim, p->r,
                    p->kind == STENCIL_BOX ? "box" : "star", p->dtype);
    }
    int k = 1;
    if (method == STENCIL_METHOD_FUSED) {
        if (o.fused_k > 0) {
            if (o.fused_k > max_k_of(p, variant))
                return fail(STENCIL_E_UNSUPPORTED, "fused_k=%d exceeds the compiled maximum %d",
                            o.fused_k, max_k_of(p, variant));
            k = o.fused_k;
        } else {
            k = default_k(p, variant);
            if (mc && variant == mc->variant && mc->k <= max_k_of(p, variant)) k = mc->k;
            // The measured depths were chosen on 512^3 grids.  On a quarter of
            // that or less the balanced chunks get short, and the fill of a deep
            // pass (k(2r+1) planes per chunk) outweighs the saved passes, so the
            // order-1 stencils stop earlier there: FP32 and 16-bit stars at k = 4
            // (256^3 FP32, T = 10 per call: k = 6 1149, k = 5 1254, k = 4 1295
            // GStencil/s), FP64 stars at k = 3 and FP64 boxes at k = 2 (128^3,
            // T = 1000: 7-point 227 at k = 4, 242 at k = 3; 27-point 120 at
            // k = 3, 156 at k = 2).
            if (p->dim == 3 && p->r == 1 && p->points <= kPlainSmallGrid / 2) {
                const int cap = p->dtype != STENCIL_F64 ? (p->kind == STENCIL_STAR ? 4 : k)
                                                        : (p->kind == STENCIL_STAR ? 3 : 2);
                if (k > cap) k = cap;
            }
        }
    }
    ex.method = method;
    ex.variant = variant;
    ex.k = k;
    ex.chunk = chunk > 0 ? chunk : auto_chunk(p, variant, k);
    // a default depth beyond what the in-place pass compiles drops to its deepest
    if (o.inplace && o.fused_k == 0 && method == STENCIL_METHOD_FUSED && inplace_max_k(p, ex.variant) > 0 &&
        inplace_max_k(p, ex.variant) < ex.k) {
        ex.k = inplace_max_k(p, ex.variant);
        ex.chunk = chunk > 0 ? chunk : auto_chunk(p, ex.variant, ex.k);
    }
    if (o.inplace && inplace_max_k(p, ex.variant) < ex.k) {
        // the in-place pass is compiled for fewer variants: the widest that is
        int alt = 0;
        for (int v = 1; v <= num_variants_of(p->dim) && alt == 0; ++v)
            if (inplace_max_k(p, v) >= ex.k && variant_fits_shape(p, v) && (o.variant == 0 || v == o.variant))
                alt = v;
        if (alt == 0)
            return fail(STENCIL_E_UNSUPPORTED, "no in-place kernel is compiled for this stencil at k=%d", ex.k);
        ex.variant = alt;
        ex.chunk = chunk > 0 ? chunk : auto_chunk(p, alt, ex.k);
    }
    p->exec = ex;
    return STENCIL_OK;
}

// ---------------------------------------------------------------------------
// autotune cache: signature -> best execution
static std::mutex &tune_mutex() {
    static std::mutex m;
    return m;
}
static std::map<std::string, Exec> &tune_cache() {
    static std::map<std::string, Exec> m;
    return m;
}
// The tuned choice depends on the device architecture, the stencil, the grid
// and every option that narrows the candidates (method, depth, variant, chunk).
static std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');  // drop feature suffixes (":sramecc+:xnack-")
    return colon == std::string::npos ? a : a.substr(0, colon);
}
static std::string signature(const stencil_plan *p) {
    char buf[320];
    snprintf(buf, sizeof buf, "%s d%d r%d k%d bc%d t%d m%d fk%d v%d c%d ip%d %lld %lld %lld", device_arch().c_str(),
             p->dim, p->r, p->kind, p->bc, p->dtype, p->opts.method, p->opts.fused_k, p->opts.variant,
             p->opts.chunk, p->opts.inplace, (long long)p->shape[0], (long long)p->shape[1],
             (long long)p->shape[2]);
    return buf;
}

// Persisted autotune results: one "signature<TAB>method variant k chunk" line per
// entry in the file named by STENCIL_TUNE_CACHE (unset: $XDG_CACHE_HOME or
// ~/.cache, file paper_2103_08825_amd/autotune.txt; empty: not persisted).  A
// missing, unreadable or corrupt file (or line) is ignored: the plan tunes again.
static std::string tune_cache_path() {
    const char *env = getenv("STENCIL_TUNE_CACHE");
    if (env) return env;
    const char *xdg = getenv("XDG_CACHE_HOME");
    const char *home = getenv("HOME");
    std::string dir = xdg && *xdg ? std::string(xdg) : (home && *home ? std::string(home) + "/.cache" : "");
    return dir.empty() ? "" : dir + "/paper_2103_08825_amd/autotune.txt";
}

// An entry is used only if it names a choice the plan can run.
static bool exec_valid_for(const stencil_plan *p, const Exec &e) {
    if (e.method != p->exec.method || e.chunk < 0 || e.k < 1) return false;
    if (!variant_fits_shape(p, e.variant)) return false;
    if (p->opts.inplace) return inplace_max_k(p, e.variant) >= e.k;
    return max_k_of(p, e.variant) >= e.k;
}

static void tune_file_load(std::map<std::string, Exec> &m) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        char *tab = strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        Exec e{0, 0, 0, 0};
        if (sscanf(tab + 1, "%d %d %d %d", &e.method, &e.variant, &e.k, &e.chunk) != 4) continue;
        if (m.find(line) == m.end()) m[line] = e;
    }
    fclose(f);
}

static void tune_file_store(const std::map<std::string, Exec> &m) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        // create the directory chain (best effort; a failure only skips persisting)
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    bool ok = true;
    for (const auto &kv : m)
        ok = ok && fprintf(f, "%s\t%d %d %d %d\n", kv.first.c_str(), kv.second.method, kv.second.variant,
                           kv.second.k, kv.second.chunk) > 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path.c_str()) != 0) remove(tmp.c_str());
}

// One pool per device, created on first use, that keeps up to kPoolKeepBytes of
// freed blocks reserved across synchronisations (beyond that it releases them,
// as the device's default pool releases everything).  With the default pool
// the adjoint's workspace (about 28 fields) was mapped again on every call
// (256^3 FP32, T = 100: 7.6 ms per call, 7.25 ms with the memory kept).
constexpr uint64_t kPoolKeepBytes = (uint64_t)8 << 30;
hipError_t workspace_alloc(void **ptr, size_t bytes, hipStream_t st) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static hipMemPool_t pools[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipMallocAsync(ptr, bytes, st);
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> g(mu);
        if (!pools[dev]) {
            hipMemPoolProps props;
            std::memset(&props, 0, sizeof props);
            props.allocType = hipMemAllocationTypePinned;
            props.handleTypes = hipMemHandleTypeNone;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = dev;
            hipMemPool_t np = nullptr;
            e = hipMemPoolCreate(&np, &props);
            if (e != hipSuccess) return e;
            uint64_t keep = kPoolKeepBytes;
            e = hipMemPoolSetAttribute(np, hipMemPoolAttrReleaseThreshold, &keep);
            if (e != hipSuccess) {
                (void)hipMemPoolDestroy(np);
                return e;
            }
            pools[dev] = np;
        }
        pool = pools[dev];
    }
    return hipMallocFromPoolAsync(ptr, bytes, pool, st);
}

int plan_prepare(stencil_plan *p, hipStream_t st) {
    int dev = 0;
    STN_HIP(hipGetDevice(&dev));
    if (p->device >= 0) {
        if (p->device != dev)
            return fail(STENCIL_E_INVALID, "plan was prepared on device %d, current device is %d",
                        p->device, dev);
        return STENCIL_OK;
    }
    const size_t bytes = (size_t)p->points * elem_bytes(p->dtype);
    void *s = nullptr;
    if (!p->opts.inplace) STN_HIP(hipMalloc(&s, bytes));  // in place: no ping-pong field
    // generic-kernel tables: offsets placed on the axes of the kernel view
    // (n0, n1, n2) -- 3D (z, y, x), 2D (y, 1, x), 1D (1, 1, x) -- and weights in
    // compute precision
    static const int view_axis[4][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 1, 2}};
    std::vector<int> off3(3 * p->npts, 0);
    for (int j = 0; j < p->npts; ++j)
        for (int i = 0; i < p->dim; ++i) off3[3 * j + view_axis[p->dim][i]] = p->offsets[j * p->dim + i];
    int *d_off = nullptr;
    void *d_coef = nullptr;
    hipError_t e = hipMalloc(&d_off, off3.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&d_coef, (size_t)p->npts * 8);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_off, off3.data(), off3.size() * sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        if (p->dtype == STENCIL_F64) {
            e = hipMemcpyAsync(d_coef, p->coeffs.data(), (size_t)p->npts * 8, hipMemcpyHostToDevice, st);
        } else {
            std::vector<float> cf(p->npts);
            for (int j = 0; j < p->npts; ++j) cf[j] = (float)p->coeffs[j];
            e = hipMemcpyAsync(d_coef, cf.data(), (size_t)p->npts * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);  // cf leaves scope
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(s);
        if (d_off) (void)hipFree(d_off);
        if (d_coef) (void)hipFree(d_coef);
        return fail(e == hipErrorOutOfMemory ? STENCIL_E_NOMEM : STENCIL_E_DEVICE,
                    "plan device setup: %s", hipGetErrorString(e));
    }
    p->scratch[0] = s;
    p->d_off = d_off;
    p->d_coef = d_coef;
    p->device = dev;
    if (p->opts.inplace) {
        const int64_t sb = inplace_side_bytes(p, p->exec);
        if (sb > 0) {
            STN_HIP(hipMalloc(&p->slope, (size_t)sb));
            p->slope_bytes = sb;
        }
    }
    if (p->exec.method == STENCIL_METHOD_TESSELLATE) {
        const int64_t sb = tess_slope_bytes(p->r, p->exec.k, tess_tile_rows(p, p->exec.variant), p->n0, p->n1,
                                            p->n2, p->bc, p->dtype == STENCIL_F64 ? 8 : 4);
        if (sb > 0) {
            STN_HIP(hipMalloc(&p->slope, (size_t)sb));
            p->slope_bytes = sb;
        }
    }
    return STENCIL_OK;
}

void plan_drop_graph(stencil_plan *p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->graph_in = nullptr;
    p->graph_out = nullptr;
    p->graph_T = -1;
}

int plan_alloc_alias(stencil_plan *p) {
    if (p->scratch[1]) return STENCIL_OK;
    const size_t bytes = (size_t)p->points * elem_bytes(p->dtype);
    STN_HIP(hipMalloc(&p->scratch[1], bytes));
    return STENCIL_OK;
}

static int launch_pass(stencil_plan *p, const Exec &ex, int k, const void *src, void *dst,
                       hipStream_t st, bool in_place = false) {
    if (ex.method == STENCIL_METHOD_GENERIC) {
        const hipError_t e = launch_generic(p->dtype, src, dst, p->n0, p->n1, p->n2, p->npts, p->bc,
                                            p->d_off, p->d_coef, st);
        if (e != hipSuccess) return fail(STENCIL_E_DEVICE, "generic sweep launch: %s", hipGetErrorString(e));
        return STENCIL_OK;
    }
    SweepLauncher fn = pass_launcher(p, ex, k, in_place);
    if (!fn)
        return fail(STENCIL_E_UNSUPPORTED, "no %skernel for variant %d with k=%d", in_place ? "in-place " : "",
                    ex.variant, k);
    SweepLaunch L{src, dst, p->n0, p->n1, p->n2, p->bc, p->dense.data(), ex.chunk, p->slope};
    const hipError_t e = fn(L, st);
    if (e != hipSuccess) return fail(STENCIL_E_DEVICE, "fused sweep launch (k=%d): %s", k, hipGetErrorString(e));
    return STENCIL_OK;
}

int run_passes(stencil_plan *p, const Exec &ex, const void *src, void *dst, int64_t T, hipStream_t st) {
    const size_t bytes = (size_t)p->points * elem_bytes(p->dtype);
    if (T == 0) {
        if (src != dst) STN_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
        return STENCIL_OK;
    }
    const int kk = ex.method == STENCIL_METHOD_GENERIC ? 1 : ex.k;
    const int64_t full = T / kk;
    const int rem = (int)(T % kk);
    const int64_t P = full + (rem ? 1 : 0);
    if (p->opts.inplace) {
        if (ex.method == STENCIL_METHOD_GENERIC)  // no ping-pong field to fall back on
            return fail(STENCIL_E_UNSUPPORTED, "in-place plan: the buffers' alignment forbids the plan's kernels");
        // the first pass moves src into dst (unless they coincide), the others
        // update dst in place
        for (int64_t i = 1; i <= P; ++i) {
            const int k = (i <= full) ? kk : rem;
            const void *from = (i == 1) ? src : dst;
            const int rc = launch_pass(p, ex, k, from, dst, st, from == dst);
            if (rc != STENCIL_OK) return rc;
        }
        return STENCIL_OK;
    }
    // buffers: b_0 = src, b_P = dst, b_i alternates dst / scratch backwards from P
    const void *cur = src;
    for (int64_t i = 1; i <= P; ++i) {
        void *nxt = ((P - i) % 2 == 0) ? dst : p->scratch[0];
        const int k = (i <= full) ? kk : rem;
        const int rc = launch_pass(p, ex, k, cur, nxt, st);
        if (rc != STENCIL_OK) return rc;
        cur = nxt;
    }
    return STENCIL_OK;
}

// one step per launch for this plan: the measured plain choice, else the plan's
// own tile at k = 1 (the generic kernel stays generic)
Exec one_step_exec(const stencil_plan *p) {
    Exec ex = p->exec;
    if (ex.method == STENCIL_METHOD_GENERIC) return ex;
    ex.method = STENCIL_METHOD_PLAIN;
    ex.k = 1;
    ex.chunk = 0;
    const Choice *mc = measured_choice(p);
    if (mc) {
        int pv = 0, pc = 0;
        plain_choice(p, mc, &pv, &pc);
        if (variant_fits_shape(p, pv) && max_k_of(p, pv) >= 1) {
            ex.variant = pv;
            ex.chunk = pc;
        }
    }
    return ex;
}

// choose an execution whose lane width suits both pointers
Exec exec_for_ptrs(const stencil_plan *p, const void *a, const void *b) { return exec_for_ptrs(p, p->exec, a, b); }

Exec exec_for_ptrs(const stencil_plan *p, Exec ex, const void *a, const void *b) {
    if (ex.method == STENCIL_METHOD_GENERIC || variant_fits_ptr(p, ex.variant, a, b)) return ex;
    for (int v = 1; v <= num_variants_of(p->dim); ++v) {
        if (variant_fits_ptr(p, v, a, b) && max_k_of(p, v) >= ex.k) {
            ex.variant = v;
            return ex;
        }
    }
    ex.method = STENCIL_METHOD_GENERIC;
    ex.variant = 0;
    ex.k = 1;
    return ex;
}

static int time_exec(stencil_plan *p, const Exec &ex, hipStream_t st, float *ms_per_step) {
    hipEvent_t e0, e1;
    STN_HIP(hipEventCreate(&e0));
    STN_HIP(hipEventCreate(&e1));
    int rc = STENCIL_OK;
    float best = 1e30f;
    for (int rep = 0; rep < 4 && rc == STENCIL_OK; ++rep) {
        (void)hipEventRecord(e0, st);
        rc = launch_pass(p, ex, ex.k, p->scratch[0], p->scratch[1], st);
        (void)hipEventRecord(e1, st);
        if (rc != STENCIL_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(STENCIL_E_DEVICE, "autotune timing failed");
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best = std::min(best, ms);  // first run warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_step = best / (float)ex.k;
    return rc;
}

static int autotune_impl(stencil_plan *p, hipStream_t st) {
    // the generic kernel has nothing to choose; the tessellated method and
    // in-place plans keep the measured (variant, k) (their passes need buffers
    // sized for it)
    if (p->exec.method == STENCIL_METHOD_GENERIC || p->exec.method == STENCIL_METHOD_TESSELLATE ||
        p->opts.inplace) {
        p->tuned = 1;
        return STENCIL_OK;
    }
    const std::string sig = signature(p);
    {
        std::lock_guard<std::mutex> g(tune_mutex());
        static bool loaded = false;
        if (!loaded) {
            tune_file_load(tune_cache());
            loaded = true;
        }
        auto it = tune_cache().find(sig);
        if (it != tune_cache().end() && exec_valid_for(p, it->second)) {
            plan_drop_graph(p);
            p->exec = it->second;
            p->tuned = 1;
            return STENCIL_OK;
        }
    }
    int rc = plan_prepare(p, st);
    if (rc != STENCIL_OK) return rc;
    rc = plan_alloc_alias(p);
    if (rc != STENCIL_OK) return rc;
    STN_HIP(hipMemsetAsync(p->scratch[0], 0, (size_t)p->points * elem_bytes(p->dtype), st));
    Exec best = p->exec;
    float best_ms = 1e30f;
    const bool plain = p->exec.method == STENCIL_METHOD_PLAIN;
    const bool fixed_k = p->opts.fused_k > 0;
    const bool fixed_v = p->opts.variant > 0;
    for (int v = 1; v <= num_variants_of(p->dim); ++v) {
        if (fixed_v && v != p->opts.variant) continue;
        if (!variant_fits_shape(p, v)) continue;
        const int kmax = max_k_of(p, v);
        for (int k = 1; k <= kmax; ++k) {
            if (plain && k != 1) continue;
            if (fixed_k && k != p->opts.fused_k) continue;
            std::vector<int> chunks{p->opts.chunk};
            if (p->dim >= 2 && p->opts.chunk == 0) {
                for (int c : {16, 32, 64, 128, 256, 512})
                    if (c >= 2 * k * (2 * p->r + 1) && c < p->n0) chunks.push_back(c);
            }
            for (int c : chunks) {
                Exec ex{p->exec.method, v, k, c > 0 ? c : auto_chunk(p, v, k)};
                float ms = 0;
                rc = time_exec(p, ex, st, &ms);
                if (rc != STENCIL_OK) return rc;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = ex;
                }
            }
        }
    }
    plan_drop_graph(p);
    p->exec = best;
    p->tuned = 1;
    std::lock_guard<std::mutex> g(tune_mutex());
    tune_cache()[sig] = best;
    tune_file_store(tune_cache());
    return STENCIL_OK;
}

static int check_plan(const stencil_plan *p) {
    if (!p) return fail(STENCIL_E_INVALID, "plan is NULL");
    return STENCIL_OK;
}

}  // namespace stn

using namespace stn;

extern "C" {

int stencil_version(void) { return STENCIL_VERSION; }

const char *stencil_last_error(void) { return t_err.c_str(); }

int stencil_num_points(int dim, int radius, int kind) {
    clear_error();
    if (dim < 1 || dim > STENCIL_MAX_DIM) return fail(STENCIL_E_INVALID, "dim must be 1..3 (got %d)", dim);
    if (radius < 1) return fail(STENCIL_E_INVALID, "radius must be >= 1 (got %d)", radius);
    if (kind != STENCIL_STAR && kind != STENCIL_BOX) return fail(STENCIL_E_INVALID, "unknown kind %d", kind);
    if (kind == STENCIL_STAR) return 2 * dim * radius + 1;
    int n = 1;
    for (int i = 0; i < dim; ++i) n *= 2 * radius + 1;
    return n;
}

int stencil_offsets(int dim, int radius, int kind, int32_t *out) {
    const int n = stencil_num_points(dim, radius, kind);
    if (n < 0) return n;
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    return enumerate_offsets(dim, radius, kind, out);
}

int stencil_plan_create(stencil_plan **out, int dim, const int64_t *shape, int radius, int kind,
                        const double *coeffs, int ncoeffs, int bc, int dtype, const stencil_opts *opts) {
    clear_error();
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    *out = nullptr;
    const int npts = stencil_num_points(dim, radius, kind);
    if (npts < 0) return npts;
    if (radius > STENCIL_MAX_RADIUS)
        return fail(STENCIL_E_UNSUPPORTED, "radius %d exceeds the maximum %d", radius, STENCIL_MAX_RADIUS);
    if (!shape) return fail(STENCIL_E_INVALID, "shape is NULL");
    if (!coeffs) return fail(STENCIL_E_INVALID, "coeffs is NULL");
    if (ncoeffs != npts)
        return fail(STENCIL_E_INVALID, "ncoeffs=%d but the stencil has %d points", ncoeffs, npts);
    if (bc != STENCIL_BC_ZERO && bc != STENCIL_BC_PERIODIC) return fail(STENCIL_E_INVALID, "unknown bc %d", bc);
    if (elem_bytes(dtype) == 0) return fail(STENCIL_E_INVALID, "unknown dtype %d", dtype);
    int64_t points = 1;
    for (int i = 0; i < dim; ++i) {
        if (shape[i] < 1) return fail(STENCIL_E_INVALID, "shape[%d]=%lld must be >= 1", i, (long long)shape[i]);
        if (shape[i] > ((int64_t)1 << 40) || points > ((int64_t)1 << 46) / shape[i])
            return fail(STENCIL_E_INVALID, "grid too large");
        points *= shape[i];
    }
    if (opts) {
        if (opts->method < STENCIL_METHOD_AUTO || opts->method > STENCIL_METHOD_TESSELLATE)
            return fail(STENCIL_E_INVALID, "unknown method %d", opts->method);
        if (opts->fused_k < 0) return fail(STENCIL_E_INVALID, "fused_k must be >= 0");
        if (opts->variant < 0) return fail(STENCIL_E_INVALID, "variant must be >= 0");
        if (opts->chunk < 0) return fail(STENCIL_E_INVALID, "chunk must be >= 0");
    }
    stencil_plan *p = new (std::nothrow) stencil_plan();
    if (!p) return fail(STENCIL_E_NOMEM, "out of host memory");
    p->dim = dim;
    p->r = radius;
    p->kind = kind;
    p->bc = bc;
    p->dtype = dtype;
    p->npts = npts;
    for (int i = 0; i < 3; ++i) p->shape[i] = i < dim ? shape[i] : 0;
    p->points = points;
    if (dim == 3) {
        p->n0 = shape[0];
        p->n1 = shape[1];
        p->n2 = shape[2];
    } else if (dim == 2) {
        p->n0 = shape[0];
        p->n1 = 1;
        p->n2 = shape[1];
    } else {
        p->n0 = 1;
        p->n1 = 1;
        p->n2 = shape[0];
    }
    p->offsets.resize((size_t)npts * dim);
    enumerate_offsets(dim, radius, kind, p->offsets.data());
    p->coeffs.assign(coeffs, coeffs + npts);
    const int W = 2 * radius + 1;
    int ndense = 1;
    for (int i = 0; i < dim; ++i) ndense *= W;
    p->dense.assign(ndense, 0.0);
    for (int j = 0; j < npts; ++j) {
        int idx = 0;
        for (int i = 0; i < dim; ++i) idx = idx * W + (p->offsets[j * dim + i] + radius);
        p->dense[idx] = coeffs[j];
    }
    p->opts = opts ? *opts : stencil_opts{0, 0, 0, 0, 0, 0, 0};
    p->tuned = 0;
    p->device = -1;
    p->scratch[0] = p->scratch[1] = nullptr;
    p->d_off = nullptr;
    p->d_coef = nullptr;
    p->slope = nullptr;
    p->slope_bytes = 0;
    p->graph = nullptr;
    p->graph_exec = nullptr;
    p->graph_in = nullptr;
    p->graph_out = nullptr;
    p->graph_T = -1;
    p->graph_failed = 0;
    const int rc = resolve_exec(p);
    if (rc != STENCIL_OK) {
        delete p;
        return rc;
    }
    *out = p;
    return STENCIL_OK;
}

void stencil_plan_destroy(stencil_plan *p) {
    if (!p) return;
    plan_drop_graph(p);
    if (p->scratch[0]) (void)hipFree(p->scratch[0]);
    if (p->scratch[1]) (void)hipFree(p->scratch[1]);
    if (p->d_off) (void)hipFree(p->d_off);
    if (p->d_coef) (void)hipFree(p->d_coef);
    if (p->slope) (void)hipFree(p->slope);
    for (hipEvent_t e : p->aux_ev)
        if (e) (void)hipEventDestroy(e);
    if (p->aux_stream) (void)hipStreamDestroy(p->aux_stream);
    delete p;
}

int stencil_plan_info(const stencil_plan *p, stencil_plan_desc *out) {
    clear_error();
    if (check_plan(p) != STENCIL_OK) return STENCIL_E_INVALID;
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    std::memset(out, 0, sizeof *out);
    out->dim = p->dim;
    out->radius = p->r;
    out->kind = p->kind;
    out->bc = p->bc;
    out->dtype = p->dtype;
    out->npts = p->npts;
    for (int i = 0; i < 3; ++i) out->shape[i] = p->shape[i];
    out->points = p->points;
    out->method = p->exec.method;
    out->fused_k = p->exec.method == STENCIL_METHOD_GENERIC ? 1 : p->exec.k;
    out->variant = p->exec.variant;
    out->elem_bytes = elem_bytes(p->dtype);
    if (p->exec.method != STENCIL_METHOD_GENERIC) {
        VariantShape v;
        if (shape_of(p->dim, p->exec.variant, &v)) {
            const Geometry g = p->dim == 1 ? seg1d_geometry(p->r, p->exec.k, v, p->n2)
                                           : stream_geometry(p->dim, p->r, p->exec.k, v, p->n0, p->n1,
                                                             p->n2, p->exec.chunk);
            out->tile[0] = g.out_x;
            out->tile[1] = p->dim == 3 ? g.out_y : 0;
            out->tile[2] = p->dim >= 2 ? g.chunk : 0;
            if (p->exec.method == STENCIL_METHOD_TESSELLATE) out->tile[1] = v.nw * v.rw;  // y tile rows
        }
    }
    const int64_t field = p->points * elem_bytes(p->dtype);
    out->scratch_bytes = (p->scratch[0] ? field : 0) + (p->scratch[1] ? field : 0) + p->slope_bytes;
    out->tuned = p->tuned;
    return STENCIL_OK;
}

int stencil_plan_prepare(stencil_plan *p, void *stream) {
    clear_error();
    if (check_plan(p) != STENCIL_OK) return STENCIL_E_INVALID;
    return plan_prepare(p, (hipStream_t)stream);
}

int stencil_autotune(stencil_plan *p, void *stream) {
    clear_error();
    if (check_plan(p) != STENCIL_OK) return STENCIL_E_INVALID;
    return autotune_impl(p, (hipStream_t)stream);
}

int stencil_run(stencil_plan *p, const void *d_in, void *d_out, int64_t T, void *stream) {
    clear_error();
    if (check_plan(p) != STENCIL_OK) return STENCIL_E_INVALID;
    if (!d_in || !d_out) return fail(STENCIL_E_INVALID, "d_in and d_out must not be NULL");
    if (T < 0) return fail(STENCIL_E_INVALID, "T must be >= 0 (got %lld)", (long long)T);
    hipStream_t st = (hipStream_t)stream;
    int rc = plan_prepare(p, st);
    if (rc != STENCIL_OK) return rc;
    if (p->opts.autotune && !p->tuned) {
        rc = autotune_impl(p, st);
        if (rc != STENCIL_OK) return rc;
    }
    const bool copy_alias = d_in == d_out && T > 0 && !p->opts.inplace;
    if (copy_alias) {
        rc = plan_alloc_alias(p);
        if (rc != STENCIL_OK) return rc;
    }
    // enqueue the whole sweep on `s` (the caller's stream, or a capture stream)
    auto enqueue = [&](hipStream_t s) -> int {
        const void *src = d_in;
        if (copy_alias) {
            STN_HIP(hipMemcpyAsync(p->scratch[1], d_in, (size_t)p->points * elem_bytes(p->dtype),
                                   hipMemcpyDeviceToDevice, s));
            src = p->scratch[1];
        }
        const Exec ex = exec_for_ptrs(p, src, d_out);
        return run_passes(p, ex, src, d_out, T, s);
    };
    if (!p->opts.graph || T == 0 || p->graph_failed) return enqueue(st);
    if (!(p->graph_exec && p->graph_in == d_in && p->graph_out == d_out && p->graph_T == T)) {
        // record on a private stream: the caller's stream may be the legacy default
        // stream, which cannot be captured; the launches depend on nothing else.
        // If capturing or instantiating fails, nothing was enqueued: the plan
        // stops recording and runs the sweep with direct launches.
        plan_drop_graph(p);
        hipStream_t cap = nullptr;
        STN_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cap);
            (void)hipGetLastError();
            p->graph_failed = 1;
            return enqueue(st);
        }
        rc = enqueue(cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cap, &g);
        (void)hipStreamDestroy(cap);
        if (rc != STENCIL_OK && e == hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc;  // an argument or launch error, not a capture failure
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            p->graph_exec = nullptr;
            (void)hipGetLastError();
            p->graph_failed = 1;
            return enqueue(st);
        }
        p->graph = g;
        p->graph_in = d_in;
        p->graph_out = d_out;
        p->graph_T = T;
    }
    STN_HIP(hipGraphLaunch(p->graph_exec, st));
    return STENCIL_OK;
}

int stencil_reduce(int dtype, const void *d_u, const void *d_ref, int64_t n, double *d_out, void *stream) {
    clear_error();
    if (elem_bytes(dtype) == 0) return fail(STENCIL_E_INVALID, "unknown dtype %d", dtype);
    if (n < 0) return fail(STENCIL_E_INVALID, "n must be >= 0");
    if (!d_out || (!d_u && n > 0)) return fail(STENCIL_E_INVALID, "NULL pointer");
    // stream-ordered partials: concurrent reductions on different streams never share them
    hipStream_t st = (hipStream_t)stream;
    double *part = nullptr;
    STN_HIP(workspace_alloc((void **)&part, reduce_partials_bytes(), st));
    const hipError_t e = launch_reduce(dtype, d_u, d_ref, n, part, d_out, st);
    const hipError_t f = hipFreeAsync(part, st);
    if (e != hipSuccess) return fail(STENCIL_E_DEVICE, "reduction launch: %s", hipGetErrorString(e));
    if (f != hipSuccess) return fail(STENCIL_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(f));
    return STENCIL_OK;
}

}  // extern "C"
