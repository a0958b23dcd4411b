// Host runtime of the dctsn library: the C ABI declared in include/dctsn.h.
//
// Input validation mirrors the "Launch Solver only with complete, consistent
// input" rule of Sec. II-B: each set_* call checks its own arguments (EINVAL);
// consistency between calls (material ids vs M, G of the source vs the cross
// sections, sources inside the grid, P_N order vs the quadrature) is checked
// when the solve starts (ESTATE).
//
// dct_solve enqueues, on the context's stream:
//   sigma tables -> ray trace -> [transition, M map, sweep(s), D map, combine]*
//   -> dose
// where the bracket is one iteration set of the device-driven machine (see
// k_source.hip).  The host enqueues sets in chunks and polls a single device
// counter of unfinished right-hand sides one chunk behind, so the GPU never
// waits for the host inside a solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dctsn.h"
#include "dct_internal.h"

using namespace dct;

// Fixed device scratch of dct_effective_dose_noalloc: the per-group
// fluence-to-dose factors (FP64, at most 256 groups, the cap of dct_set_xs)
// at byte 0 and the per-material zero flags (at most DCT_MAXMAT) at byte 2048.
// Every GPU holds its own copy for the life of the process; host code only
// ever uses the device address resolved for that GPU (scratch_dev), never
// this name.
#define DCT_NOALLOC_MAXG 256
#define DCT_NOALLOC_ZOFF 2048
static __device__ __align__(256) unsigned char scratch[DCT_NOALLOC_ZOFF + 256];

namespace {

thread_local std::string g_create_error;

// DCT_LOG = 0..3: messages up to that level go to stderr (1: schedule choices
// and tuning results, 2: one line per solve, 3: every tuning candidate)
int log_level()
{
    static const int lv = [] {
        const char *e = std::getenv("DCT_LOG");
        return e ? std::atoi(e) : 0;
    }();
    return lv;
}

__attribute__((format(printf, 2, 3))) void dlog(int level, const char *fmt, ...)
{
    if (log_level() < level) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[dctsn] %s\n", buf);
}

// Persisted sweep schedules: with DCT_TUNE_CACHE = path, every tuning result
// is appended to that text file as one line, and a new context on a device of
// the same architecture and compute-unit count starts from the file's entries
// (the last entry of a shape wins), so a new process need not tune again.
constexpr const char *kTuneTag = "dctsn-tune-1";

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), resolved
// once per device.
hipError_t scratch_resolve(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[device] = p;
    return hipSuccess;
}

void *scratch_dev(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct dct_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    std::string err;

    bool has_geo = false, has_xs = false, has_quad = false, has_src = false;
    int nx = 0, ny = 0, nz = 0;
    double dx = 0, dy = 0, dz = 0, org[3] = {0, 0, 0};
    std::vector<uint8_t> mat;
    std::vector<double> rho;
    bool rho_dev = false;       // the densities were last set from a device buffer (no host copy)
    int G = 0, M = 0, L = 0;
    std::vector<double> st, ss, kap;
    std::vector<double> edges;  // group edges (keV, descending) when given
    int N = 0;
    std::vector<double> dirs, w;
    int B = 0;
    std::vector<double> pos, axis, gw;
    double fan = 0, cone = 0;
    std::vector<double> iso;

    std::map<std::string, DevBuf> bufs;
    bool dev_dirty = true;      // inputs changed since the last upload
    int tab_prec = -1;          // precision of the uploaded moment-map tables
    bool solved = false;
    int solved_prec = 0;
    int solved_Nm = 0;
    int solved_S = 1;           // sources per right-hand side of the last solve
    bool kept = false;          // the last solve kept per-group fluxes and fixup sets

    // sweep schedules chosen by the autotuner, per problem shape
    struct Tuned {
        int nx, ny, nz, N, B, prec, keep, bk, sync, chain, rhs;
    };
    std::vector<Tuned> tuned;
    int last_bk = 16, last_sync = 1;   // schedule of the last solve (reused by the adjoint)
    int last_chain = 1;
    int last_rhs = 1;
    bool last_fused = false;
    bool last_warm = false;
    // moments left in the "phi" buffer by the last completed solve (warm starts)
    struct WarmState {
        bool valid;
        int B, G, Nm;
        long C;
        int prec;
        void *phi;
    } warm = {false, 0, 0, 0, 0, 0, nullptr};
    size_t lds_max = 65536;            // LDS bytes one workgroup may allocate on the device
    int ncu = 256;                     // compute units of the device
    std::string arch;                  // the device's architecture name (tune-cache key)
    bool pipe_clean = false;           // pipelined-block face buffers hold only the empty marker
    unsigned sweep_seq = 0;            // counts sweep launches (part of the pipelined blocks' launch tag)
    hipStream_t own_stream = nullptr;  // capture stream when the context's stream is the null stream
    hipStream_t half_stream = nullptr; // second stream of the split iteration sets (default priority)
    hipEvent_t ev_half[3] = {nullptr, nullptr, nullptr};   // fork, and the second stream's chunk ends
    int last_streams = 1;              // streams the last solve's iteration sets ran on

    std::vector<hipEvent_t> evpool, evpool_m;   // event pairs around timed sweep / fused-map launches
    hipEvent_t ev_poll[2] = {nullptr, nullptr};
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
    int *h_unf = nullptr;
    void *h_stage = nullptr;
    size_t h_stage_bytes = 0;
};

static int fail(dct_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HC(call)                                                                                  \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, e_ == hipErrorOutOfMemory ? DCT_ENOMEM : DCT_EDEVICE,                \
                        std::string(#call) + ": " + hipGetErrorString(e_));                      \
    } while (0)

static hipError_t dbuf(dct_ctx *ctx, const std::string &name, size_t bytes, void **out)
{
    DevBuf &b = ctx->bufs[name];
    if (bytes == 0) bytes = 256;
    if (b.bytes < bytes) {
        if (b.p) (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        hipError_t e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) return e;
        b.bytes = bytes;
    }
    *out = b.p;
    return hipSuccess;
}

static bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

static void tune_cache_load(dct_ctx *ctx)
{
    const char *path = std::getenv("DCT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512], tag[32], arch[128];
    int n = 0;
    while (std::fgets(line, sizeof(line), f)) {
        dct_ctx::Tuned t;
        int ncu = 0;
        if (std::sscanf(line, "%31s %127s %d %d %d %d %d %d %d %d %d %d %d %d", tag, arch, &ncu, &t.nx, &t.ny, &t.nz,
                        &t.N, &t.B, &t.prec, &t.keep, &t.bk, &t.sync, &t.chain, &t.rhs) != 14)
            continue;
        if (std::strcmp(tag, kTuneTag) != 0 || ctx->arch != arch || ncu != ctx->ncu) continue;
        ctx->tuned.push_back(t);
        ++n;
    }
    std::fclose(f);
    dlog(1, "tune cache %s: %d schedule(s) for %s with %d CUs", path, n, ctx->arch.c_str(), ctx->ncu);
}

static void tune_cache_save(const dct_ctx *ctx, const dct_ctx::Tuned &t)
{
    const char *path = std::getenv("DCT_TUNE_CACHE");
    if (!path || !*path) return;
    char line[512];
    const int len = std::snprintf(line, sizeof(line), "%s %s %d %d %d %d %d %d %d %d %d %d %d %d\n", kTuneTag,
                                  ctx->arch.c_str(), ctx->ncu, t.nx, t.ny, t.nz, t.N, t.B, t.prec, t.keep, t.bk,
                                  t.sync, t.chain, t.rhs);
    FILE *f = std::fopen(path, "a");
    if (!f) {
        dlog(1, "tune cache %s: cannot append", path);
        return;
    }
    std::fwrite(line, 1, (size_t)len, f);   // one write per line, so appending processes do not interleave
    std::fclose(f);
}

static void invalidate(dct_ctx *ctx)
{
    ctx->solved = false;
    ctx->kept = false;
    ctx->dev_dirty = true;
    ctx->tab_prec = -1;
}

extern "C" {

int dct_create(dct_ctx **out, int device, void *stream)
{
    if (!out) {
        g_create_error = "dct_create: out is NULL";
        return DCT_EINVAL;
    }
    *out = nullptr;
    dct_ctx *ctx = nullptr;
    try {
        ctx = new dct_ctx();
    } catch (const std::bad_alloc &) {
        g_create_error = "dct_create: out of host memory";
        return DCT_ENOMEM;
    }
    ctx->device = device;
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || device >= n) {
            g_create_error = std::string("dct_create: no HIP device ") + std::to_string(device) + " (" +
                             (e != hipSuccess ? hipGetErrorString(e) : "device index out of range") + ")";
            delete ctx;
            return DCT_EDEVICE;
        }
        e = hipSetDevice(device);
        if (e == hipSuccess && device < kMaxDevices) e = scratch_resolve(device);
        if (e == hipSuccess) {
            int lds = 0;
            if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
                ctx->lds_max = (size_t)lds;
            int ncu = 0;
            if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
                ctx->ncu = ncu;
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
                ctx->arch = prop.gcnArchName;
                // the name's feature suffix (":sramecc+:xnack-") is not part of the key
                ctx->arch = ctx->arch.substr(0, ctx->arch.find(':'));
            }
            if (ctx->arch.empty()) ctx->arch = "unknown";
            tune_cache_load(ctx);
        }
        if (e == hipSuccess) e = hipEventCreate(&ctx->ev_poll[0]);
        if (e == hipSuccess) e = hipEventCreate(&ctx->ev_poll[1]);
        if (e == hipSuccess) e = hipEventCreate(&ctx->ev_t0);
        if (e == hipSuccess) e = hipEventCreate(&ctx->ev_t1);
        if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->h_unf, 4 * sizeof(int), hipHostMallocDefault);
        if (e != hipSuccess) {
            g_create_error = std::string("dct_create: ") + hipGetErrorString(e);
            delete ctx;
            return DCT_EDEVICE;
        }
        ctx->stream = (hipStream_t)stream;
    }
    g_create_error.clear();
    *out = ctx;
    return DCT_OK;
}

int dct_destroy(dct_ctx *ctx)
{
    if (!ctx) return DCT_OK;
    if (ctx->device >= 0) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (auto &kv : ctx->bufs)
            if (kv.second.p) (void)hipFree(kv.second.p);
        for (hipEvent_t e : ctx->evpool) (void)hipEventDestroy(e);
        for (hipEvent_t e : ctx->evpool_m) (void)hipEventDestroy(e);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
        if (ctx->half_stream) (void)hipStreamDestroy(ctx->half_stream);
        for (hipEvent_t e : ctx->ev_half)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : {ctx->ev_poll[0], ctx->ev_poll[1], ctx->ev_t0, ctx->ev_t1})
            if (e) (void)hipEventDestroy(e);
        if (ctx->h_unf) (void)hipHostFree(ctx->h_unf);
        if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    }
    delete ctx;
    return DCT_OK;
}

const char *dct_last_error(const dct_ctx *ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

int dct_set_geometry(dct_ctx *ctx, int nx, int ny, int nz, double dx, double dy, double dz,
                     const double *origin, const uint8_t *material, const double *density)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(ctx, DCT_EINVAL, "set_geometry: nx, ny, nz must be > 0");
    if (!(dx > 0) || !(dy > 0) || !(dz > 0) || !std::isfinite(dx) || !std::isfinite(dy) || !std::isfinite(dz))
        return fail(ctx, DCT_EINVAL, "set_geometry: voxel sizes must be finite and > 0");
    // the kernels address a per-voxel array through 32-bit byte offsets of
    // FP64 elements (buffer descriptors), so C * 8 must stay below 2^31
    if (nx > 4096 || ny > 4096 || nz > 4096 || (long long)nx * ny * nz * 8 >= (1LL << 31))
        return fail(ctx, DCT_EINVAL, "set_geometry: grid too large (nx * ny * nz must be below 2^28 = 268435456 voxels)");
    if (!origin || !material || !density) return fail(ctx, DCT_EINVAL, "set_geometry: NULL array");
    if (!finite_all(origin, 3)) return fail(ctx, DCT_EINVAL, "set_geometry: origin not finite");
    size_t C = (size_t)nx * ny * nz;
    for (size_t v = 0; v < C; ++v)
        if (!std::isfinite(density[v]) || density[v] < 0)
            return fail(ctx, DCT_EINVAL, "set_geometry: density must be finite and >= 0 (voxel " +
                                             std::to_string(v) + ")");
    try {
        ctx->mat.assign(material, material + C);
        ctx->rho.assign(density, density + C);
        ctx->rho_dev = false;
    } catch (const std::bad_alloc &) {
        return fail(ctx, DCT_ENOMEM, "set_geometry: out of host memory");
    }
    ctx->nx = nx;
    ctx->ny = ny;
    ctx->nz = nz;
    ctx->dx = dx;
    ctx->dy = dy;
    ctx->dz = dz;
    std::memcpy(ctx->org, origin, sizeof(ctx->org));
    ctx->has_geo = true;
    ctx->iso.clear();
    invalidate(ctx);
    return DCT_OK;
}

int dct_set_density_dev(dct_ctx *ctx, const double *density)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (!ctx->has_geo) return fail(ctx, DCT_ESTATE, "set_density_dev: no geometry (call dct_set_geometry first)");
    if (!density) return fail(ctx, DCT_EINVAL, "set_density_dev: NULL array");
    const long C = (long)ctx->nx * ctx->ny * ctx->nz;
    HC(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    void *d_rho, *d_bad;
    HC(dbuf(ctx, "scr_bad", 8, &d_bad));
    HC(hipMemsetAsync(d_bad, 0xff, 8, s));
    HC(launch_screen(density, C, 1, (unsigned long long *)d_bad, s));
    unsigned long long bad = 0;
    HC(hipMemcpyAsync(&bad, d_bad, 8, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    if (bad != ~0ULL)
        return fail(ctx, DCT_EINVAL, "set_density_dev: density must be finite and >= 0 (voxel " + std::to_string(bad) + ")");
    HC(dbuf(ctx, "rho", (size_t)C * 8, &d_rho));
    HC(hipMemcpyAsync(d_rho, density, (size_t)C * 8, hipMemcpyDeviceToDevice, s));
    HC(hipStreamSynchronize(s));
    ctx->rho_dev = true;
    invalidate(ctx);
    return DCT_OK;
}

int dct_set_xs(dct_ctx *ctx, int G, const double *edges_keV, int M, int L, const double *sigma_t,
               const double *sigma_s, const double *kerma)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (G < 1 || G > 256) return fail(ctx, DCT_EINVAL, "set_xs: G must be in [1, 256]");
    if (M < 1 || M > DCT_MAXMAT) return fail(ctx, DCT_EINVAL, "set_xs: M must be in [1, 8]");
    if (L < 0 || L > DCT_MAXL) return fail(ctx, DCT_EINVAL, "set_xs: L must be in [0, 5]");
    if (!sigma_t || !sigma_s || !kerma) return fail(ctx, DCT_EINVAL, "set_xs: NULL array");
    if (edges_keV)
        for (int g = 0; g < G; ++g)
            if (!(edges_keV[g] > edges_keV[g + 1]))
                return fail(ctx, DCT_EINVAL, "set_xs: edges must be strictly descending");
    size_t nss = (size_t)M * (L + 1) * G * G;
    if (!finite_all(sigma_t, (size_t)M * G) || !finite_all(sigma_s, nss) || !finite_all(kerma, (size_t)M * G))
        return fail(ctx, DCT_EINVAL, "set_xs: non-finite value");
    for (int i = 0; i < M * G; ++i)
        if (sigma_t[i] < 0 || kerma[i] < 0) return fail(ctx, DCT_EINVAL, "set_xs: negative sigma_t or kerma");
    for (int m = 0; m < M; ++m)
        for (int l = 0; l <= L; ++l)
            for (int gf = 0; gf < G; ++gf)
                for (int gt = 0; gt < gf; ++gt)
                    if (sigma_s[(((size_t)m * (L + 1) + l) * G + gf) * G + gt] != 0.0)
                        return fail(ctx, DCT_EINVAL, "set_xs: upscatter entry sigma_s[" + std::to_string(m) +
                                                         "][" + std::to_string(l) + "][" + std::to_string(gf) +
                                                         "][" + std::to_string(gt) + "] != 0");
    ctx->st.assign(sigma_t, sigma_t + (size_t)M * G);
    ctx->ss.assign(sigma_s, sigma_s + nss);
    ctx->kap.assign(kerma, kerma + (size_t)M * G);
    if (edges_keV) ctx->edges.assign(edges_keV, edges_keV + G + 1);
    else ctx->edges.clear();
    ctx->G = G;
    ctx->M = M;
    ctx->L = L;
    ctx->has_xs = true;
    invalidate(ctx);
    return DCT_OK;
}

int dct_set_quadrature(dct_ctx *ctx, int n, const double *dirs, const double *w)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (n < 1 || n > 4096) return fail(ctx, DCT_EINVAL, "set_quadrature: n must be in [1, 4096]");
    if (!dirs || !w) return fail(ctx, DCT_EINVAL, "set_quadrature: explicit dirs and weights are required");
    if (!finite_all(dirs, 3 * (size_t)n) || !finite_all(w, n))
        return fail(ctx, DCT_EINVAL, "set_quadrature: non-finite value");
    for (int i = 0; i < n; ++i) {
        const double *o = dirs + 3 * i;
        double nn = std::sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
        if (std::fabs(nn - 1.0) > 1e-12) return fail(ctx, DCT_EINVAL, "set_quadrature: direction not unit length");
        if (o[0] == 0.0 || o[1] == 0.0 || o[2] == 0.0)
            return fail(ctx, DCT_EINVAL, "set_quadrature: direction with a zero component");
        if (!(w[i] > 0)) return fail(ctx, DCT_EINVAL, "set_quadrature: weights must be > 0");
    }
    ctx->dirs.assign(dirs, dirs + 3 * (size_t)n);
    ctx->w.assign(w, w + n);
    ctx->N = n;
    ctx->has_quad = true;
    invalidate(ctx);
    return DCT_OK;
}

int dct_set_source(dct_ctx *ctx, int B, const double *pos, const double *axis, double fan_deg, double cone_deg,
                   const double *group_w)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (!ctx->has_xs) return fail(ctx, DCT_ESTATE, "set_source: call set_xs first (group weights need G)");
    if (B < 1 || B > 65535) return fail(ctx, DCT_EINVAL, "set_source: B must be in [1, 65535]");
    if (!pos || !group_w) return fail(ctx, DCT_EINVAL, "set_source: NULL array");
    if (!(fan_deg > 0 && fan_deg <= 360) || !(cone_deg > 0 && cone_deg <= 180))
        return fail(ctx, DCT_EINVAL, "set_source: fan must be in (0, 360], cone in (0, 180] degrees");
    if (!finite_all(pos, 3 * (size_t)B) || !finite_all(group_w, ctx->G) || (axis && !finite_all(axis, 3 * (size_t)B)))
        return fail(ctx, DCT_EINVAL, "set_source: non-finite value");
    for (int g = 0; g < ctx->G; ++g)
        if (group_w[g] < 0) return fail(ctx, DCT_EINVAL, "set_source: negative group weight");
    std::vector<double> ax(3 * (size_t)B);
    for (int b = 0; b < B; ++b) {
        double a0, a1, a2;
        if (axis) {
            a0 = axis[3 * b];
            a1 = axis[3 * b + 1];
            a2 = axis[3 * b + 2];
        } else {
            a0 = -pos[3 * b];
            a1 = -pos[3 * b + 1];
            a2 = 0.0;
        }
        if (std::hypot(a0, a1) == 0.0)
            return fail(ctx, DCT_EINVAL, "set_source: beam axis has no component in the z = 0 plane");
        ax[3 * b] = a0;
        ax[3 * b + 1] = a1;
        ax[3 * b + 2] = a2;
    }
    ctx->pos.assign(pos, pos + 3 * (size_t)B);
    ctx->axis = ax;
    ctx->gw.assign(group_w, group_w + ctx->G);
    ctx->fan = fan_deg;
    ctx->cone = cone_deg;
    ctx->B = B;
    ctx->has_src = true;
    invalidate(ctx);
    return DCT_OK;
}

int dct_set_volume_source(dct_ctx *ctx, const double *S)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (!S) {
        ctx->iso.clear();
        invalidate(ctx);
        return DCT_OK;
    }
    if (!ctx->has_geo || !ctx->has_xs) return fail(ctx, DCT_ESTATE, "set_volume_source: set geometry and xs first");
    size_t n = (size_t)ctx->G * ctx->nx * ctx->ny * ctx->nz;
    if (!finite_all(S, n)) return fail(ctx, DCT_EINVAL, "set_volume_source: non-finite value");
    ctx->iso.assign(S, S + n);
    invalidate(ctx);
    return DCT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- solve
namespace {

struct Plan {
    int prec = 0, Nm = 0, Nc[2] = {0, 0}, NcP = 0, NmP = 0;
    int BK = 1, NBJ = 1, NBK = 1, nblk = 1, ndiag = 1;
    size_t tsz = 8;
    std::vector<int> cdir;   // [2][N]
};

// Sweep blocks: 64 y rows (lanes) x bk z layers (waves) per workgroup; the
// blocks of one sweep run as ndiag block diagonals.
static void set_blocks(Plan &pl, int bk, int ny, int nz)
{
    pl.BK = std::min(bk, nz);
    pl.NBJ = (ny + 63) / 64;
    pl.NBK = (nz + pl.BK - 1) / pl.BK;
    pl.nblk = pl.NBJ * pl.NBK;
    pl.ndiag = pl.NBJ + pl.NBK - 1;
}

static int check_consistency(dct_ctx *ctx, const dct_opts &o, Plan &pl)
{
    if (!ctx->has_geo || !ctx->has_xs || !ctx->has_quad || !ctx->has_src)
        return fail(ctx, DCT_ESTATE, std::string("solve: missing input:") + (ctx->has_geo ? "" : " geometry") +
                                         (ctx->has_xs ? "" : " cross-sections") + (ctx->has_quad ? "" : " quadrature") +
                                         (ctx->has_src ? "" : " source"));
    if ((int)ctx->gw.size() != ctx->G)
        return fail(ctx, DCT_ESTATE, "solve: source group weights were given for a different G; call set_source again");
    if (!ctx->iso.empty() && ctx->iso.size() != (size_t)ctx->G * ctx->nx * ctx->ny * ctx->nz)
        return fail(ctx, DCT_ESTATE, "solve: volume source shape does not match the current G and grid");
    for (uint8_t m : ctx->mat)
        if ((int)m >= ctx->M) return fail(ctx, DCT_ESTATE, "solve: material id >= M");
    for (int b = 0; b < ctx->B; ++b) {
        const double *p = &ctx->pos[3 * b];
        double hi[3] = {ctx->org[0] + ctx->nx * ctx->dx, ctx->org[1] + ctx->ny * ctx->dy, ctx->org[2] + ctx->nz * ctx->dz};
        bool inside = true;
        for (int a = 0; a < 3; ++a) inside = inside && p[a] >= ctx->org[a] && p[a] <= hi[a];
        if (inside) return fail(ctx, DCT_ESTATE, "solve: source " + std::to_string(b) + " lies inside the voxel grid");
    }
    if (o.precision < DCT_FP64 || o.precision > DCT_FP32_BF16X3) return fail(ctx, DCT_EINVAL, "solve: bad precision");
    if (o.max_iter < 1) return fail(ctx, DCT_EINVAL, "solve: max_iter must be >= 1");
    if (!(o.tol >= 0) || !std::isfinite(o.tol)) return fail(ctx, DCT_EINVAL, "solve: tol must be finite and >= 0");
    if (o.fixed_iters)
        for (int g = 0; g < ctx->G; ++g)
            if (o.fixed_iters[g] < 1 || o.fixed_iters[g] > 1000000)
                return fail(ctx, DCT_EINVAL, "solve: fixed_iters entries must be in [1, 1e6]");
    if (o.test_inflow && !finite_all(o.test_inflow, ctx->G))
        return fail(ctx, DCT_EINVAL, "solve: test_inflow not finite");

    const int L = ctx->L, N = ctx->N;
    const int Nm = (L + 1) * (L + 1);
    pl.Nm = Nm;
    pl.prec = o.precision;
    pl.tsz = o.precision == DCT_FP64 ? 8 : 4;
    if ((size_t)16 * ((ctx->nx | 1) + 1) * pl.tsz > 65536)
        return fail(ctx, DCT_EINVAL, "solve: nx too large for the 64 KiB combine tile (nx <= 510 in FP64, 1022 in FP32)");
    // moment maps and the check that the quadrature integrates them: D M = I
    std::vector<double> Y((size_t)N * Nm);
    for (int n = 0; n < N; ++n)
        real_sh_cart<double>(L, ctx->dirs[3 * n], ctx->dirs[3 * n + 1], ctx->dirs[3 * n + 2], &Y[(size_t)n * Nm]);
    double worst = 0.0;
    for (int a = 0; a < Nm; ++a) {
        int la = 0;
        while ((la + 1) * (la + 1) <= a) ++la;
        for (int bb = 0; bb < Nm; ++bb) {
            int lb = 0;
            while ((lb + 1) * (lb + 1) <= bb) ++lb;
            double s = 0.0;
            for (int n = 0; n < N; ++n)
                s += ctx->w[n] * Y[(size_t)n * Nm + a] * (2.0 * lb + 1.0) / (4.0 * DCT_PI) * Y[(size_t)n * Nm + bb];
            worst = std::max(worst, std::fabs(s - (a == bb ? 1.0 : 0.0)));
        }
    }
    if (worst > 1e-10)
        return fail(ctx, DCT_ESTATE, "solve: the quadrature does not integrate the P_" + std::to_string(L) +
                                         " moments (|D M - I| = " + std::to_string(worst) + "); lower L or refine S_N");
    pl.cdir.assign(2 * (size_t)N, 0);
    for (int n = 0; n < N; ++n) {
        int c = dir_class(ctx->dirs[3 * n], ctx->dirs[3 * n + 1]);
        pl.cdir[(size_t)c * N + pl.Nc[c]++] = n;
    }
    pl.NcP = 16 * ((std::max(pl.Nc[0], pl.Nc[1]) + 15) / 16);
    if (pl.NcP == 0) pl.NcP = 16;
    pl.NmP = 16 * ((Nm + 15) / 16);
    {
        // the map kernels stage one class's table (padded rows) and its direction slots in LDS
        const size_t lm = (size_t)pl.NcP * (pl.NmP + 1) * pl.tsz, ld = (size_t)pl.NmP * (pl.NcP + 1) * pl.tsz;
        if (std::max(lm, ld) + (size_t)N * 4 > 65536)
            return fail(ctx, DCT_EINVAL, "solve: too many directions per octant class for the moment-map tables (" +
                                             std::to_string(std::max(pl.Nc[0], pl.Nc[1])) + ")");
    }
    if (o.sweep_bk < 0 || o.sweep_bk > 16) return fail(ctx, DCT_EINVAL, "solve: sweep_bk must be in [0, 16]");
    if (o.sweep_sync < 0 || o.sweep_sync > 10) return fail(ctx, DCT_EINVAL, "solve: sweep_sync must be in [0, 10]");
    if (o.sweep_rhs_chain < 0 || o.sweep_rhs_chain > DCT_MAXRC)
        return fail(ctx, DCT_EINVAL, "solve: sweep_rhs_chain must be in [0, " + std::to_string(DCT_MAXRC) + "]");
    if (o.accel_depth < 0 || o.accel_depth > DCT_AA_MAXM)
        return fail(ctx, DCT_EINVAL, "solve: accel_depth must be in [0, " + std::to_string(DCT_AA_MAXM) + "]");
    if (o.rhs_streams < 0 || o.rhs_streams > 2) return fail(ctx, DCT_EINVAL, "solve: rhs_streams must be in [0, 2]");
    if (o.sweep_chain < -1 || o.sweep_chain > DCT_MAXCHAIN)
        return fail(ctx, DCT_EINVAL, "solve: sweep_chain must be in [-1, " + std::to_string(DCT_MAXCHAIN) + "]");
    if (o.superpose < 0 || (o.superpose > 1 && ctx->B % o.superpose != 0))
        return fail(ctx, DCT_EINVAL, "solve: superpose must divide the number of sources (" + std::to_string(ctx->B) + ")");
    if (o.superpose > 1 && o.keep_adjoint)
        return fail(ctx, DCT_EINVAL, "solve: keep_adjoint is not supported with superposed sources");
    set_blocks(pl, o.sweep_bk > 0 ? o.sweep_bk : 16, ctx->ny, ctx->nz);
    return DCT_OK;
}

static float bf16_value(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

static uint16_t bf16_bits(double x)
{
    float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace

extern "C" int dct_solve(dct_ctx *ctx, const dct_opts *opts, dct_stats *stats)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    dct_opts o;
    if (opts) o = *opts;
    else {
        std::memset(&o, 0, sizeof(o));
        o.precision = DCT_FP64;
        o.tol = 1e-6;
        o.max_iter = 1000;
        o.fixup = 1;
    }
    if (ctx->device < 0) return fail(ctx, DCT_EDEVICE, "solve: host-only context (created with device = -1)");
    Plan pl;
    int rc = check_consistency(ctx, o, pl);
    if (rc != DCT_OK) return rc;
    ctx->solved = false;
    HC(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int nx = ctx->nx, ny = ctx->ny, nz = ctx->nz, G = ctx->G, M = ctx->M, L = ctx->L, N = ctx->N;
    // right-hand sides: one per source, or groups of S superposed sources
    const int nsrc = ctx->B, S = o.superpose > 1 ? o.superpose : 1, B = nsrc / S;
    const long C = (long)nx * ny * nz;
    const int Nm = pl.Nm;
    const size_t ts = pl.tsz;
    const int is64 = o.precision == DCT_FP64;
    const int mode = o.precision == DCT_FP64 ? 0 : (o.precision == DCT_FP32 ? 1 : (o.precision == DCT_FP32_BF16X3 ? 3 : 2));

    // ---------------- device buffers
    void *d_mat, *d_rho, *d_st, *d_ss, *d_kap, *d_pos, *d_axis, *d_gw, *d_dirs, *d_w, *d_cdir, *d_Mt, *d_Dt;
    void *d_iso = nullptr, *d_infl = nullptr, *d_fixed = nullptr;
    void *d_phiu, *d_sigc, *d_ext, *d_Qc, *d_q, *d_psi, *d_part, *d_phi, *d_yf, *d_zf, *d_leak, *d_state, *d_bal,
        *d_iters, *d_eps, *d_unf, *d_dose;
    HC(dbuf(ctx, "mat", C, &d_mat));
    HC(dbuf(ctx, "rho", C * 8, &d_rho));
    HC(dbuf(ctx, "st", ctx->st.size() * 8, &d_st));
    HC(dbuf(ctx, "ss", ctx->ss.size() * 8, &d_ss));
    HC(dbuf(ctx, "kap", ctx->kap.size() * 8, &d_kap));
    HC(dbuf(ctx, "pos", ctx->pos.size() * 8, &d_pos));
    HC(dbuf(ctx, "axis", ctx->axis.size() * 8, &d_axis));
    HC(dbuf(ctx, "gw", ctx->gw.size() * 8, &d_gw));
    HC(dbuf(ctx, "dirs", ctx->dirs.size() * 8, &d_dirs));
    HC(dbuf(ctx, "w", ctx->w.size() * 8, &d_w));
    HC(dbuf(ctx, "cdir", pl.cdir.size() * 4, &d_cdir));
    void *d_band;
    HC(dbuf(ctx, "band", (size_t)G * 4, &d_band));
    // bf16 tables: both classes' high parts, then (split mode) both classes' remainders
    const size_t tabsz = (size_t)2 * pl.NcP * pl.NmP * (mode >= 2 ? 2 * (mode == 3 ? 2 : 1) : ts);
    HC(dbuf(ctx, "Mt", tabsz, &d_Mt));
    HC(dbuf(ctx, "Dt", tabsz, &d_Dt));
    if (!ctx->iso.empty()) HC(dbuf(ctx, "iso", ctx->iso.size() * 8, &d_iso));
    if (o.test_inflow) HC(dbuf(ctx, "infl", (size_t)G * 8, &d_infl));
    if (o.fixed_iters) HC(dbuf(ctx, "fixed", (size_t)G * 4, &d_fixed));
    HC(dbuf(ctx, "phiu", (size_t)nsrc * G * C * 8, &d_phiu));
    HC(dbuf(ctx, "sigc", (size_t)2 * G * C * ts, &d_sigc));
    const bool keep = o.keep_adjoint != 0;
    // chain lengths K > 1 whose chains [c K, c K + K) each lie in one octant
    // (chained sweeps: one block, ny <= nx, no kept fluxes)
    std::vector<int> chain_ks;
    if (ny <= 64 && nz <= 16 && !keep && ny <= nx) {
        auto oct = [&](int n) {
            return (ctx->dirs[3 * n] > 0 ? 0 : 1) + (ctx->dirs[3 * n + 1] > 0 ? 0 : 2) + (ctx->dirs[3 * n + 2] > 0 ? 0 : 4);
        };
        for (int K = 2; K <= std::min(N, DCT_MAXCHAIN); ++K) {
            if (N % K) continue;
            bool ok = true;
            for (int n = 0; n < N && ok; ++n) ok = oct(n) == oct(n - n % K);
            if (ok) chain_ks.push_back(K);
        }
    }
    // right-hand sides chained through one sweep workgroup (source-chained
    // sweeps: one block, ny <= nx, nx >= 8, no kept fluxes or test inflow,
    // 32-bit offsets into q and psi)
    std::vector<int> rhs_ks;
    if (ny <= 64 && nz <= 16 && !keep && ny <= nx && nx >= 8 && !o.test_inflow &&
        (size_t)B * N * C * ts <= ((size_t)1 << 31))
        for (int K : {2, 3, 4, 6, 8})
            if (K <= std::min(B, DCT_MAXRC)) rhs_ks.push_back(K);
    void *d_chn0, *d_chxo, *d_sigch = nullptr;
    HC(dbuf(ctx, "chn0", (size_t)N * 4, &d_chn0));
    HC(dbuf(ctx, "chxo", (size_t)N * 4, &d_chxo));
    if (!chain_ks.empty())
        HC(dbuf(ctx, "sigch", (size_t)2 * G * chain_ks.back() * C * ts, &d_sigch));
    HC(dbuf(ctx, "ext", (size_t)B * Nm * C * ts, &d_ext));
    HC(dbuf(ctx, "Qc", (size_t)2 * B * Nm * C * ts, &d_Qc));
    HC(dbuf(ctx, "q", (size_t)B * N * C * ts, &d_q));
    HC(dbuf(ctx, "psi", (size_t)B * (keep ? G : 1) * N * C * ts, &d_psi));
    void *d_mask = nullptr;
    if (keep) HC(dbuf(ctx, "mask", (size_t)B * G * N * C, &d_mask));
    HC(dbuf(ctx, "part", (size_t)2 * B * Nm * C * ts, &d_part));
    HC(dbuf(ctx, "phi", (size_t)B * G * Nm * C * ts, &d_phi));
    // block-face buffers, two copies each (ping-pong by block parity)
    HC(dbuf(ctx, "yf", (size_t)2 * B * N * nx * nz * ts, &d_yf));
    // z faces: per y block a diagonal strip of (nx + 63) x 64 elements
    const size_t zstrip = (size_t)(nx + 63) * 64;
    HC(dbuf(ctx, "zf", (size_t)2 * B * N * pl.NBJ * zstrip * ts, &d_zf));
    // faces handed over inside a pipelined launch: one slot per block boundary
    // (blocks of at least 2 z layers)
    void *d_yfp = nullptr, *d_zfp = nullptr;
    const size_t yfp_bytes = (size_t)B * N * pl.NBJ * nx * nz * ts;
    const size_t zfp_bytes = (size_t)B * N * ((nz + 1) / 2) * pl.NBJ * zstrip * ts;
    void *d_hint = nullptr;
    {
        void *old_y = ctx->bufs["yfp"].p, *old_z = ctx->bufs["zfp"].p, *old_h = ctx->bufs["hint"].p;
        HC(dbuf(ctx, "yfp", yfp_bytes, &d_yfp));
        HC(dbuf(ctx, "zfp", zfp_bytes, &d_zfp));
        HC(dbuf(ctx, "hint", (size_t)B * N * pl.NBJ * ((nz + 1) / 2) * 8, &d_hint));
        if (d_yfp != old_y || d_zfp != old_z) ctx->pipe_clean = false;
        if (d_hint != old_h) HC(hipMemsetAsync(d_hint, 0, (size_t)B * N * pl.NBJ * ((nz + 1) / 2) * 8, s));
    }
    const size_t leak_max = (size_t)B * N * pl.NBJ * nz * 3 * 8;   // any block split (z layers >= 1)
    HC(dbuf(ctx, "leak", leak_max, &d_leak));
    HC(dbuf(ctx, "state", (size_t)B * sizeof(RhsState), &d_state));
    void *d_ccnt;
    HC(dbuf(ctx, "ccnt", (size_t)B * DCT_MAXNM * 128, &d_ccnt));
    // transition kernels: completion sub-counters and per-workgroup balance sums
    const int tr_blocks = (int)((C + 255) / 256), tr_nsub = (tr_blocks + 31) / 32;
    void *d_tsub, *d_pbal;
    HC(dbuf(ctx, "tsub", (size_t)B * tr_nsub * 128, &d_tsub));
    HC(dbuf(ctx, "pbal", (size_t)B * tr_blocks * 16, &d_pbal));
    HC(dbuf(ctx, "bal", (size_t)B * G * 3 * 8, &d_bal));
    HC(dbuf(ctx, "iters", (size_t)B * G * 4, &d_iters));
    HC(dbuf(ctx, "eps", (size_t)B * G * 8, &d_eps));
    HC(dbuf(ctx, "unf", 256, &d_unf));
    void *d_err;
    HC(dbuf(ctx, "err", 256, &d_err));
    HC(dbuf(ctx, "dose", (size_t)B * C * 8, &d_dose));

    // ---------------- inputs: uploaded once, kept on the device until a set_* call
    if (ctx->dev_dirty || ctx->tab_prec != o.precision) {
        std::vector<unsigned char> Mt(tabsz, 0), Dt(tabsz, 0);
        std::vector<int> band;   // host copy alive until the synchronisation below
        std::vector<double> Y(Nm);
        for (int c = 0; c < 2; ++c)
            for (int nl = 0; nl < pl.Nc[c]; ++nl) {
                int n = pl.cdir[(size_t)c * N + nl];
                real_sh_cart<double>(L, ctx->dirs[3 * n], ctx->dirs[3 * n + 1], ctx->dirs[3 * n + 2], Y.data());
                for (int lm = 0; lm < Nm; ++lm) {
                    int l = 0;
                    while ((l + 1) * (l + 1) <= lm) ++l;
                    double mv = (2.0 * l + 1.0) / (4.0 * DCT_PI) * Y[lm];
                    double dv = ctx->w[n] * Y[lm];
                    size_t im = ((size_t)c * pl.NcP + nl) * pl.NmP + lm;
                    size_t id = ((size_t)c * pl.NmP + lm) * pl.NcP + nl;
                    if (mode == 0) {
                        ((double *)Mt.data())[im] = mv;
                        ((double *)Dt.data())[id] = dv;
                    } else if (mode == 1) {
                        ((float *)Mt.data())[im] = (float)mv;
                        ((float *)Dt.data())[id] = (float)dv;
                    } else {
                        ((uint16_t *)Mt.data())[im] = bf16_bits(mv);
                        ((uint16_t *)Dt.data())[id] = bf16_bits(dv);
                        if (mode == 3) {
                            const size_t lo = (size_t)2 * pl.NcP * pl.NmP;
                            ((uint16_t *)Mt.data())[lo + im] = bf16_bits((double)((float)mv - bf16_value(bf16_bits(mv))));
                            ((uint16_t *)Dt.data())[lo + id] = bf16_bits((double)((float)dv - bf16_value(bf16_bits(dv))));
                        }
                    }
                }
            }
        HC(hipMemcpyAsync(d_Mt, Mt.data(), tabsz, hipMemcpyHostToDevice, s));
        HC(hipMemcpyAsync(d_Dt, Dt.data(), tabsz, hipMemcpyHostToDevice, s));
        if (ctx->dev_dirty) {
            HC(hipMemcpyAsync(d_mat, ctx->mat.data(), C, hipMemcpyHostToDevice, s));
            if (!ctx->rho_dev) HC(hipMemcpyAsync(d_rho, ctx->rho.data(), C * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_st, ctx->st.data(), ctx->st.size() * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_ss, ctx->ss.data(), ctx->ss.size() * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_kap, ctx->kap.data(), ctx->kap.size() * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_pos, ctx->pos.data(), ctx->pos.size() * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_axis, ctx->axis.data(), ctx->axis.size() * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_gw, ctx->gw.data(), ctx->gw.size() * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_dirs, ctx->dirs.data(), ctx->dirs.size() * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_w, ctx->w.data(), ctx->w.size() * 8, hipMemcpyHostToDevice, s));
            HC(hipMemcpyAsync(d_cdir, pl.cdir.data(), pl.cdir.size() * 4, hipMemcpyHostToDevice, s));

            // lowest group that scatters into each group in some material and order
            band.assign(G, 0);
            for (int g = 0; g < G; ++g) {
                int lo = g;
                for (int gp = 0; gp < g && lo == g; ++gp)
                    for (int m = 0; m < M && lo == g; ++m)
                        for (int l = 0; l <= L; ++l)
                            if (ctx->ss[(((size_t)m * (L + 1) + l) * G + gp) * G + g] != 0.0) {
                                lo = gp;
                                break;
                            }
                band[g] = lo;
            }
            HC(hipMemcpyAsync(d_band, band.data(), (size_t)G * 4, hipMemcpyHostToDevice, s));
            if (d_iso) HC(hipMemcpyAsync(d_iso, ctx->iso.data(), ctx->iso.size() * 8, hipMemcpyHostToDevice, s));
        }
        HC(hipStreamSynchronize(s));   // host tables must outlive the copies
        ctx->dev_dirty = false;
        ctx->tab_prec = o.precision;
    }
    // per-solve options and the initial state of every right-hand side (small,
    // from pinned host memory so the copies are truly asynchronous)
    {
        size_t need = (size_t)B * sizeof(RhsState) + (size_t)G * 12 + 64;
        if (ctx->h_stage_bytes < need) {
            if (ctx->h_stage) HC(hipHostFree(ctx->h_stage));
            ctx->h_stage = nullptr;
            ctx->h_stage_bytes = 0;
            HC(hipHostMalloc(&ctx->h_stage, need, hipHostMallocDefault));
            ctx->h_stage_bytes = need;
        }
        HC(hipEventSynchronize(ctx->ev_t1));   // the previous solve no longer reads the staging area
        unsigned char *hs = (unsigned char *)ctx->h_stage;
        RhsState *hst = (RhsState *)hs;
        for (int b = 0; b < B; ++b) {
            std::memset(&hst[b], 0, sizeof(RhsState));
            hst[b].pending = 1;
        }
        size_t off = (size_t)B * sizeof(RhsState);
        int *hunf = (int *)(hs + off);
        *hunf = B;
        off += 8;
        HC(hipMemcpyAsync(d_state, hst, (size_t)B * sizeof(RhsState), hipMemcpyHostToDevice, s));
        HC(hipMemcpyAsync(d_unf, hunf, 4, hipMemcpyHostToDevice, s));
        if (d_infl) {
            std::memcpy(hs + off, o.test_inflow, (size_t)G * 8);
            HC(hipMemcpyAsync(d_infl, hs + off, (size_t)G * 8, hipMemcpyHostToDevice, s));
            off += (size_t)G * 8;
        }
        if (d_fixed) {
            std::memcpy(hs + off, o.fixed_iters, (size_t)G * 4);
            HC(hipMemcpyAsync(d_fixed, hs + off, (size_t)G * 4, hipMemcpyHostToDevice, s));
        }
    }
    HC(hipMemsetAsync(d_bal, 0, (size_t)B * G * 3 * 8, s));
    HC(hipMemsetAsync(d_iters, 0, (size_t)B * G * 4, s));
    HC(hipMemsetAsync(d_eps, 0, (size_t)B * G * 8, s));
    HC(hipMemsetAsync(d_leak, 0, leak_max, s));
    HC(hipMemsetAsync(d_err, 0, 4, s));
    HC(hipMemsetAsync(d_ccnt, 0, (size_t)B * DCT_MAXNM * 128, s));
    HC(hipMemsetAsync(d_tsub, 0, (size_t)B * tr_nsub * 128, s));

    Geo geo;
    geo.nx = nx;
    geo.ny = ny;
    geo.nz = nz;
    geo.C = C;
    geo.dx = ctx->dx;
    geo.dy = ctx->dy;
    geo.dz = ctx->dz;
    std::memcpy(geo.org, ctx->org, sizeof(geo.org));

    HC(hipEventRecord(ctx->ev_t0, s));
    HC(launch_sigc(geo, (const uint8_t *)d_mat, (const double *)d_rho, (const double *)d_st, G, M, d_sigc, is64, s));
    {
        TraceArgs ta;
        ta.geo = geo;
        ta.mat = (const uint8_t *)d_mat;
        ta.rho = (const double *)d_rho;
        ta.st = (const double *)d_st;
        ta.G = G;
        ta.M = M;
        ta.B = nsrc;
        ta.pos = (const double *)d_pos;
        ta.axis = (const double *)d_axis;
        ta.half_fan = ctx->fan * DCT_PI / 360.0;
        ta.half_cone = ctx->cone * DCT_PI / 360.0;
        ta.gw = (const double *)d_gw;
        ta.phi_u = (double *)d_phiu;
        HC(launch_trace(ta, s));
    }

    TransArgs tr;
    tr.geo = geo;
    tr.G = G;
    tr.M = M;
    tr.L = L;
    tr.Nm = Nm;
    tr.N = N;
    tr.B = B;
    tr.S = S;
    tr.V = ctx->dx * ctx->dy * ctx->dz;
    tr.mat = (const uint8_t *)d_mat;
    tr.rho = (const double *)d_rho;
    tr.st = (const double *)d_st;
    tr.ss = (const double *)d_ss;
    tr.pos = (const double *)d_pos;
    tr.phi_u = (const double *)d_phiu;
    tr.ext_iso = (const double *)d_iso;
    tr.inflow = (const double *)d_infl;
    tr.band_lo = (const int *)d_band;
    tr.dirs = (const double *)d_dirs;
    tr.w = (const double *)d_w;
    tr.leak_part = (const double *)d_leak;
    tr.nblk = pl.nblk;
    tr.phi_all = d_phi;
    tr.ext = d_ext;
    tr.Qc = d_Qc;
    tr.state = (RhsState *)d_state;
    tr.bal = (double *)d_bal;
    tr.n_unfinished = (int *)d_unf;
    tr.cnt_sub = (unsigned *)d_tsub;
    tr.nsub = tr_nsub;
    tr.part_bal = (double *)d_pbal;
    // warm start: every group starts from the moments the last solve on this
    // context left in the same buffer (same right-hand sides, groups, moments,
    // grid and precision); otherwise from phi = 0
    const bool warm = o.warm_start && ctx->warm.valid && ctx->warm.B == B && ctx->warm.G == G &&
                      ctx->warm.Nm == Nm && ctx->warm.C == C && ctx->warm.prec == o.precision &&
                      ctx->warm.phi == d_phi;
    tr.warm = warm ? 1 : 0;
    // Anderson acceleration of the within-group iteration (depth accel_depth)
    const int aam = o.accel_depth;
    AAArgs aa;
    std::memset(&aa, 0, sizeof(aa));
    tr.aa_phik = nullptr;
    if (aam > 0) {
        const int nblk_aa = (int)((C + 255) / 256), nsub_aa = (nblk_aa + 31) / 32;
        void *t;
        HC(dbuf(ctx, "aa_phik", (size_t)B * C * 8, &t));
        aa.phik = (double *)t;
        HC(dbuf(ctx, "aa_hG", (size_t)B * (aam + 1) * C * 8, &t));
        aa.hG = (double *)t;
        HC(dbuf(ctx, "aa_hF", (size_t)B * (aam + 1) * C * 8, &t));
        aa.hF = (double *)t;
        HC(dbuf(ctx, "aa_part", (size_t)B * nblk_aa * DCT_AA_NDOT * 8, &t));
        aa.part = (double *)t;
        HC(dbuf(ctx, "aa_sub", (size_t)B * nsub_aa * 128, &t));
        aa.cnt_sub = (unsigned *)t;
        HC(hipMemsetAsync(t, 0, (size_t)B * nsub_aa * 128, s));
        HC(dbuf(ctx, "aa_top", (size_t)B * 128, &t));
        aa.cnt_top = (unsigned *)t;
        HC(hipMemsetAsync(t, 0, (size_t)B * 128, s));
        aa.nsub = nsub_aa;
        aa.geo = geo;
        aa.G = G;
        aa.Nm = Nm;
        aa.L = L;
        aa.B = B;
        aa.m = aam;
        aa.reverse = 0;
        aa.state = (RhsState *)d_state;
        aa.mat = (const uint8_t *)d_mat;
        aa.rho = (const double *)d_rho;
        aa.ss = (const double *)d_ss;
        aa.phi_all = d_phi;
        aa.ext = d_ext;
        aa.Qc = d_Qc;
        tr.aa_phik = aa.phik;
    }

    MapArgs ma;
    ma.C = C;
    ma.B = B;
    ma.N = N;
    ma.Nm = Nm;
    ma.Nc[0] = pl.Nc[0];
    ma.Nc[1] = pl.Nc[1];
    ma.cdir = (const int *)d_cdir;
    ma.Mtab = d_Mt;
    ma.Dtab = d_Dt;
    ma.NcP = pl.NcP;
    ma.NmP = pl.NmP;
    ma.Qc = d_Qc;
    ma.q = d_q;
    ma.psi = d_psi;
    ma.psi_bs = keep ? (long)G * N : N;
    ma.psi_gs = keep ? N : 0;
    ma.G = G;
    ma.reverse = 0;
    ma.part = d_part;
    ma.state = (const RhsState *)d_state;
    ma.chainK = 1;
    ma.nx = nx;
    ma.ny = ny;
    ma.chn0 = (const int *)d_chn0;
    ma.chxo = (const int *)d_chxo;
    ma.first_only = 0;

    SweepArgs sw;
    sw.nx = nx;
    sw.ny = ny;
    sw.nz = nz;
    sw.C = C;
    sw.N = N;
    sw.B = B;
    sw.G = G;
    sw.BK = pl.BK;
    sw.NBJ = pl.NBJ;
    sw.NBK = pl.NBK;
    sw.nblk = pl.nblk;
    sw.dirs = (const double *)d_dirs;
    sw.dx = ctx->dx;
    sw.dy = ctx->dy;
    sw.dz = ctx->dz;
    sw.q = d_q;
    sw.psi = d_psi;
    sw.psi_bs = keep ? (long)G * N : N;
    sw.psi_gs = keep ? N : 0;
    sw.mask = (uint8_t *)d_mask;
    sw.reverse = 0;
    sw.adjoint = 0;
    sw.sigc = d_sigc;
    sw.yface = d_yf;
    sw.zface = d_zf;
    sw.leak_part = (double *)d_leak;
    sw.state = (const RhsState *)d_state;
    sw.inflow = (const double *)d_infl;
    sw.fixup = o.fixup;
    sw.sync = o.sweep_sync == 2 ? 0 : 1;
    sw.pipe = 0;
    sw.layers = 0;
    sw.chainK = 1;
    sw.sigch = d_sigch;
    sw.rhsK = 1;
    sw.yface_p = d_yfp;
    sw.zface_p = d_zfp;
    sw.hint = (unsigned long long *)d_hint;
    sw.seq = 0;
    sw.err = (int *)d_err;

    CombArgs cb;
    cb.geo = geo;
    cb.G = G;
    cb.L = L;
    cb.Nm = Nm;
    cb.B = B;
    cb.M = M;
    cb.mat = (const uint8_t *)d_mat;
    cb.rho = (const double *)d_rho;
    cb.ss = (const double *)d_ss;
    cb.part = d_part;
    cb.ext = d_ext;
    cb.phi_all = d_phi;
    cb.Qc = d_Qc;
    cb.state = (RhsState *)d_state;
    cb.iters = (int *)d_iters;
    cb.eps = (double *)d_eps;
    cb.cnt_mom = (unsigned *)d_ccnt;
    // several moments per combine workgroup once there are workgroups to spare
    // (the slab's material and density then stay in the CU's caches)
    cb.mpw = (long)nz * ((ny + 15) / 16) * B * Nm >= 8192 ? 4 : 1;
    cb.fixed_iters = (const int *)d_fixed;
    cb.tol = o.tol;
    cb.max_iter = o.max_iter;
    cb.stall_window = o.precision == DCT_FP64 ? 0 : (o.stall_window == 0 ? 4 : (o.stall_window > 0 ? o.stall_window : 0));
    cb.reverse = 0;
    cb.warm = warm ? 1 : 0;

    auto apply_blocks = [&](int bk) {
        set_blocks(pl, bk, ny, nz);
        sw.BK = pl.BK;
        sw.NBJ = pl.NBJ;
        sw.NBK = pl.NBK;
        sw.nblk = pl.nblk;
        tr.nblk = pl.nblk;
    };
    auto sweep_all = [&]() -> hipError_t {
        for (int d = 0; d < (sw.pipe ? 1 : pl.ndiag); ++d) {
            sw.diag = d;
            hipError_t e = launch_sweep(sw, is64, s, ctx->sweep_seq++);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };

    // ---------------- sweep schedule: given, cached, or timed now
    // schedule = (z layers per workgroup, coupling, chain): coupling 1 = LDS
    // progress counters between the waves of a workgroup, 2 = one barrier per
    // step, 3 = as 2 with every block of a sweep in one launch (pipelined
    // blocks), 4 / 5 = layered waves (every wave sweeps 4 / 2 z layers; one
    // block, ny <= 64 and nz <= 16, forward sweeps), 6 / 7 / 8 = the K
    // consecutive directions of one octant chained through one workgroup,
    // with 1 / 2 / 4 z layers per wave (one block, ny <= nx, forward sweeps
    // without kept fluxes; q and psi in the chain layout), 9 / 10 = one
    // direction of R right-hand sides chained through one workgroup, with 2 / 1
    // z layers per wave (same conditions, class layouts)
    double tune_ms = 0.0;
    const bool layered_ok = ny <= 64 && nz <= 16;
    auto set_coupling = [&](int cpl) {
        sw.sync = cpl == 1;
        sw.pipe = cpl == 3;
        sw.layers = (cpl == 4 && layered_ok) ? 4 : ((cpl == 5 && layered_ok) ? 2 : 0);
        if (cpl >= 6 && cpl <= 8) sw.layers = cpl == 6 ? 1 : (cpl == 7 ? 2 : 4);
        if (cpl >= 9) sw.layers = cpl == 9 ? 2 : 1;
    };
    // q and psi in the layout of chain length K (1 = class layouts), sigma_t
    // copied into it
    std::vector<int> chtab((size_t)2 * N);   // host staging of the chain tables (kept until the solve ends)
    auto set_chain = [&](int K) -> hipError_t {
        ma.chainK = K;
        sw.chainK = K;
        if (K <= 1) return hipSuccess;
        for (int n = 0; n < N; ++n) {
            const int d = n % K;
            chtab[n] = n - d;
            chtab[N + n] = (ctx->dirs[3 * n] > 0 ? d : K - 1 - d) * nx;
        }
        hipError_t e = hipMemcpyAsync(d_chn0, chtab.data(), (size_t)N * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_chxo, chtab.data() + N, (size_t)N * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // the staging vector is refilled by the next call
        if (e != hipSuccess) return e;
        return launch_sigch(geo, d_sigc, G, K, d_sigch, is64, s);
    };
    auto pipe_ready = [&]() -> int {
        // faces handed over inside a launch start out empty (all bits set)
        if (!ctx->pipe_clean) {
            HC(hipMemsetAsync(d_yfp, 0xff, yfp_bytes, s));
            HC(hipMemsetAsync(d_zfp, 0xff, zfp_bytes, s));
            ctx->pipe_clean = true;
        }
        return DCT_OK;
    };
    int chainK = 1, rhsK = 1;
    {
        int bk = o.sweep_bk > 0 ? o.sweep_bk : 16, cpl = o.sweep_sync > 0 ? o.sweep_sync : 1;
        chainK = o.sweep_chain > 1 ? o.sweep_chain :
                 ((cpl >= 6 && cpl <= 8 && !chain_ks.empty()) ? chain_ks.back() : 1);
        rhsK = o.sweep_rhs_chain > 0 ? o.sweep_rhs_chain : std::min(B, 4);
        const bool free_rhs = o.sweep_rhs_chain == 0;
        // chained candidates take part in tuning only when asked for (sweep_chain
        // = -1): the tuner times sweeps alone, and the chain layout also costs
        // the maps some address arithmetic
        const bool free_bk = o.sweep_bk == 0, free_cpl = o.sweep_sync == 0, free_chain = o.sweep_chain < 0;
        if (o.autotune && (free_bk || free_cpl || free_chain)) {
            const dct_ctx::Tuned *hit = nullptr;
            for (const auto &t : ctx->tuned)
                if (t.nx == nx && t.ny == ny && t.nz == nz && t.N == N && t.B == B && t.prec == o.precision &&
                    t.keep == (int)keep)
                    hit = &t;
            if (hit) {
                if (free_bk) bk = hit->bk;
                if (free_cpl) cpl = hit->sync;
                if (free_chain) chainK = hit->chain;
                if (free_rhs) rhsK = hit->rhs;
            } else {
                // first iteration set up to the sweep: the transition sets up
                // group 0 (the first real set then finds nothing pending) and
                // the M map fills q; the candidate sweeps below all compute
                // that same first sweep
                HC(launch_transition(tr, is64, s));
                HC(launch_qinit(cb, is64, s));
                HC(launch_mmap(ma, mode, s));
                while (ctx->evpool.size() < 2) {
                    hipEvent_t ev;
                    HC(hipEventCreate(&ev));
                    ctx->evpool.push_back(ev);
                }
                struct Cand { int bk, cpl, K, R; };
                std::vector<Cand> cands;
                std::vector<int> bks;
                if (free_bk) {
                    for (int c : {16, 8, 4, 2}) {
                        int v = std::min(c, nz);
                        if (std::find(bks.begin(), bks.end(), v) == bks.end()) bks.push_back(v);
                    }
                } else {
                    bks.push_back(std::min(bk, nz));
                }
                for (int cb : bks) {
                    const bool multi = (ny + 63) / 64 > 1 || (nz + cb - 1) / cb > 1;
                    for (int cc : {1, 2, 3, 4, 5, 6, 7, 8, 9, 10}) {
                        if (!free_cpl && cc != cpl) continue;
                        if (cc == 3 && (!multi || cb < 2)) continue;   // pipelining needs several blocks
                        if (cc >= 4 && (!layered_ok || cb != std::min(16, nz))) continue;   // one block of every layer
                        if (cc >= 9) {
                            for (int R : rhs_ks)
                                if (free_rhs || R == rhsK) cands.push_back({cb, cc, 1, R});
                        } else if (cc >= 6) {
                            for (int K : chain_ks)
                                if (free_chain || (K == chainK && o.sweep_chain > 1)) cands.push_back({cb, cc, K, 1});
                        } else if (free_chain || chainK == 1) {
                            cands.push_back({cb, cc, 1, 1});
                        }
                    }
                }
                float best = 1e30f;
                int cur_K = 1;
                for (auto cand : cands) {
                    apply_blocks(cand.bk);
                    set_coupling(cand.cpl);
                    sw.rhsK = cand.R;
                    if (cand.cpl == 3) {
                        int r = pipe_ready();
                        if (r != DCT_OK) return r;
                    }
                    if (cand.K != cur_K) {
                        // q of the first sweep in this candidate's layout
                        HC(set_chain(cand.K));
                        HC(launch_mmap(ma, mode, s));
                        cur_K = cand.K;
                    }
                    HC(sweep_all());   // warm-up
                    HC(hipEventRecord(ctx->evpool[0], s));
                    for (int r = 0; r < 3; ++r) HC(sweep_all());
                    HC(hipEventRecord(ctx->evpool[1], s));
                    HC(hipEventSynchronize(ctx->evpool[1]));
                    int h_err = 0;
                    HC(hipMemcpy(&h_err, d_err, 4, hipMemcpyDeviceToHost));
                    if (h_err) {
                        // a bounded wait gave up: drop this candidate, reset the
                        // flag and the handed-over faces
                        HC(hipMemsetAsync(d_err, 0, 4, s));
                        ctx->pipe_clean = false;
                        continue;
                    }
                    float ms = 0.0f;
                    HC(hipEventElapsedTime(&ms, ctx->evpool[0], ctx->evpool[1]));
                    dlog(3, "tuning candidate: z layers %d, coupling %d, chained directions %d, chained sources %d: "
                            "%.3f ms per sweep", cand.bk, cand.cpl, cand.K, cand.R, ms / 3.0);
                    tune_ms += ms * 4.0 / 3.0;
                    if (ms < best) {
                        best = ms;
                        bk = cand.bk;
                        cpl = cand.cpl;
                        chainK = cand.K;
                        rhsK = cand.R;
                    }
                }
                if (best == 1e30f) return fail(ctx, DCT_EDEVICE, "solve: no sweep schedule completed during tuning");
                ctx->tuned.push_back({nx, ny, nz, N, B, o.precision, (int)keep, bk, cpl, chainK, rhsK});
                tune_cache_save(ctx, ctx->tuned.back());
                dlog(1, "tuned %dx%dx%d N=%d B=%d precision %d: z layers %d, coupling %d, chained directions %d, "
                        "chained sources %d (%.2f ms per sweep)", nx, ny, nz, N, B, o.precision, bk, cpl, chainK, rhsK,
                     best / 3.0);
            }
        }
        apply_blocks(bk);
        if (cpl == 3 && (pl.nblk == 1 || pl.BK < 2)) cpl = 1;   // one block (or 1-layer blocks): not pipelined
        if (cpl >= 4 && cpl <= 5 && (!layered_ok || pl.nblk != 1)) cpl = 2;   // layered waves need one block
        if (cpl >= 6 && cpl <= 8 &&
            (pl.nblk != 1 || std::find(chain_ks.begin(), chain_ks.end(), chainK) == chain_ks.end())) {
            cpl = 2;   // chains need one block and chains inside octants
            chainK = 1;
        }
        if (cpl < 6 || cpl > 8) chainK = 1;
        if (cpl >= 6 && cpl <= 8 && chainK == 1) cpl = 2;
        if (cpl >= 9 && (pl.nblk != 1 || rhs_ks.empty() || rhsK < 2 || rhsK > DCT_MAXRC))
            cpl = 2;   // source chains need one block, several right-hand sides and 32-bit offsets
        if (cpl < 9) rhsK = 1;
        set_coupling(cpl);
        sw.rhsK = rhsK;
        HC(set_chain(chainK));
        if (cpl == 3) {
            int r = pipe_ready();
            if (r != DCT_OK) return r;
        }
        ctx->last_bk = pl.BK;
        ctx->last_sync = cpl;
        ctx->last_chain = chainK;
        ctx->last_rhs = rhsK;
    }

    // D map, combine and M map as one kernel (k_dcm): FP64 / FP32, the slab
    // tile and tables within the workgroup's LDS, at most 32 DCT_MAXNM slabs
    // (completion sub-counters); by default when there are enough slabs to
    // fill the GPU (one or two workgroups per CU at a time)
    bool fused = false;
    int dcm_wg = 0;
    {
        const long nslab = (long)nz * ((ny + 15) / 16);
        const size_t lds = dcm_lds_bytes(cb, ma, is64) + 1024;
        const bool fuse_ok = mode <= 1 && lds <= ctx->lds_max && nslab <= 32L * DCT_MAXNM &&
                             std::max(pl.Nc[0], pl.Nc[1]) <= 48 &&   // one round of psi loads per class
                             (size_t)std::max(N, Nm) * C * ts < ((size_t)1 << 31);   // 32-bit offsets of one
                                                                                      // source's q, psi, ext, phi
        // by default: at least one slab per CU (measured: 36 sources FP64 220
        // against 302 ms, the 128x128x32 abdomen FP32 98 against 109 ms)
        fused = fuse_ok && aam == 0 && (o.fuse_maps > 0 || (o.fuse_maps == 0 && nslab * B >= ctx->ncu));
        ma.first_only = fused ? 1 : 0;
        // persistent workgroups: as many as fit the device at once
        dcm_wg = (2 * lds <= ctx->lds_max ? 2 : 1) * ctx->ncu;
    }
    ctx->last_fused = fused;
    ctx->last_warm = warm;

    // upper bound of iteration sets: every group at its cap plus one transition each
    long cap_sets = 2;
    for (int g = 0; g < G; ++g) cap_sets += (o.fixed_iters ? o.fixed_iters[g] : o.max_iter) + 1;
    const int chunk = o.chunk > 0 ? o.chunk : 4;
    const bool profile = o.profile && !o.use_graph;
    const int pevery = o.profile > 1 ? o.profile : 1;   // time every pevery-th sweep launch
    int nprof = 0, nprof_m = 0;
    long nsweeps = 0, nmaps = 0;
    // right-hand sides in two halves on two streams: one half's sweep (issue-
    // and latency-bound) runs beside the other half's fused kernel (memory-
    // bound); the halves share no data, so each keeps its own order
    int nstreams = 1;
    const bool lw_cpl = ctx->last_sync == 4 || ctx->last_sync == 5;
    const bool rc_cpl = (ctx->last_sync == 9 || ctx->last_sync == 10) && sw.rhsK > 1;
    if (!o.use_graph && fused && ((lw_cpl && B >= 2) || (rc_cpl && B >= 4)) &&
        (o.rhs_streams == 2 || (o.rhs_streams == 0 && (long)B * N >= 4L * ctx->ncu)))
        nstreams = 2;
    ctx->last_streams = nstreams;
    dlog(2, "solve %dx%dx%d N=%d B=%d G=%d precision %d: z layers %d, coupling %d, chained directions %d, "
            "chained sources %d, fused maps %d, streams %d", nx, ny, nz, N, B, G, o.precision, pl.BK, ctx->last_sync,
         ctx->last_chain, ctx->last_rhs, (int)fused, nstreams);
    const int hb = nstreams == 2 ? B / 2 : B;   // first half: right-hand sides 0 .. hb - 1
    // chained sources on two streams: a half's launch keeps the chains per
    // direction of a one-stream launch, ceil(B / R), with fewer sources each
    const int rc_nch = sw.rhsK > 1 ? (B + sw.rhsK - 1) / sw.rhsK : 1;
    auto enqueue_set = [&](hipStream_t es, int b0, int nb) -> hipError_t {
        TransArgs trh = tr;
        CombArgs cbh = cb;
        SweepArgs swh = sw;
        trh.b0 = cbh.b0 = swh.b0 = b0;
        trh.nb = cbh.nb = swh.nb = nb;
        if (swh.rhsK > 1 && nb != B) swh.rhsK = std::max(2, std::min(DCT_MAXRC, (nb + rc_nch - 1) / rc_nch));
        hipError_t e = launch_transition(trh, is64, es);
        if (e != hipSuccess) return e;
        if (fused) {
            // first iteration of a group: q from ext in one pass over the slabs
            if ((e = launch_dcm(cbh, ma, is64, es, 1, dcm_wg)) != hipSuccess) return e;
        } else {
            if ((e = launch_qinit(cb, is64, es)) != hipSuccess) return e;
            if ((e = launch_mmap(ma, mode, es)) != hipSuccess) return e;
        }
        for (int d = 0; d < (swh.pipe ? 1 : pl.ndiag); ++d) {
            swh.diag = d;
            const bool timed = profile && nsweeps++ % pevery == 0;
            if (timed) {
                while ((int)ctx->evpool.size() < 2 * (nprof + 1)) {
                    hipEvent_t ev;
                    if ((e = hipEventCreate(&ev)) != hipSuccess) return e;
                    ctx->evpool.push_back(ev);
                }
                if ((e = hipEventRecord(ctx->evpool[2 * nprof], es)) != hipSuccess) return e;
            }
            if ((e = launch_sweep(swh, is64, es, ctx->sweep_seq++)) != hipSuccess) return e;
            if (timed) {
                if ((e = hipEventRecord(ctx->evpool[2 * nprof + 1], es)) != hipSuccess) return e;
                ++nprof;
            }
        }
        if (fused) {
            const bool timed = profile && nmaps++ % pevery == 0;
            if (timed) {
                while ((int)ctx->evpool_m.size() < 2 * (nprof_m + 1)) {
                    hipEvent_t ev;
                    if ((e = hipEventCreate(&ev)) != hipSuccess) return e;
                    ctx->evpool_m.push_back(ev);
                }
                if ((e = hipEventRecord(ctx->evpool_m[2 * nprof_m], es)) != hipSuccess) return e;
            }
            if ((e = launch_dcm(cbh, ma, is64, es, 0, dcm_wg)) != hipSuccess) return e;
            if (timed) {
                if ((e = hipEventRecord(ctx->evpool_m[2 * nprof_m + 1], es)) != hipSuccess) return e;
                ++nprof_m;
            }
            return hipSuccess;
        }
        if ((e = launch_dmap(ma, mode, es)) != hipSuccess) return e;
        if ((e = launch_combine(cb, is64, es)) != hipSuccess) return e;
        return aam > 0 ? launch_aa(aa, is64, es) : hipSuccess;
    };

    // ---------------- iteration sets: enqueued in chunks (or one captured
    // chunk replayed), the host polls the unfinished count one chunk behind
    hipStream_t ls = s;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphGuard {
        hipGraph_t &g;
        hipGraphExec_t &x;
        ~GraphGuard()
        {
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
        }
    } guard{graph, gexec};
    if (o.use_graph) {
        if (s == nullptr) {
            // the null stream cannot be captured: run the iteration loop on a
            // context-owned stream ordered after everything enqueued so far
            if (!ctx->own_stream) HC(hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
            ls = ctx->own_stream;
            HC(hipEventRecord(ctx->ev_poll[0], s));
            HC(hipStreamWaitEvent(ls, ctx->ev_poll[0], 0));
        }
        HC(hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipSuccess;
        for (int c = 0; c < chunk && ce == hipSuccess; ++c) ce = enqueue_set(ls, 0, B);
        hipError_t ee = hipStreamEndCapture(ls, &graph);
        HC(ce);
        HC(ee);
        HC(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }
    hipStream_t hs = nullptr;   // the second half's stream
    // on an early return (a failed call) the second stream may still run sets
    // on the context's buffers: wait for it, so no later call overlaps them
    struct HalfGuard {
        hipStream_t &h;
        ~HalfGuard()
        {
            if (h) (void)hipStreamSynchronize(h);
        }
    } half_guard{hs};
    if (nstreams == 2) {
        if (!ctx->half_stream) HC(hipStreamCreateWithFlags(&ctx->half_stream, hipStreamNonBlocking));
        for (hipEvent_t &e : ctx->ev_half)
            if (!e) HC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        hs = ctx->half_stream;
        // it starts after everything enqueued on the context's stream so far
        HC(hipEventRecord(ctx->ev_half[0], ls));
        HC(hipStreamWaitEvent(hs, ctx->ev_half[0], 0));
    }
    long sets = 0;
    int kpoll = 0;
    bool done = false;
    while (sets < cap_sets && !done) {
        if (gexec) {
            HC(hipGraphLaunch(gexec, ls));
            sets += chunk;
        } else {
            for (int c = 0; c < chunk && sets < cap_sets; ++c, ++sets) {
                if (hs) {
                    HC(enqueue_set(ls, 0, hb));
                    HC(enqueue_set(hs, hb, B - hb));
                } else {
                    HC(enqueue_set(ls, 0, B));
                }
            }
        }
        if (hs) {
            // the count polled below then covers the second stream up to its
            // previous chunk (the streams stay within a chunk of each other)
            HC(hipEventRecord(ctx->ev_half[1 + (kpoll & 1)], hs));
            if (kpoll > 0) HC(hipStreamWaitEvent(ls, ctx->ev_half[1 + ((kpoll - 1) & 1)], 0));
        }
        HC(hipMemcpyAsync(&ctx->h_unf[kpoll & 1], d_unf, 4, hipMemcpyDeviceToHost, ls));
        HC(hipEventRecord(ctx->ev_poll[kpoll & 1], ls));
        if (kpoll > 0) {
            HC(hipEventSynchronize(ctx->ev_poll[(kpoll - 1) & 1]));
            if (ctx->h_unf[(kpoll - 1) & 1] == 0) done = true;
        }
        ++kpoll;
    }
    if (hs) {
        // join the second stream and take the count once more with both done
        HC(hipEventRecord(ctx->ev_half[0], hs));
        HC(hipStreamWaitEvent(ls, ctx->ev_half[0], 0));
        HC(hipMemcpyAsync(&ctx->h_unf[kpoll & 1], d_unf, 4, hipMemcpyDeviceToHost, ls));
        HC(hipEventRecord(ctx->ev_poll[kpoll & 1], ls));
        ++kpoll;
        hs = nullptr;   // joined
    }
    if (ls != s) HC(hipStreamWaitEvent(s, ctx->ev_poll[(kpoll - 1) & 1], 0));
    HC(hipEventSynchronize(ctx->ev_poll[(kpoll - 1) & 1]));
    int unfinished = ctx->h_unf[(kpoll - 1) & 1];

    DoseArgs da;
    da.C = C;
    da.G = G;
    da.B = B;
    da.S = S;
    da.Nm = Nm;
    da.mat = (const uint8_t *)d_mat;
    da.kap = (const double *)d_kap;
    da.phi_u = (const double *)d_phiu;
    da.phi_all = d_phi;
    da.dose = (double *)d_dose;
    da.phi_c = nullptr;
    da.phi_u_out = nullptr;
    da.summed = 0;
    da.hg = nullptr;
    da.zero_mat = nullptr;
    HC(launch_dose(da, is64, s));
    HC(hipEventRecord(ctx->ev_t1, s));
    HC(hipEventSynchronize(ctx->ev_t1));

    std::vector<RhsState> fin(B);
    HC(hipMemcpy(fin.data(), d_state, (size_t)B * sizeof(RhsState), hipMemcpyDeviceToHost));
    std::vector<int> iters((size_t)B * G);
    HC(hipMemcpy(iters.data(), d_iters, iters.size() * 4, hipMemcpyDeviceToHost));
    int h_err = 0;
    HC(hipMemcpy(&h_err, d_err, 4, hipMemcpyDeviceToHost));
    if (h_err) {
        ctx->solved = false;
        ctx->pipe_clean = false;
        return fail(ctx, DCT_EDEVICE, "solve: a sweep wave wait exceeded its bound (inter-wave synchronisation)");
    }
    int status = DCT_OK;
    bool any_nan = false, any_nc = false;
    for (int b = 0; b < B; ++b) {
        any_nan = any_nan || fin[b].nan;
        any_nc = any_nc || fin[b].notconv;
    }
    if (stats) {
        if (stats->iters) std::memcpy(stats->iters, iters.data(), iters.size() * 4);
        if (stats->eps) HC(hipMemcpy(stats->eps, d_eps, (size_t)B * G * 8, hipMemcpyDeviceToHost));
        if (stats->balance) HC(hipMemcpy(stats->balance, d_bal, (size_t)B * G * 3 * 8, hipMemcpyDeviceToHost));
        long long upd = 0;
        for (size_t i = 0; i < iters.size(); ++i) upd += (long long)iters[i] * C * N;
        stats->sweep_updates = upd;
        float ms = 0;
        HC(hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
        stats->solve_ms = ms;
        double swms = 0;
        for (int i = 0; i < nprof; ++i) {
            float t = 0;
            HC(hipEventElapsedTime(&t, ctx->evpool[2 * i], ctx->evpool[2 * i + 1]));
            swms += t;
        }
        stats->sweep_ms = swms;
        stats->sweep_launches = nprof;
        double mms = 0;
        for (int i = 0; i < nprof_m; ++i) {
            float t = 0;
            HC(hipEventElapsedTime(&t, ctx->evpool_m[2 * i], ctx->evpool_m[2 * i + 1]));
            mms += t;
        }
        stats->fused_ms = mms;
        stats->fused_launches = nprof_m;
        stats->sweep_launches_all = (long long)sets * (sw.pipe ? 1 : pl.ndiag) * nstreams;
        stats->iteration_sets = (int)sets;
        stats->sweep_bk = pl.BK;
        stats->sweep_sync = ctx->last_sync;
        stats->sweep_chain = ctx->last_chain;
        stats->sweep_rhs_chain = ctx->last_rhs;
        stats->rhs_streams = ctx->last_streams;
        stats->fused_maps = ctx->last_fused ? 1 : 0;
        stats->warm_start = ctx->last_warm ? 1 : 0;
        stats->tune_ms = tune_ms;
    }
    if (log_level() >= 2) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1);
        long its = 0;
        for (int v : iters) its += v;
        dlog(2, "solve done: %ld iteration sets, %ld source iterations, %.2f ms on the device, unfinished %d, "
                "non-finite %d, not converged %d", sets, its, ms, unfinished, (int)any_nan, (int)any_nc);
    }
    ctx->solved = true;
    ctx->warm = {!any_nan, B, G, Nm, C, o.precision, d_phi};
    ctx->solved_prec = o.precision;
    ctx->solved_Nm = Nm;
    ctx->solved_S = S;
    ctx->kept = keep;
    if (unfinished != 0) {
        ctx->solved = false;
        return fail(ctx, DCT_ENOTCONV, "solve: iteration-set cap reached with unfinished right-hand sides");
    }
    if (any_nan) status = fail(ctx, DCT_ENUMERIC, "solve: NaN or Inf in a convergence reduction");
    else if (any_nc) status = fail(ctx, DCT_ENOTCONV, "solve: some group stopped at max_iter above tol");
    return status;
}

// hg: per-group fluence-to-dose factors (host, [G]) in place of the kerma
// factors, or null; zmat: per-material flags (host, [M]), nonzero = dose 0
static int dose_common(dct_ctx *ctx, double *dose, int summed, double *phi_u, double *phi_c, bool dev,
                       const double *hg = nullptr, const uint8_t *zmat = nullptr)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (!ctx->solved) return fail(ctx, DCT_ESTATE, "dose: no valid solve since the last set_* call");
    if (!dose && !phi_u && !phi_c) return DCT_OK;
    HC(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const long C = (long)ctx->nx * ctx->ny * ctx->nz;
    const int B = ctx->B / ctx->solved_S, G = ctx->G;
    double *o_dose = dose, *o_pu = phi_u, *o_pc = phi_c;
    if (!dev) {
        void *t;
        if (dose) { HC(dbuf(ctx, "o_dose", (size_t)(summed ? 1 : B) * C * 8, &t)); o_dose = (double *)t; }
        if (phi_u) { HC(dbuf(ctx, "o_pu", (size_t)B * G * C * 8, &t)); o_pu = (double *)t; }
        if (phi_c) { HC(dbuf(ctx, "o_pc", (size_t)B * G * C * 8, &t)); o_pc = (double *)t; }
    }
    double *scratch = nullptr;
    if (!o_dose) {
        void *t;
        HC(dbuf(ctx, "o_scratch", (size_t)B * C * 8, &t));
        scratch = (double *)t;
    }
    DoseArgs da;
    da.C = C;
    da.G = G;
    da.B = B;
    da.S = ctx->solved_S;
    da.Nm = ctx->solved_Nm;
    da.mat = (const uint8_t *)ctx->bufs["mat"].p;
    da.kap = (const double *)ctx->bufs["kap"].p;
    da.phi_u = (const double *)ctx->bufs["phiu"].p;
    da.phi_all = ctx->bufs["phi"].p;
    da.dose = o_dose ? o_dose : scratch;
    da.phi_c = o_pc;
    da.phi_u_out = o_pu;
    da.summed = o_dose ? summed : 0;
    da.hg = nullptr;
    da.zero_mat = nullptr;
    if (hg) {
        void *t;
        HC(dbuf(ctx, "o_hg", (size_t)G * 8, &t));
        HC(hipMemcpyAsync(t, hg, (size_t)G * 8, hipMemcpyHostToDevice, s));
        da.hg = (const double *)t;
    }
    if (zmat) {
        void *t;
        HC(dbuf(ctx, "o_zmat", (size_t)ctx->M, &t));
        HC(hipMemcpyAsync(t, zmat, (size_t)ctx->M, hipMemcpyHostToDevice, s));
        da.zero_mat = (const uint8_t *)t;
    }
    HC(launch_dose(da, ctx->solved_prec == DCT_FP64, s));
    if ((hg || zmat) && dev) HC(hipStreamSynchronize(s));   // the host tables are the caller's
    if (!dev) {
        if (dose) HC(hipMemcpyAsync(dose, o_dose, (size_t)(summed ? 1 : B) * C * 8, hipMemcpyDeviceToHost, s));
        if (phi_u) HC(hipMemcpyAsync(phi_u, o_pu, (size_t)B * G * C * 8, hipMemcpyDeviceToHost, s));
        if (phi_c) HC(hipMemcpyAsync(phi_c, o_pc, (size_t)B * G * C * 8, hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
    }
    return DCT_OK;
}

extern "C" int dct_dose(dct_ctx *ctx, double *dose, int summed, double *phi_u, double *phi_c)
{
    return dose_common(ctx, dose, summed, phi_u, phi_c, false);
}

extern "C" int dct_dose_dev(dct_ctx *ctx, double *dose, int summed, double *phi_u, double *phi_c)
{
    return dose_common(ctx, dose, summed, phi_u, phi_c, true);
}

// R = sum_b sum_v roi[v] dose_b(v) of the last solve from ROI weights already
// on the device: the summed dose tally, then a fixed-order FP64 dot product;
// returns with R written.
static int roi_response(dct_ctx *ctx, const double *d_roi, double *R)
{
    const long C = (long)ctx->nx * ctx->ny * ctx->nz;
    hipStream_t s = ctx->stream;
    void *dd, *dp;
    HC(dbuf(ctx, "r_dose", (size_t)C * 8, &dd));
    HC(dbuf(ctx, "r_part", (size_t)1025 * 8, &dp));
    const int r = dose_common(ctx, (double *)dd, 1, nullptr, nullptr, true);
    if (r != DCT_OK) return r;
    HC(launch_wdot(d_roi, (const double *)dd, C, (double *)dp, s));
    const int nb = (int)std::min<long>(1024, std::max<long>(1, (C + 255) / 256));
    HC(hipMemcpyAsync(R, (double *)dp + nb, 8, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    return DCT_OK;
}

extern "C" int dct_roi_dose(dct_ctx *ctx, const double *roi, double *R)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (!roi || !R) return fail(ctx, DCT_EINVAL, "roi_dose: NULL array");
    if (!ctx->solved) return fail(ctx, DCT_ESTATE, "roi_dose: no valid solve since the last set_* call");
    const long C = (long)ctx->nx * ctx->ny * ctx->nz;
    if (!finite_all(roi, C)) return fail(ctx, DCT_EINVAL, "roi_dose: roi not finite");
    HC(hipSetDevice(ctx->device));
    void *dr;
    HC(dbuf(ctx, "r_roi", (size_t)C * 8, &dr));
    HC(hipMemcpyAsync(dr, roi, (size_t)C * 8, hipMemcpyHostToDevice, ctx->stream));
    return roi_response(ctx, (const double *)dr, R);
}

// Checks of dct_effective_dose's table and its per-group factors: the table
// at each group's mid energy, linear between points, the end value beyond
// either end (Sec. III-A).
static int effective_dose_factors(dct_ctx *ctx, const char *who, int n, const double *energy_keV,
                                  const double *factor, const void *out, std::vector<double> &hg)
{
    const std::string w(who);
    if (!ctx->solved) return fail(ctx, DCT_ESTATE, w + ": no valid solve since the last set_* call");
    if ((int)ctx->edges.size() != ctx->G + 1)
        return fail(ctx, DCT_ESTATE, w + ": the group edges were not given to dct_set_xs");
    if (n < 1 || !energy_keV || !factor || !out) return fail(ctx, DCT_EINVAL, w + ": empty table or NULL");
    if (!finite_all(energy_keV, n) || !finite_all(factor, n))
        return fail(ctx, DCT_EINVAL, w + ": non-finite table entry");
    for (int i = 0; i + 1 < n; ++i)
        if (!(energy_keV[i] < energy_keV[i + 1]))
            return fail(ctx, DCT_EINVAL, w + ": table energies must be strictly increasing");
    hg.assign(ctx->G, 0.0);
    for (int g = 0; g < ctx->G; ++g) {
        const double e = 0.5 * (ctx->edges[g] + ctx->edges[g + 1]);
        double h;
        if (e <= energy_keV[0]) h = factor[0];
        else if (e >= energy_keV[n - 1]) h = factor[n - 1];
        else {
            int i = 0;
            while (energy_keV[i + 1] < e) ++i;
            const double t = (e - energy_keV[i]) / (energy_keV[i + 1] - energy_keV[i]);
            h = factor[i] + t * (factor[i + 1] - factor[i]);
        }
        hg[g] = h;
    }
    return DCT_OK;
}

extern "C" int dct_effective_dose(dct_ctx *ctx, int n, const double *energy_keV, const double *factor,
                                  const uint8_t *zero_material, double *out, int summed)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    std::vector<double> hg;
    const int rc = effective_dose_factors(ctx, "effective_dose", n, energy_keV, factor, out, hg);
    if (rc != DCT_OK) return rc;
    return dose_common(ctx, out, summed, nullptr, nullptr, false, hg.data(), zero_material);
}

extern "C" int dct_effective_dose_noalloc(dct_ctx *ctx, int n, const double *energy_keV, const double *factor,
                                          const uint8_t *zero_material, double *out_dev, int summed)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (ctx->device < 0) return fail(ctx, DCT_EDEVICE, "effective_dose_noalloc: host-only context");
    if (ctx->G > DCT_NOALLOC_MAXG || ctx->M > DCT_MAXMAT)
        return fail(ctx, DCT_EINVAL, "effective_dose_noalloc: at most " + std::to_string(DCT_NOALLOC_MAXG) +
                                         " groups and " + std::to_string(DCT_MAXMAT) +
                                         " materials fit the fixed scratch (G = " + std::to_string(ctx->G) + ")");
    std::vector<double> hg;
    const int rc = effective_dose_factors(ctx, "effective_dose_noalloc", n, energy_keV, factor, out_dev, hg);
    if (rc != DCT_OK) return rc;
    HC(hipSetDevice(ctx->device));
    unsigned char *sp = (unsigned char *)scratch_dev(ctx->device);
    if (!sp) return fail(ctx, DCT_EDEVICE, "effective_dose_noalloc: the device scratch was not resolved");
    hipStream_t s = ctx->stream;
    const long C = (long)ctx->nx * ctx->ny * ctx->nz;
    // the factors and flags travel as kernel arguments into the scratch (no
    // host buffer is read after this call returns, nothing is allocated)
    StageConsts sc;
    std::memset(&sc, 0, sizeof(sc));
    sc.nd = ctx->G;
    for (int g = 0; g < ctx->G; ++g) sc.d[g] = hg[g];
    sc.nb = zero_material ? ctx->M : 0;
    for (int m = 0; m < sc.nb; ++m) sc.b[m] = zero_material[m];
    HC(launch_stage_consts(sc, (double *)sp, sp + DCT_NOALLOC_ZOFF, s));
    DoseArgs da;
    da.C = C;
    da.G = ctx->G;
    da.B = ctx->B / ctx->solved_S;
    da.S = ctx->solved_S;
    da.Nm = ctx->solved_Nm;
    da.mat = (const uint8_t *)ctx->bufs["mat"].p;
    da.kap = (const double *)ctx->bufs["kap"].p;
    da.phi_u = (const double *)ctx->bufs["phiu"].p;
    da.phi_all = ctx->bufs["phi"].p;
    da.dose = out_dev;
    da.phi_c = nullptr;
    da.phi_u_out = nullptr;
    da.summed = summed;
    da.hg = (const double *)sp;
    da.zero_mat = zero_material ? (const uint8_t *)(sp + DCT_NOALLOC_ZOFF) : nullptr;
    HC(launch_dose(da, ctx->solved_prec == DCT_FP64, s));
    return DCT_OK;
}

extern "C" int dct_moments(dct_ctx *ctx, double *phi)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (!ctx->solved) return fail(ctx, DCT_ESTATE, "moments: no valid solve since the last set_* call");
    if (!phi) return fail(ctx, DCT_EINVAL, "moments: NULL output");
    HC(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const long n = (long)(ctx->B / ctx->solved_S) * ctx->G * ctx->solved_Nm * ctx->nx * ctx->ny * ctx->nz;
    void *t;
    HC(dbuf(ctx, "o_mom", (size_t)n * 8, &t));
    HC(launch_moments_out(ctx->bufs["phi"].p, n, (double *)t, ctx->solved_prec == DCT_FP64, s));
    HC(hipMemcpyAsync(phi, t, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    return DCT_OK;
}

// ---------------------------------------------------------------- adjoint
// The adjoint solve; dev: roi, d_density and d_group_w are device buffers.
static int adjoint_common(dct_ctx *ctx, const double *roi, const dct_opts *opts, double *R, double *d_density,
                          double *d_group_w, dct_stats *stats, bool dev)
{
    if (!ctx) return DCT_EINVAL;
    ctx->err.clear();
    if (!ctx->solved || !ctx->kept)
        return fail(ctx, DCT_ESTATE, "adjoint: needs a preceding dct_solve with keep_adjoint = 1 and no set_* since");
    if (!roi) return fail(ctx, DCT_EINVAL, "adjoint: roi is NULL");
    const int nx = ctx->nx, ny = ctx->ny, nz = ctx->nz, G = ctx->G, M = ctx->M, L = ctx->L, N = ctx->N, B = ctx->B;
    const long C = (long)nx * ny * nz;
    if (!dev && !finite_all(roi, C)) return fail(ctx, DCT_EINVAL, "adjoint: roi not finite");
    if (dev) {
        HC(hipSetDevice(ctx->device));
        void *d_bad;
        HC(dbuf(ctx, "scr_bad", 8, &d_bad));
        HC(hipMemsetAsync(d_bad, 0xff, 8, ctx->stream));
        HC(launch_screen(roi, C, 0, (unsigned long long *)d_bad, ctx->stream));
        unsigned long long bad = 0;
        HC(hipMemcpyAsync(&bad, d_bad, 8, hipMemcpyDeviceToHost, ctx->stream));
        HC(hipStreamSynchronize(ctx->stream));
        if (bad != ~0ULL) return fail(ctx, DCT_EINVAL, "adjoint: roi not finite (voxel " + std::to_string(bad) + ")");
    }
    dct_opts o;
    std::memset(&o, 0, sizeof(o));
    o.tol = 1e-6;
    o.max_iter = 1000;
    if (opts) {
        o.tol = opts->tol;
        o.max_iter = opts->max_iter;
        o.fixed_iters = opts->fixed_iters;
        o.chunk = opts->chunk;
    }
    o.precision = ctx->solved_prec;
    o.fixup = 1;
    Plan pl;
    int rc = check_consistency(ctx, o, pl);
    if (rc != DCT_OK) return rc;
    set_blocks(pl, ctx->last_bk, ctx->ny, ctx->nz);   // the forward solve's sweep schedule
    HC(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int Nm = pl.Nm;
    const size_t ts = pl.tsz;
    const int is64 = o.precision == DCT_FP64;
    const int mode = o.precision == DCT_FP64 ? 0 : (o.precision == DCT_FP32 ? 1 : (o.precision == DCT_FP32_BF16X3 ? 3 : 2));
    auto B_ = [&](const char *n) { return ctx->bufs[n].p; };

    void *d_roi, *d_amt, *d_adt, *d_lamc, *d_lam, *d_pbar, *d_pbu, *d_drho, *d_dray, *d_dgw, *d_ait, *d_aeps, *d_fix;
    HC(dbuf(ctx, "a_roi", (size_t)C * 8, &d_roi));
    // bf16 tables: both classes' high parts, then (split mode) both classes' remainders
    const size_t tabsz = (size_t)2 * pl.NcP * pl.NmP * (mode >= 2 ? 2 * (mode == 3 ? 2 : 1) : ts);
    HC(dbuf(ctx, "a_Mt", tabsz, &d_amt));
    HC(dbuf(ctx, "a_Dt", tabsz, &d_adt));
    HC(dbuf(ctx, "a_lamc", (size_t)B * N * C * ts, &d_lamc));
    HC(dbuf(ctx, "a_lam", (size_t)B * G * Nm * C * ts, &d_lam));
    HC(dbuf(ctx, "a_pbar", (size_t)B * Nm * C * ts, &d_pbar));
    HC(dbuf(ctx, "a_pbu", (size_t)B * G * C * 8, &d_pbu));
    HC(dbuf(ctx, "a_drho", (size_t)B * C * 8, &d_drho));
    HC(dbuf(ctx, "a_dray", (size_t)C * 8, &d_dray));
    HC(dbuf(ctx, "a_dgw", (size_t)G * 8, &d_dgw));
    HC(dbuf(ctx, "a_iters", (size_t)B * G * 4, &d_ait));
    HC(dbuf(ctx, "a_eps", (size_t)B * G * 8, &d_aeps));
    HC(dbuf(ctx, "a_fixed", (size_t)G * 4, &d_fix));

    // transposed maps: the "M" slot gets D^T (moments -> direction weights) and the
    // "D" slot gets M^T (direction weights -> moments)
    std::vector<unsigned char> Mt(tabsz, 0), Dt(tabsz, 0);
    {
        std::vector<double> Y(Nm);
        for (int c = 0; c < 2; ++c)
            for (int nl = 0; nl < pl.Nc[c]; ++nl) {
                int n = pl.cdir[(size_t)c * N + nl];
                real_sh_cart<double>(L, ctx->dirs[3 * n], ctx->dirs[3 * n + 1], ctx->dirs[3 * n + 2], Y.data());
                for (int lm = 0; lm < Nm; ++lm) {
                    int l = 0;
                    while ((l + 1) * (l + 1) <= lm) ++l;
                    double dT = ctx->w[n] * Y[lm];                         // D[lm][n] at (n, lm)
                    double mT = (2.0 * l + 1.0) / (4.0 * DCT_PI) * Y[lm]; // M[n][lm] at (lm, n)
                    size_t im = ((size_t)c * pl.NcP + nl) * pl.NmP + lm;
                    size_t id = ((size_t)c * pl.NmP + lm) * pl.NcP + nl;
                    if (mode == 0) {
                        ((double *)Mt.data())[im] = dT;
                        ((double *)Dt.data())[id] = mT;
                    } else if (mode == 1) {
                        ((float *)Mt.data())[im] = (float)dT;
                        ((float *)Dt.data())[id] = (float)mT;
                    } else {
                        ((uint16_t *)Mt.data())[im] = bf16_bits(dT);
                        ((uint16_t *)Dt.data())[id] = bf16_bits(mT);
                        if (mode == 3) {
                            const size_t lo = (size_t)2 * pl.NcP * pl.NmP;
                            ((uint16_t *)Mt.data())[lo + im] = bf16_bits((double)((float)dT - bf16_value(bf16_bits(dT))));
                            ((uint16_t *)Dt.data())[lo + id] = bf16_bits((double)((float)mT - bf16_value(bf16_bits(mT))));
                        }
                    }
                }
            }
    }
    std::vector<RhsState> hst(B);
    for (int b = 0; b < B; ++b) {
        std::memset(&hst[b], 0, sizeof(RhsState));
        hst[b].pending = 1;
    }
    int h_unf0 = B;
    HC(hipMemcpyAsync(d_roi, roi, (size_t)C * 8, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    HC(hipMemcpyAsync(d_amt, Mt.data(), tabsz, hipMemcpyHostToDevice, s));
    HC(hipMemcpyAsync(d_adt, Dt.data(), tabsz, hipMemcpyHostToDevice, s));
    HC(hipMemcpyAsync(B_("state"), hst.data(), (size_t)B * sizeof(RhsState), hipMemcpyHostToDevice, s));
    HC(hipMemcpyAsync(B_("unf"), &h_unf0, 4, hipMemcpyHostToDevice, s));
    if (o.fixed_iters) HC(hipMemcpyAsync(d_fix, o.fixed_iters, (size_t)G * 4, hipMemcpyHostToDevice, s));
    HC(hipMemsetAsync(d_drho, 0, (size_t)B * C * 8, s));
    HC(hipMemsetAsync(d_dray, 0, (size_t)C * 8, s));
    HC(hipMemsetAsync(d_dgw, 0, (size_t)G * 8, s));
    HC(hipMemsetAsync(d_ait, 0, (size_t)B * G * 4, s));
    HC(hipMemsetAsync(d_aeps, 0, (size_t)B * G * 8, s));
    HC(hipMemsetAsync(B_("err"), 0, 4, s));
    HC(hipMemsetAsync(B_("ccnt"), 0, (size_t)B * DCT_MAXNM * 128, s));
    const int tr_nsub = (int)(((C + 255) / 256 + 31) / 32);
    HC(hipMemsetAsync(B_("tsub"), 0, (size_t)B * tr_nsub * 128, s));
    HC(launch_adj_init(C, G, B, (const uint8_t *)B_("mat"), (const double *)B_("kap"), (const double *)d_roi,
                       (double *)d_pbu, s));
    HC(hipStreamSynchronize(s));   // host tables must outlive the copies
    if (R) {
        // the response of the forward solve, reduced as dct_roi_dose does
        const int r = roi_response(ctx, (const double *)d_roi, R);
        if (r != DCT_OK) return r;
    }

    Geo geo;
    geo.nx = nx;
    geo.ny = ny;
    geo.nz = nz;
    geo.C = C;
    geo.dx = ctx->dx;
    geo.dy = ctx->dy;
    geo.dz = ctx->dz;
    std::memcpy(geo.org, ctx->org, sizeof(geo.org));

    AdjTransArgs at;
    at.geo = geo;
    at.G = G;
    at.M = M;
    at.L = L;
    at.Nm = Nm;
    at.N = N;
    at.B = B;
    at.mat = (const uint8_t *)B_("mat");
    at.rho = (const double *)B_("rho");
    at.st = (const double *)B_("st");
    at.ss = (const double *)B_("ss");
    at.kap = (const double *)B_("kap");
    at.pos = (const double *)B_("pos");
    at.roi = (const double *)d_roi;
    at.phi_u = (const double *)B_("phiu");
    at.phi_all = B_("phi");
    at.psi_keep = B_("psi");
    at.lamc = d_lamc;
    at.dirs = (const double *)B_("dirs");
    at.lam_all = d_lam;
    at.phibar = d_pbar;
    at.Qc = B_("Qc");
    at.pbu = (double *)d_pbu;
    at.drho = (double *)d_drho;
    at.state = (RhsState *)B_("state");
    at.n_unfinished = (int *)B_("unf");
    at.cnt_sub = (unsigned *)B_("tsub");
    at.nsub = tr_nsub;

    MapArgs ma;
    ma.C = C;
    ma.B = B;
    ma.N = N;
    ma.Nm = Nm;
    ma.Nc[0] = pl.Nc[0];
    ma.Nc[1] = pl.Nc[1];
    ma.cdir = (const int *)B_("cdir");
    ma.Mtab = d_amt;
    ma.Dtab = d_adt;
    ma.NcP = pl.NcP;
    ma.NmP = pl.NmP;
    ma.Qc = B_("Qc");
    ma.q = B_("q");
    ma.psi = d_lamc;
    ma.psi_bs = N;
    ma.psi_gs = 0;
    ma.G = G;
    ma.reverse = 1;
    ma.part = B_("part");
    ma.state = (const RhsState *)B_("state");
    ma.chainK = 1;
    ma.nx = nx;
    ma.ny = ny;
    ma.chn0 = nullptr;
    ma.chxo = nullptr;
    ma.first_only = 0;

    SweepArgs sw;
    sw.nx = nx;
    sw.ny = ny;
    sw.nz = nz;
    sw.C = C;
    sw.N = N;
    sw.B = B;
    sw.G = G;
    sw.BK = pl.BK;
    sw.NBJ = pl.NBJ;
    sw.NBK = pl.NBK;
    sw.nblk = pl.nblk;
    sw.dirs = (const double *)B_("dirs");
    sw.dx = ctx->dx;
    sw.dy = ctx->dy;
    sw.dz = ctx->dz;
    sw.q = B_("q");
    sw.psi = d_lamc;
    sw.psi_bs = N;
    sw.psi_gs = 0;
    sw.mask = (uint8_t *)B_("mask");
    sw.reverse = 1;
    sw.adjoint = 1;
    sw.sigc = B_("sigc");
    sw.yface = B_("yf");
    sw.zface = B_("zf");
    sw.leak_part = (double *)B_("leak");
    sw.state = (const RhsState *)B_("state");
    sw.inflow = nullptr;
    sw.fixup = 0;
    sw.sync = ctx->last_sync == 1;
    sw.pipe = ctx->last_sync == 3;
    sw.layers = 0;                     // transposed sweeps run on k_sweep (barrier coupling for layered schedules)
    sw.chainK = 1;
    sw.rhsK = 1;
    sw.sigch = nullptr;
    sw.yface_p = B_("yfp");
    sw.zface_p = B_("zfp");
    sw.hint = (unsigned long long *)B_("hint");
    sw.seq = 0;
    sw.err = (int *)B_("err");

    CombArgs cb;
    cb.geo = geo;
    cb.G = G;
    cb.L = L;
    cb.Nm = Nm;
    cb.B = B;
    cb.M = M;
    cb.mat = (const uint8_t *)B_("mat");
    cb.rho = (const double *)B_("rho");
    cb.ss = (const double *)B_("ss");
    cb.part = B_("part");
    cb.ext = d_pbar;
    cb.phi_all = d_lam;
    cb.Qc = B_("Qc");
    cb.state = (RhsState *)B_("state");
    cb.iters = (int *)d_ait;
    cb.eps = (double *)d_aeps;
    cb.cnt_mom = (unsigned *)B_("ccnt");
    cb.mpw = (long)nz * ((ny + 15) / 16) * B * Nm >= 8192 ? 4 : 1;
    cb.fixed_iters = o.fixed_iters ? (const int *)d_fix : nullptr;
    cb.tol = o.tol;
    cb.max_iter = o.max_iter;
    cb.stall_window = o.precision == DCT_FP64 ? 0 : (o.stall_window == 0 ? 4 : (o.stall_window > 0 ? o.stall_window : 0));
    cb.reverse = 1;
    cb.warm = 0;

    long cap_sets = 2;
    for (int g = 0; g < G; ++g) cap_sets += (o.fixed_iters ? o.fixed_iters[g] : o.max_iter) + 1;
    const int chunk = o.chunk > 0 ? o.chunk : 4;
    auto enqueue_set = [&]() -> hipError_t {
        hipError_t e = launch_adj_transition(at, is64, s);
        if (e != hipSuccess) return e;
        if ((e = launch_qinit(cb, is64, s)) != hipSuccess) return e;
        if ((e = launch_mmap(ma, mode, s)) != hipSuccess) return e;
        for (int d = 0; d < (sw.pipe ? 1 : pl.ndiag); ++d) {
            sw.diag = d;
            if ((e = launch_sweep(sw, is64, s, ctx->sweep_seq++)) != hipSuccess) return e;
        }
        if ((e = launch_dmap(ma, mode, s)) != hipSuccess) return e;
        return launch_combine(cb, is64, s);
    };
    HC(hipEventRecord(ctx->ev_t0, s));
    long sets = 0;
    int kpoll = 0;
    bool done = false;
    while (sets < cap_sets && !done) {
        for (int c = 0; c < chunk && sets < cap_sets; ++c, ++sets) HC(enqueue_set());
        HC(hipMemcpyAsync(&ctx->h_unf[kpoll & 1], B_("unf"), 4, hipMemcpyDeviceToHost, s));
        HC(hipEventRecord(ctx->ev_poll[kpoll & 1], s));
        if (kpoll > 0) {
            HC(hipEventSynchronize(ctx->ev_poll[(kpoll - 1) & 1]));
            if (ctx->h_unf[(kpoll - 1) & 1] == 0) done = true;
        }
        ++kpoll;
    }
    HC(hipEventSynchronize(ctx->ev_poll[(kpoll - 1) & 1]));
    const int unfinished = ctx->h_unf[(kpoll - 1) & 1];

    AdjRayArgs ar;
    ar.geo = geo;
    ar.mat = (const uint8_t *)B_("mat");
    ar.rho = (const double *)B_("rho");
    ar.st = (const double *)B_("st");
    ar.G = G;
    ar.M = M;
    ar.B = B;
    ar.pos = (const double *)B_("pos");
    ar.axis = (const double *)B_("axis");
    ar.half_fan = ctx->fan * DCT_PI / 360.0;
    ar.half_cone = ctx->cone * DCT_PI / 360.0;
    ar.gw = (const double *)B_("gw");
    ar.pbu = (const double *)d_pbu;
    ar.drho_ray = (double *)d_dray;
    ar.dgw = (double *)d_dgw;
    HC(launch_adj_ray(ar, s));
    HC(hipEventRecord(ctx->ev_t1, s));
    HC(hipEventSynchronize(ctx->ev_t1));
    int h_err = 0;
    HC(hipMemcpy(&h_err, B_("err"), 4, hipMemcpyDeviceToHost));
    if (h_err) {
        ctx->pipe_clean = false;
        return fail(ctx, DCT_EDEVICE, "adjoint: a sweep wave wait exceeded its bound");
    }
    if (unfinished != 0) return fail(ctx, DCT_ENOTCONV, "adjoint: iteration-set cap reached");

    if (dev) {
        if (d_density) HC(launch_adj_gather((const double *)d_drho, (const double *)d_dray, C, B, d_density, s));
        if (d_group_w) HC(hipMemcpyAsync(d_group_w, d_dgw, (size_t)G * 8, hipMemcpyDeviceToDevice, s));
        HC(hipStreamSynchronize(s));
    } else if (d_density || d_group_w) {
        std::vector<double> drho((size_t)B * C), dray(C);
        HC(hipMemcpy(drho.data(), d_drho, drho.size() * 8, hipMemcpyDeviceToHost));
        HC(hipMemcpy(dray.data(), d_dray, dray.size() * 8, hipMemcpyDeviceToHost));
        if (d_density)
            for (long v = 0; v < C; ++v) {
                double t = dray[v];
                for (int b = 0; b < B; ++b) t += drho[(size_t)b * C + v];
                d_density[v] = t;
            }
        if (d_group_w) HC(hipMemcpy(d_group_w, d_dgw, (size_t)G * 8, hipMemcpyDeviceToHost));
    }
    if (stats) {
        if (stats->iters) HC(hipMemcpy(stats->iters, d_ait, (size_t)B * G * 4, hipMemcpyDeviceToHost));
        if (stats->eps) HC(hipMemcpy(stats->eps, d_aeps, (size_t)B * G * 8, hipMemcpyDeviceToHost));
        float ms = 0;
        HC(hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
        stats->solve_ms = ms;
        stats->iteration_sets = (int)sets;
    }
    return DCT_OK;
}

extern "C" int dct_adjoint(dct_ctx *ctx, const double *roi, const dct_opts *opts, double *R, double *d_density,
                           double *d_group_w, dct_stats *stats)
{
    return adjoint_common(ctx, roi, opts, R, d_density, d_group_w, stats, false);
}

extern "C" int dct_adjoint_dev(dct_ctx *ctx, const double *roi, const dct_opts *opts, double *R, double *d_density,
                               double *d_group_w, dct_stats *stats)
{
    return adjoint_common(ctx, roi, opts, R, d_density, d_group_w, stats, true);
}
