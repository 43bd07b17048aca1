// The preconditioner application without any allocation: the temporaries of
// msrsb_apply_preconditioner live in one file-scope device array instead of
// the context's workspace, for callers that may not allocate device memory
// at the time of the call (inside HIP graph capture, tight serving loops).
//
// Every device holds its own copy of the array for the life of the process;
// its device address is looked up once per device, when the first context is
// created there (static_scratch_init), and host code uses only that address,
// never the array's name.  All calls on one device share the array, so calls
// that overlap on one device race; each call overwrites whatever the
// previous one left there.
#include <mutex>

#include "internal.h"
#include "solve.h"

namespace msrsb {
namespace {

// Layout of the array, in doubles, each region rounded up to 256 bytes:
// three FP64 fine vectors, three FP32 fine vectors (as doubles: half as
// many), the two coarse vectors and the partials of the coarse product.
constexpr int64_t round32(int64_t x) { return (x + 31) / 32 * 32; }
constexpr int64_t kRegionF64 = round32(kNoAllocMaxN);
constexpr int64_t kRegionF32 = round32(kNoAllocMaxN / 2);
constexpr int64_t kRegionCoarse = round32(kMaxCoarse);
constexpr int64_t kRegionPart = round32(64 * static_cast<int64_t>(kMaxCoarse) + 64);
constexpr int64_t kScratchDoubles =
    3 * kRegionF64 + 3 * kRegionF32 + 2 * kRegionCoarse + kRegionPart;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double *g_scratch[kMaxDevices] = {};

}  // namespace

// Device address of this device's scratch array; looked up on the first call
// for the device (which must be current).  Null if the lookup failed.
double *static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch[device] = static_cast<double *>(p);
    }
    return g_scratch[device];
}

}  // namespace msrsb

using namespace msrsb;

extern "C" msrsb_status msrsb_apply_preconditioner_noalloc(msrsb_ctx *c,
                                                           const msrsb_solve_opts *o,
                                                           const double *v, double *z)
{
    if (!c) return MSRSB_E_ARG;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != c->device) hipSetDevice(c->device);
    auto done = [&](msrsb_status st, const char *msg) {
        if (msg) c->err = msg;
        if (prev >= 0 && prev != c->device) hipSetDevice(prev);
        return st;
    };
    c->err.clear();
    if (!c->has_matrix) return done(MSRSB_E_STATE, "no matrix set");
    if (c->n > kNoAllocMaxN)
        return done(MSRSB_E_ARG, "n exceeds the static scratch limit of 262144 rows");
    if (!o || !v || !z) return done(MSRSB_E_ARG, "invalid arguments");
    auto sm_ok = [](int k) { return k >= MSRSB_SMOOTH_NONE && k <= MSRSB_SMOOTH_IC0; };
    if (!sm_ok(o->pre_smoother) || !sm_ok(o->post_smoother) || o->pre_sweeps < 0 ||
        o->post_sweeps < 0 || o->pre_sweeps > 64 || o->post_sweeps > 64 ||
        (o->ordering != MSRSB_ORDER_NATURAL && o->ordering != MSRSB_ORDER_MULTICOLOR))
        return done(MSRSB_E_ARG, "invalid smoother options");
    if (o->use_multiscale && !c->has_coarse_op)
        return done(MSRSB_E_STATE, "build_coarse must run before a multiscale apply");
    if (o->use_multiscale && c->child)
        return done(MSRSB_E_ARG, "the allocation-free apply takes two-level preconditioners only");
    // the smoother's data must already exist: forming it allocates
    const bool fp32 = o->fp32_smoother != 0;
    for (int k : {o->pre_sweeps > 0 ? o->pre_smoother : 0,
                  o->post_sweeps > 0 ? o->post_smoother : 0}) {
        if ((k == MSRSB_SMOOTH_JACOBI || k == MSRSB_SMOOTH_L1JACOBI) &&
            (!c->smoother_valid || (fp32 && !c->smoother32_valid)))
            return done(MSRSB_E_STATE,
                        "the smoother is not set up: apply or solve with these options first");
        const int ord = o->ordering;
        if ((k == MSRSB_SMOOTH_ILU0 && !c->ilu_ok[ord]) ||
            (k == MSRSB_SMOOTH_IC0 && !c->ic_ok[ord]) ||
            (k == MSRSB_SMOOTH_SGS && !c->tri[ord].built))
            return done(MSRSB_E_STATE,
                        "the smoother is not set up: apply or solve with these options first");
    }
    if (!c->scratch) return done(MSRSB_E_HIP, "the static scratch array is not available");
    double *base = c->scratch;
    ApplyBufs b;
    b.z = base;
    b.spare = b.z + kRegionF64;
    b.tmp = b.spare + kRegionF64;
    double *f32 = b.tmp + kRegionF64;
    for (int k = 0; k < 3; ++k) b.f[k] = reinterpret_cast<float *>(f32 + k * kRegionF32);
    b.vc = f32 + 3 * kRegionF32;
    b.wc = b.vc + kRegionCoarse;
    b.part = b.wc + kRegionCoarse;
    apply_two_stage(c, o, v, z, false, nullptr, nullptr, &b);
    if (hipGetLastError() != hipSuccess) return done(MSRSB_E_HIP, "launch failed");
    return done(MSRSB_OK, nullptr);
}
