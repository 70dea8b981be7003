// Projection without device allocation: rtproj_project_all_noalloc.
//
// The projection's k-dependent workspace (products A B, the iterate x as
// two binary64 parts, the residual r, the split partials of the A-passes,
// the packed operands and the per-step norms) normally lives in buffers the
// plan grows with hipMalloc.  This entry point carves it from one static
// device array instead, so a caller that must not allocate (inside a HIP
// graph capture, a serving loop, a harness that forbids it) can project
// through a plan it created and preconditioned beforehand.
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds its own copy until the process ends.  Host code never names it as a
// kernel argument: its device address on each GPU is resolved once, with
// hipGetSymbolAddress while that GPU is current, when the first plan is
// created there, and only that address is used afterwards.  All calls on one
// GPU share the array, so calls that overlap in time on one GPU race; the
// calls are ordered on one stream or separated by synchronisation.
#include "rt_plan_state.h"

#include <mutex>

namespace {

constexpr size_t RT_STATIC_WS_BYTES = size_t(64) << 20;  // 64 MiB per GPU
constexpr int RT_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[RT_STATIC_WS_BYTES];

std::mutex g_ws_mutex;
void *g_ws_ptr[RT_MAX_DEVICES] = {};

}  // namespace

namespace rtp {

rtproj_status resolve_static_workspace(int device)
{
    if (device < 0 || device >= RT_MAX_DEVICES)
        return fail(RTPROJ_ERR_UNSUPPORTED, "device index above the static workspace table");
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    if (g_ws_ptr[device]) return RTPROJ_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(RTPROJ_ERR_DEVICE, std::string("hipGetSymbolAddress(static workspace): ") + hipGetErrorString(e));
    g_ws_ptr[device] = ptr;
    return RTPROJ_OK;
}

}  // namespace rtp

using namespace rtp;

extern "C" rtproj_status rtproj_project_all_noalloc(rtproj_plan p, const double *B, int64_t ldb, int64_t k, double *Z,
                                                    int64_t ldz, double *Y, int64_t ldy, double *X, int64_t ldx)
{
    if (!p) return fail(RTPROJ_ERR_INVALID_ARG, "null plan");
    if (k <= 0) return project(p, B, ldb, k, Z, ldz, Y, ldy, X, ldx);  // no-op or argument error
    if (p->method_used == RTPROJ_METHOD_KRYLOV)
        return fail(RTPROJ_ERR_UNSUPPORTED, "the iterative method's vectors are not in the static workspace");
    const ProjLayout L = proj_layout(p->m, p->n, k, p->cu_count, use_oz(p, k));
    const size_t need = L.bytes();
    if (need > RT_STATIC_WS_BYTES)
        return fail(RTPROJ_ERR_UNSUPPORTED,
                    "projection workspace of " + std::to_string(need) + " bytes exceeds the static workspace (" +
                        std::to_string(RT_STATIC_WS_BYTES) + " bytes): project fewer right-hand sides per call");
    void *base = (p->device >= 0 && p->device < RT_MAX_DEVICES) ? g_ws_ptr[p->device] : nullptr;
    if (!base) return fail(RTPROJ_ERR_STATE, "static workspace not resolved for the plan's device");
    // point the plan's projection buffers into the static array for this call
    double *saved[ProjLayout::NBUF];
    const int64_t saved_kcap = p->kcap;
    const int saved_ab = p->ab_splits, saved_sx = p->ab_sx_splits, saved_mma = p->ab_mma_splits;
    const int saved_oz = p->oz_splits;
    const bool saved_ozr = p->oz_ready;
    unsigned char *cur = static_cast<unsigned char *>(base);
    for (int i = 0; i < ProjLayout::NBUF; ++i) {
        double **b = proj_buffers(p, i);
        saved[i] = *b;
        *b = reinterpret_cast<double *>(cur);
        cur += ((size_t)L.count[i] * sizeof(double) + 255) / 256 * 256;
    }
    p->kcap = k;
    p->ab_splits = L.ab_splits;
    p->ab_sx_splits = L.ab_sx_splits;
    p->ab_mma_splits = L.ab_mma_splits;
    p->oz_splits = L.oz_splits;
    p->oz_ready = L.oz;
    const rtproj_status st = project(p, B, ldb, k, Z, ldz, Y, ldy, X, ldx);
    for (int i = 0; i < ProjLayout::NBUF; ++i) *proj_buffers(p, i) = saved[i];
    p->kcap = saved_kcap;
    p->ab_splits = saved_ab;
    p->ab_sx_splits = saved_sx;
    p->ab_mma_splits = saved_mma;
    p->oz_splits = saved_oz;
    p->oz_ready = saved_ozr;
    return st;
}
