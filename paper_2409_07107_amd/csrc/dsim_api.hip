// dsim_api.hip -- kernels for gfx950 and the C ABI of include/dsim.h.
//
// One workgroup (an "environment team" of 64, 128, 256 or 512 threads) handles one
// environment at a time; its scratch lives in LDS when it fits (160 KB per
// workgroup on gfx950), otherwise in a caller-provided device workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/dsim.h"
#include "dsim_pipeline.h"

using namespace dsim;

static_assert(kLdStride == DSIM_WS_ENV_DOUBLES && kLdWork == DSIM_WS_WORK,
              "the documented layout of the impulse hand-over");

// The workspace of dsim_step_vjp_noalloc: a file-scope device array that
// every GPU the library runs on holds until the process ends.  In host code
// its name is only a stand-in for the symbol: the device address comes from
// hipGetSymbolAddress, once per device (with that device current), and is
// the only form host code hands to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr size_t kLdsLimit = 160 * 1024;  // bytes of LDS per workgroup on gfx950

template <class R>
BatchView<R> view(const dsim_batch* b) {
    BatchView<R> v;
    v.n_env = b->n_env;
    v.body_off = b->body_off;
    v.dof_off = b->dof_off;
    v.cfg_off = b->cfg_off;
    v.contact_off = b->contact_off;
    v.jac_off = b->jac_off;
    v.parent = b->parent;
    v.jtype = b->jtype;
    v.cbody = b->cbody;
    v.axis = static_cast<const R*>(b->axis);
    v.jrot = static_cast<const R*>(b->jrot);
    v.jpos = static_cast<const R*>(b->jpos);
    v.mass = static_cast<const R*>(b->mass);
    v.com = static_cast<const R*>(b->com);
    v.inertia = static_cast<const R*>(b->inertia);
    v.cpoint = static_cast<const R*>(b->cpoint);
    v.mu = static_cast<const R*>(b->mu);
    v.order = b->order;
    v.pjac_off = b->pjac_off;
    v.cradius = static_cast<const R*>(b->cradius);
    return v;
}

Params params_of(const dsim_params* p) {
    Params q;
    q.dt = p->dt;
    q.gx = p->gravity[0];
    q.gy = p->gravity[1];
    q.gz = p->gravity[2];
    q.gap_mode = p->gap_mode;
    q.ncp_sweeps = p->ncp_sweeps;
    q.ncp_rounds = p->ncp_rounds;
    q.newton_iters = p->newton_iters;
    q.ncp_tol = p->ncp_tol;
    q.rank_tol = p->rank_tol;
    q.mode_eps = p->mode_eps;
    q.kp = p->kp;
    q.kd = p->kd;
    q.pass = 0;
    return q;
}

Dims dims_of(const dsim_batch* b) {
    Dims d;
    d.NB = b->max_bodies > 0 ? b->max_bodies : 1;
    d.NV = b->max_dofs > 0 ? b->max_dofs : 1;
    d.NC = b->max_contacts > 0 ? b->max_contacts : 1;
    d.K = 3 * d.NC;
    return d;
}

size_t team_bytes(const dsim_batch* b, const dsim_params* p, int entry) {
    Dims d = dims_of(b);
    if (p->precision == DSIM_F32) {
        Env<float> E;
        return carve<float>(nullptr, d, entry, E);
    }
    Env<double> E;
    return carve<double>(nullptr, d, entry, E);
}

// Team size of a launch: the caller's choice, else 128 threads, except 512
// for the derivative launch of large trees (24 dofs or more).  The step
// launch is a chain of dependent small solves in one wavefront per
// environment, so more threads only add waves that wait (and fewer teams fit
// a compute unit); the derivative launch of a large tree (one team per
// compute unit, its LDS being the limit) is dense products that a larger team
// spreads.  Measured on tree36 x 16384: FP32 19.5 ms with 128 threads,
// 16.4 ms with 256, 14.9 ms with 512; FP64 17.7, 17.0 and 14.8 ms.  The
// NCP and FBK launches of a derivative entry (the contact solve and its
// fallback, from the record) use one wavefront unless the caller sets a
// team size: their team-wide phases are short loops over the contact rows,
// and where ten teams share a compute unit more wavefronts only wait.  (For
// a batch whose largest environment leaves room for three teams per compute
// unit, 256 threads measured faster: 104 against 119 ms per call on the
// ragged batch, whose planner sets the team size.)
int team_threads(const dsim_params* p, const dsim_batch* b, int entry) {
    if (p->threads > 0) return p->threads;
    if (entry == ENTRY_NCP || entry == ENTRY_FBK) return 64;
    const bool big = b->max_dofs >= 24;
    return (entry_has_derivative(entry) && big) ? 512 : 128;
}

// One workgroup (team) per environment; the team's whole working set is
// carved from the dynamic LDS allocation.
template <class R, int ENTRY>
__global__ __launch_bounds__(512) void env_kernel(BatchView<R> B, Params P, Dims D, const R* q, const R* v,
                                                  const R* tau, const R* gbar, const R* gbar2, R* v_next, R* lam,
                                                  int8_t* mode, int32_t* status, R* o1, R* o2, R* o3, R* o4, R* o5,
                                                  double* ld) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    Team T;
    T.tid = threadIdx.x;
    T.nt = blockDim.x;
    T.lane = threadIdx.x & 63;
    T.wave = threadIdx.x >> 6;
    T.wsize = 64;
    const int e = B.order ? B.order[blockIdx.x] : int(blockIdx.x);
    if (e < 0 || e >= B.n_env) return;  // the whole workgroup skips an invalid list entry
    // an environment larger than the launch's buffers is not computed
    if (B.body_off[e + 1] - B.body_off[e] > D.NB || B.dof_off[e + 1] - B.dof_off[e] > D.NV ||
        B.contact_off[e + 1] - B.contact_off[e] > D.NC) {
        if (threadIdx.x == 0) status[e] = ST_SIZE;
        return;
    }
    // the fallback pass of the solve recomputes only the environments the
    // first pass left unsolved (the whole workgroup exits for the others)
    if (P.pass == 1 && !(status[e] & (ST_NCP | ST_POLISH))) return;
    // a derivative launch split in two: pass 2 differentiates the
    // environments the first step pass solved (while the fallback pass runs
    // on the others), pass 3 the others, after the fallback pass
    if (P.pass >= 2 && ld) {
        const bool fb = ld[size_t(e) * kLdStride + kLdFallback] != 0.0;
        if (fb != (P.pass == 3)) return;
    }
    Env<R> E;
    carve<R>(smem, D, ENTRY, E);
    run_env<R>(T, E, B, P, D, ENTRY, e, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5, ld);
}

// Tangent gradient on q -> gradient on the stored coordinates of q: per body,
// a revolute angle copies; a free flyer (q = p, quaternion) maps the
// body-frame linear part by R(quat) and the angular part g to
// 2 quat * (g, 0), the gradient whose pairing with the coordinate change
// of q (+) d reproduces the tangent gradient for every d.
template <class R>
__global__ __launch_bounds__(64) void ambient_kernel(BatchView<R> B, const R* q, const R* gt, R* ga) {
    const int e = blockIdx.x;
    const int b0 = B.body_off[e], nb = B.body_off[e + 1] - b0;
    const int q0 = B.cfg_off[e], d0 = B.dof_off[e];
    // configuration and velocity offsets of each body follow from the joint
    // types in body order: computed redundantly by every lane
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        int cfg = 0, dof = 0;
        for (int i = 0; i < b; ++i) {
            const bool ff = B.jtype[b0 + i] == 1;
            cfg += ff ? 7 : 1;
            dof += ff ? 6 : 1;
        }
        const R* qq = q + q0 + cfg;
        const R* g = gt + d0 + dof;
        R* o = ga + q0 + cfg;
        if (B.jtype[b0 + b] == 1) {
            const double x = qq[3], y = qq[4], z = qq[5], w = qq[6];
            const double Rm[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                                  2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                                  2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
            for (int i = 0; i < 3; ++i)
                o[i] = R(Rm[3 * i] * double(g[0]) + Rm[3 * i + 1] * double(g[1]) + Rm[3 * i + 2] * double(g[2]));
            const double gx = g[3], gy = g[4], gz = g[5];
            // 2 (x y z w) * (gx gy gz 0)
            o[3] = R(2 * (w * gx + (y * gz - z * gy)));
            o[4] = R(2 * (w * gy + (z * gx - x * gz)));
            o[5] = R(2 * (w * gz + (x * gy - y * gx)));
            o[6] = R(-2 * (x * gx + y * gy + z * gz));
        } else {
            o[0] = g[0];
        }
    }
}

// The transpose of the tangent map: a gradient on the stored coordinates of q
// -> the tangent adjoint, g_tangent = (d (q (+) delta) / d delta)^T g_ambient
// at delta = 0.  Revolute entries copy; a free flyer gets R(quat)^T g_p for
// the linear part and (w g_v - v x g_v - v g_w) / 2 for the angular part,
// with (v, w) the quaternion's vector and scalar parts and (g_v, g_w) the
// gradient on them (the differential of quat * exp(delta / 2)).
template <class R>
__global__ __launch_bounds__(64) void tangent_kernel(BatchView<R> B, const R* q, const R* ga, R* gt) {
    const int e = blockIdx.x;
    const int b0 = B.body_off[e], nb = B.body_off[e + 1] - b0;
    const int q0 = B.cfg_off[e], d0 = B.dof_off[e];
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        int cfg = 0, dof = 0;
        for (int i = 0; i < b; ++i) {
            const bool ff = B.jtype[b0 + i] == 1;
            cfg += ff ? 7 : 1;
            dof += ff ? 6 : 1;
        }
        const R* qq = q + q0 + cfg;
        const R* g = ga + q0 + cfg;
        R* o = gt + d0 + dof;
        if (B.jtype[b0 + b] == 1) {
            const double x = qq[3], y = qq[4], z = qq[5], w = qq[6];
            const double Rm[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                                  2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                                  2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
            for (int i = 0; i < 3; ++i)
                o[i] = R(Rm[i] * double(g[0]) + Rm[3 + i] * double(g[1]) + Rm[6 + i] * double(g[2]));
            const double gx = g[3], gy = g[4], gz = g[5], gw = g[6];
            o[3] = R(0.5 * (w * gx - (y * gz - z * gy) - x * gw));
            o[4] = R(0.5 * (w * gy - (z * gx - x * gz) - y * gw));
            o[5] = R(0.5 * (w * gz - (x * gy - y * gx) - z * gw));
        } else {
            o[0] = g[0];
        }
    }
}

int check_common(const dsim_batch* b, const dsim_params* p) {
    if (!b || !p) return DSIM_ERR_ARG;
    int rc = dsim_validate_params(p);
    if (rc) return rc;
    if (b->n_env < 0) return DSIM_ERR_ARG;
    if (b->max_bodies > DSIM_MAX_BODIES || b->max_dofs > DSIM_MAX_DOFS || b->max_contacts > DSIM_MAX_CONTACTS)
        return DSIM_ERR_SIZE;
    if (b->max_bodies < 0 || b->max_dofs < 0 || b->max_contacts < 0 || b->max_cfg < 0) return DSIM_ERR_ARG;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!b->body_off || !b->dof_off || !b->cfg_off || !b->contact_off || !b->parent || !b->jtype || !b->axis ||
        !b->jrot || !b->jpos || !b->mass || !b->com || !b->inertia)
        return DSIM_ERR_ARG;
    if (b->max_contacts > 0 && (!b->cbody || !b->cpoint || !b->mu)) return DSIM_ERR_ARG;
    return DSIM_SUCCESS;
}

// One launch of env_kernel<R, ENTRY> over the batch (or its launch list).
template <class R, int ENTRY>
int launch_one(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
               const void* gbar, const void* gbar2, void* v_next, void* lam, int8_t* mode, int32_t* status,
               void* o1, void* o2, void* o3, void* o4, void* o5, double* ld, void* stream, int pass = 0) {
    const size_t bytes = team_bytes(b, p, ENTRY);
    if (bytes > kLdsLimit) return DSIM_ERR_SIZE;  // the team's working set must fit in LDS
    const int threads = team_threads(p, b, ENTRY);
    auto kern = env_kernel<R, ENTRY>;
    const unsigned lds = unsigned(bytes);
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(lds)) != hipSuccess)
            return DSIM_ERR_LAUNCH;
    }
    const int grid = b->order ? b->n_order : b->n_env;
    if (grid <= 0) return DSIM_SUCCESS;
    Params P = params_of(p);
    P.pass = pass;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, static_cast<hipStream_t>(stream), view<R>(b),
                       P, dims_of(b), static_cast<const R*>(q), static_cast<const R*>(v),
                       static_cast<const R*>(tau), static_cast<const R*>(gbar), static_cast<const R*>(gbar2),
                       static_cast<R*>(v_next), static_cast<R*>(lam), mode, status, static_cast<R*>(o1),
                       static_cast<R*>(o2), static_cast<R*>(o3), static_cast<R*>(o4), static_cast<R*>(o5), ld);
    return hipGetLastError() == hipSuccess ? DSIM_SUCCESS : DSIM_ERR_LAUNCH;
}

// Bytes of the hand-over between the step and derivative launches: the FP64
// impulses, then one record of the step's quantities per environment.
size_t handover_bytes(const dsim_batch* b, const dsim_params* p) {
    const Dims d = dims_of(b);
    const size_t rec = p->precision == DSIM_F32 ? handover_layout<float>(d).bytes : handover_layout<double>(d).bytes;
    const size_t imp = ((size_t(b->n_env) * kLdStride + 1) & ~size_t(1)) * sizeof(double);
    return imp + size_t(b->n_env) * rec;
}

constexpr int kMaxDevices = 64;

// Per device, a second stream (default priority) and two events with which a
// derivative entry runs its fallback pass beside the derivative launch of
// the environments the first pass solved; created on first use.  The
// enqueue sequence that uses them is serialised by `mutex`, so concurrent
// callers may share them.  A call on a stream under graph capture does not
// use them: its launches stay on the caller's stream in order (a fork of
// the capture onto this shared stream made the runtime crash when the
// capture ended).
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool failed = false;
    std::mutex mutex;
};
SideStream g_side[kMaxDevices];
std::mutex g_side_setup;

SideStream* side_stream(hipStream_t caller) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(caller, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    SideStream& ss = g_side[dev];
    std::lock_guard<std::mutex> lock(g_side_setup);
    if (ss.stream) return &ss;
    if (ss.failed) return nullptr;
    hipStream_t st = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
        if (st) (void)hipStreamDestroy(st);
        if (a) (void)hipEventDestroy(a);
        ss.failed = true;
        return nullptr;
    }
    ss.stream = st;
    ss.fork = a;
    ss.join = b;
    return &ss;
}

// The first pass of a derivative entry's step: the ASM launch (the step up to
// its contact system, written to each environment's record) and the NCP
// launch (the contact solve and the rest of the step, from the record, in a
// layout several times smaller: more teams share a compute unit during the
// latency-bound iterations).  Same arithmetic as one step launch.
template <class R>
int first_pass(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
               void* v_next, void* lam, int8_t* mode, int32_t* status, double* ld, void* stream) {
    int rc = launch_one<R, ENTRY_ASM>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, nullptr,
                                      nullptr, nullptr, nullptr, nullptr, ld, stream, 0);
    if (rc) return rc;
    return launch_one<R, ENTRY_NCP>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, nullptr,
                                    nullptr, nullptr, nullptr, nullptr, ld, stream, 0);
}

// The step is two launches of the step kernel on the same stream: the first
// pass of the solve over every environment, then its fallback pass, whose
// workgroups exit at once for the environments the first pass solved (its
// status output tells them) and recompute the others from the first pass's
// impulses.  A hard environment's fallback then overlaps with the others'
// instead of lengthening one team's chain of rounds.  A derivative entry
// runs its first pass as two launches (first_pass) and its fallback pass
// from the contact system in the record (FBK: no tree recursions again, the
// small layout), then the derivative launch: the step launches have a small
// on-chip footprint (several teams share a compute unit while they iterate
// on the contact problem) and hand their FP64 impulses and other quantities
// over through the workspace to the derivative launch, which loads them.
template <class R, int ENTRY>
int launch(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
           const void* gbar, const void* gbar2, void* v_next, void* lam, int8_t* mode, int32_t* status, void* o1,
           void* o2, void* o3, void* o4, void* o5, void* ws, size_t ws_bytes, void* stream, bool fork) {
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (ENTRY == ENTRY_STEP && ws && ws_bytes >= handover_bytes(b, p)) {
        // the step with a workspace: the derivative entries' step launches
        // (the same outputs, bit for bit; more teams iterate per compute unit)
        double* ld = static_cast<double*>(ws);
        int rc = first_pass<R>(b, p, q, v, tau, v_next, lam, mode, status, ld, stream);
        if (rc) return rc;
        return launch_one<R, ENTRY_FBK>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, nullptr,
                                        nullptr, nullptr, nullptr, nullptr, ld, stream, 1);
    }
    if (!entry_has_derivative(ENTRY)) {
        int rc = launch_one<R, ENTRY>(b, p, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5,
                                      nullptr, stream, 0);
        if (rc) return rc;
        return launch_one<R, ENTRY>(b, p, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5,
                                    nullptr, stream, 1);
    }
    if (!ws || ws_bytes < handover_bytes(b, p)) return DSIM_ERR_WORKSPACE;
    if (team_bytes(b, p, ENTRY) > kLdsLimit) return DSIM_ERR_SIZE;  // before any launch
    double* ld = static_cast<double*>(ws);
    int rc = first_pass<R>(b, p, q, v, tau, v_next, lam, mode, status, ld, stream);
    if (rc) return rc;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // a launch list (a plan's size class, whose caller runs the classes on
    // streams of its own) keeps its launches on the caller's stream: the
    // classes would otherwise queue their fallback passes on the one second
    // stream
    SideStream* side = (fork && !b->order) ? side_stream(s) : nullptr;
    if (!side) {
        rc = launch_one<R, ENTRY_FBK>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, nullptr,
                                      nullptr, nullptr, nullptr, nullptr, ld, stream, 1);
        if (rc) return rc;
        return launch_one<R, ENTRY>(b, p, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5,
                                    ld, stream);
    }
    // The fallback pass on the side stream, beside the derivative of the
    // environments the first pass solved (each launch touches only its own
    // environments' outputs and records); then the derivative of the others.
    std::lock_guard<std::mutex> lock(side->mutex);
    if (hipEventRecord(side->fork, s) != hipSuccess || hipStreamWaitEvent(side->stream, side->fork, 0) != hipSuccess)
        return DSIM_ERR_LAUNCH;
    rc = launch_one<R, ENTRY_FBK>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, nullptr, nullptr,
                                  nullptr, nullptr, nullptr, ld, side->stream, 1);
    const bool joined = hipEventRecord(side->join, side->stream) == hipSuccess;
    const int rc2 = launch_one<R, ENTRY>(b, p, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5,
                                         ld, stream, 2);
    // the caller's stream waits for the side stream whatever failed, so that
    // no work of this call is left outside its stream's order
    if (!joined || hipStreamWaitEvent(s, side->join, 0) != hipSuccess) return DSIM_ERR_LAUNCH;
    if (rc) return rc;
    if (rc2) return rc2;
    return launch_one<R, ENTRY>(b, p, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5, ld,
                                stream, 3);
}

// The halves of a derivative entry as separate calls: the step launches
// writing the hand-over into `ws` (half 1), or the derivative launch reading
// it (half 2) -- the same launches, in the same order, as the whole entry.
template <class R, int ENTRY>
int launch_half(int half, const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                const void* tau, const void* gbar, const void* gbar2, void* v_next, void* lam, int8_t* mode,
                int32_t* status, void* o1, void* o2, void* o3, void* ws, size_t ws_bytes, void* stream) {
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!ws || ws_bytes < handover_bytes(b, p)) return DSIM_ERR_WORKSPACE;
    if (team_bytes(b, p, ENTRY) > kLdsLimit) return DSIM_ERR_SIZE;  // before any launch
    double* ld = static_cast<double*>(ws);
    if (half == 1) {
        int rc = first_pass<R>(b, p, q, v, tau, v_next, lam, mode, status, ld, stream);
        if (rc) return rc;
        return launch_one<R, ENTRY_FBK>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, nullptr,
                                        nullptr, nullptr, nullptr, nullptr, ld, stream, 1);
    }
    return launch_one<R, ENTRY>(b, p, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, nullptr,
                                nullptr, ld, stream);
}

template <int ENTRY>
int dispatch(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
             const void* gbar, const void* gbar2, void* v_next, void* lam, int8_t* mode, int32_t* status, void* o1,
             void* o2, void* o3, void* o4, void* o5, void* ws, size_t ws_bytes, void* stream, bool fork = true) {
    int rc = check_common(b, p);
    if (rc) return rc;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!q || !v || !tau || !v_next || !status || !mode || !lam) return DSIM_ERR_ARG;
    if (p->precision == DSIM_F32)
        return launch<float, ENTRY>(b, p, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5,
                                    ws, ws_bytes, stream, fork);
    return launch<double, ENTRY>(b, p, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5,
                                 ws, ws_bytes, stream, fork);
}

// The step and the position update (the step kernel's two launches, as the
// step-only entry runs them) that also write the hand-over record and the
// FP64 impulses into `ws`, for a later reverse pass through
// dsim_step_integrate_vjp_kept.
template <class R>
int keep_integrate(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
                   void* q_next, void* v_next, void* lam, int8_t* mode, int32_t* status, void* ws, size_t ws_bytes,
                   void* stream) {
    if (!ws || ws_bytes < handover_bytes(b, p)) return DSIM_ERR_WORKSPACE;
    if (team_bytes(b, p, ENTRY_RVJP) > kLdsLimit) return DSIM_ERR_SIZE;  // its reverse pass must fit as well
    double* ld = static_cast<double*>(ws);
    for (int pass = 0; pass < 2; ++pass) {
        const int rc = launch_one<R, ENTRY_SINT>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, q_next,
                                                 nullptr, nullptr, nullptr, nullptr, ld, stream, pass);
        if (rc) return rc;
    }
    return DSIM_SUCCESS;
}

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (set up on the first call on
// that device), or nullptr if the device or the symbol is not available.
void* scratch_address() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

size_t dsim_noalloc_scratch_bytes(void) { return kScratchBytes; }

int32_t dsim_step_vjp_noalloc(const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                              const void* tau, const void* g_vnext, const void* g_lam, void* v_next, void* lam,
                              int8_t* mode, int32_t* status, void* g_q, void* g_v, void* g_tau, void* stream) {
    if (!g_vnext || !g_q || !g_v || !g_tau) return DSIM_ERR_ARG;
    int rc = check_common(b, p);
    if (rc) return rc;
    if (b->n_env == 0) return DSIM_SUCCESS;
    // the batch's hand-over must fit the static workspace; checked before
    // any device call
    if (handover_bytes(b, p) > kScratchBytes) return DSIM_ERR_WORKSPACE;
    void* ws = scratch_address();
    if (!ws) return DSIM_ERR_DEVICE;
    // the step launches write every hand-over record the derivative launch
    // reads, so nothing in the array needs clearing between calls
    // one stream, no side stream or events: nothing is created
    return dispatch<ENTRY_VJP>(b, p, q, v, tau, g_vnext, g_lam, v_next, lam, mode, status, g_q, g_v, g_tau,
                               nullptr, nullptr, ws, kScratchBytes, stream, false);
}

void dsim_default_params(dsim_params* p, int32_t precision) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->dt = 1e-3;
    p->gravity[0] = 0.0;
    p->gravity[1] = 0.0;
    p->gravity[2] = -9.81;
    p->gap_mode = 0;
    p->precision = precision;
    p->ncp_sweeps = 30;
    p->ncp_rounds = 4;
    p->newton_iters = 6;
    p->threads = 0;
    if (precision == DSIM_F32) {
        p->ncp_tol = 1e-5;
        p->rank_tol = 1e-5;
        p->mode_eps = 1e-5;
    } else {
        p->ncp_tol = 1e-12;
        p->rank_tol = 1e-10;
        p->mode_eps = 1e-9;
    }
}

int32_t dsim_abi_version(void) { return DSIM_ABI_VERSION; }

size_t dsim_struct_size(int32_t which) {
    return which == 0 ? sizeof(dsim_batch) : which == 1 ? sizeof(dsim_params) : 0;
}

const char* dsim_error_string(int32_t code) {
    switch (code) {
        case DSIM_SUCCESS: return "success";
        case DSIM_ERR_ARG: return "invalid argument";
        case DSIM_ERR_SIZE: return "size beyond the supported maxima";
        case DSIM_ERR_LAUNCH: return "kernel launch failed";
        case DSIM_ERR_WORKSPACE: return "workspace too small";
        case DSIM_ERR_MODEL: return "non-physical model";
        case DSIM_ERR_DEVICE: return "no usable gfx950 device";
        default: return "unknown error";
    }
}

const char* dsim_status_string(int32_t bit) {
    switch (bit) {
        case DSIM_ST_NCP_NOT_CONVERGED: return "NCP residual above ncp_tol";
        case DSIM_ST_RANK_DEFICIENT: return "reduced system rank-deficient (redundant contacts)";
        case DSIM_ST_MODE_DEGENERATE: return "a contact within mode_eps of a mode switch";
        case DSIM_ST_NONFINITE: return "non-finite value in the outputs";
        case DSIM_ST_POLISH_FAILED: return "Newton refinement did not reach a consistent mode set";
        case DSIM_ST_SIZE_EXCEEDED: return "environment larger than the launch's sizes: not computed";
        case 0: return "ok";
        default: return "not a single status bit";
    }
}

int32_t dsim_validate_params(const dsim_params* p) {
    if (!p) return DSIM_ERR_ARG;
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return DSIM_ERR_ARG;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->gravity[i])) return DSIM_ERR_ARG;
    if (p->gap_mode != 0 && p->gap_mode != 1) return DSIM_ERR_ARG;
    if (p->precision != DSIM_F64 && p->precision != DSIM_F32) return DSIM_ERR_ARG;
    if (p->ncp_sweeps < 1 || p->ncp_rounds < 1 || p->newton_iters < 0) return DSIM_ERR_ARG;
    if (p->threads != 0 && p->threads != 64 && p->threads != 128 && p->threads != 256 && p->threads != 512)
        return DSIM_ERR_ARG;
    if (!(p->ncp_tol > 0) || !(p->rank_tol > 0) || !(p->mode_eps >= 0)) return DSIM_ERR_ARG;
    if (!(p->kp >= 0 && p->kp <= 1) || !(p->kd >= 0) || !std::isfinite(p->kd)) return DSIM_ERR_ARG;
    return DSIM_SUCCESS;
}

int32_t dsim_validate_host(const dsim_batch* b, int32_t* bad_env) {
    if (bad_env) *bad_env = -1;
    if (!b || b->n_env < 0) return DSIM_ERR_ARG;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!b->body_off || !b->dof_off || !b->cfg_off || !b->contact_off || !b->parent || !b->jtype || !b->axis ||
        !b->jrot || !b->jpos || !b->mass || !b->com || !b->inertia)
        return DSIM_ERR_ARG;
    if (b->max_bodies > DSIM_MAX_BODIES || b->max_dofs > DSIM_MAX_DOFS || b->max_contacts > DSIM_MAX_CONTACTS)
        return DSIM_ERR_SIZE;
    const double* axis = static_cast<const double*>(b->axis);
    const double* jrot = static_cast<const double*>(b->jrot);
    const double* mass = static_cast<const double*>(b->mass);
    const double* inertia = static_cast<const double*>(b->inertia);
    const double* mu = static_cast<const double*>(b->mu);
    const double* crad = static_cast<const double*>(b->cradius);
    if (b->body_off[0] != 0 || b->dof_off[0] != 0 || b->cfg_off[0] != 0 || b->contact_off[0] != 0)
        return DSIM_ERR_ARG;
    for (int e = 0; e < b->n_env; ++e) {
        auto fail = [&](int code) {
            if (bad_env) *bad_env = e;
            return code;
        };
        const int b0 = b->body_off[e], nb = b->body_off[e + 1] - b0;
        const int nc = b->contact_off[e + 1] - b->contact_off[e];
        const int nvv = b->dof_off[e + 1] - b->dof_off[e];
        const int nqq = b->cfg_off[e + 1] - b->cfg_off[e];
        if (nb < 1 || nc < 0 || nvv < 1 || nqq < 1) return fail(DSIM_ERR_ARG);
        if (nb > b->max_bodies || nc > b->max_contacts || nvv > b->max_dofs || nqq > b->max_cfg)
            return fail(DSIM_ERR_SIZE);
        int nv = 0, nq = 0;
        for (int i = 0; i < nb; ++i) {
            const int gi = b0 + i;
            const int par = b->parent[gi], jt = b->jtype[gi];
            if (par >= i || par < -1) return fail(DSIM_ERR_MODEL);
            if (jt != DSIM_JOINT_REVOLUTE && jt != DSIM_JOINT_FREEFLYER) return fail(DSIM_ERR_MODEL);
            if (jt == DSIM_JOINT_FREEFLYER && (i != 0 || par != -1)) return fail(DSIM_ERR_MODEL);
            nv += jt == DSIM_JOINT_FREEFLYER ? 6 : 1;
            nq += jt == DSIM_JOINT_FREEFLYER ? 7 : 1;
            if (jt == DSIM_JOINT_REVOLUTE) {
                const double* a = axis + 3 * gi;
                const double na = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
                if (!(std::fabs(na - 1.0) < 1e-6)) return fail(DSIM_ERR_MODEL);
            }
            const double* Rm = jrot + 9 * gi;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k) s += Rm[3 * r + k] * Rm[3 * c + k];
                    if (!(std::fabs(s - (r == c ? 1.0 : 0.0)) < 1e-6)) return fail(DSIM_ERR_MODEL);
                }
            if (!(mass[gi] > 0) || !std::isfinite(mass[gi])) return fail(DSIM_ERR_MODEL);
            const double* I = inertia + 6 * gi;
            // positive definite (Sylvester) and principal moments satisfying the
            // triangle inequality (checked on the diagonal of any frame as a
            // necessary condition: Ixx + Iyy >= Izz etc.)
            const double d1 = I[0], d2 = I[0] * I[1] - I[3] * I[3];
            const double d3 = I[0] * (I[1] * I[2] - I[5] * I[5]) - I[3] * (I[3] * I[2] - I[5] * I[4]) +
                              I[4] * (I[3] * I[5] - I[1] * I[4]);
            if (!(d1 > 0 && d2 > 0 && d3 > 0)) return fail(DSIM_ERR_MODEL);
            if (!(I[0] + I[1] >= I[2] * (1 - 1e-9) && I[0] + I[2] >= I[1] * (1 - 1e-9) &&
                  I[1] + I[2] >= I[0] * (1 - 1e-9)))
                return fail(DSIM_ERR_MODEL);
        }
        if (nv != nvv || nq != nqq) return fail(DSIM_ERR_ARG);
        for (int c = 0; c < nc; ++c) {
            const int gc = b->contact_off[e] + c;
            if (!b->cbody || !b->cpoint || !b->mu) return fail(DSIM_ERR_ARG);
            if (b->cbody[gc] < 0 || b->cbody[gc] >= nb) return fail(DSIM_ERR_MODEL);
            if (!(mu[gc] >= 0) || !std::isfinite(mu[gc])) return fail(DSIM_ERR_MODEL);
            if (crad && (!(crad[gc] >= 0) || !std::isfinite(crad[gc]))) return fail(DSIM_ERR_MODEL);
        }
        if (b->jac_off && b->jac_off[e + 1] - b->jac_off[e] != nv * nv) return fail(DSIM_ERR_ARG);
    }
    return DSIM_SUCCESS;
}

size_t dsim_lds_bytes(const dsim_batch* b, const dsim_params* p, int32_t entry) {
    if (!b || !p || entry < 0 || entry > DSIM_ENTRY_JACOBIAN_PARAMS) return 0;
    return team_bytes(b, p, entry);
}

size_t dsim_workspace_bytes(const dsim_batch* b, const dsim_params* p, int32_t entry) {
    if (!b || !p || b->n_env <= 0) return 0;
    return entry_has_derivative(entry) ? handover_bytes(b, p) : 0;
}

int32_t dsim_step(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
                  void* v_next, void* lam, int8_t* mode, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    return dispatch<ENTRY_STEP>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, nullptr, nullptr,
                                nullptr, nullptr, nullptr, ws, ws_bytes, stream);
}

int32_t dsim_step_jacobian(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
                           void* v_next, void* lam, int8_t* mode, int32_t* status, void* dvdq, void* dvdv,
                           void* dvdtau, void* ws, size_t ws_bytes, void* stream) {
    if (!dvdq || !dvdv || !dvdtau || (b && b->n_env > 0 && !b->jac_off)) return DSIM_ERR_ARG;
    return dispatch<ENTRY_JAC>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, dvdq, dvdv, dvdtau,
                               nullptr, nullptr, ws, ws_bytes, stream);
}

int32_t dsim_step_jacobian_params(const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                                  const void* tau, void* v_next, void* lam, int8_t* mode, int32_t* status,
                                  void* dvdq, void* dvdv, void* dvdtau, void* dvdp, void* ws, size_t ws_bytes,
                                  void* stream) {
    if (!dvdq || !dvdv || !dvdtau || !dvdp || (b && b->n_env > 0 && (!b->jac_off || !b->pjac_off)))
        return DSIM_ERR_ARG;
    return dispatch<ENTRY_PJAC>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, dvdq, dvdv, dvdtau,
                                dvdp, nullptr, ws, ws_bytes, stream);
}

int32_t dsim_step_vjp(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
                      const void* g_vnext, const void* g_lam, void* v_next, void* lam, int8_t* mode,
                      int32_t* status, void* g_q, void* g_v, void* g_tau, void* ws, size_t ws_bytes, void* stream) {
    if (!g_vnext || !g_q || !g_v || !g_tau) return DSIM_ERR_ARG;
    return dispatch<ENTRY_VJP>(b, p, q, v, tau, g_vnext, g_lam, v_next, lam, mode, status, g_q, g_v, g_tau,
                               nullptr, nullptr, ws, ws_bytes, stream);
}

int32_t dsim_step_keep(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
                       void* v_next, void* lam, int8_t* mode, int32_t* status, void* ws, size_t ws_bytes,
                       void* stream) {
    int rc = check_common(b, p);
    if (rc) return rc;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!q || !v || !tau || !v_next || !status || !mode || !lam) return DSIM_ERR_ARG;
    if (p->precision == DSIM_F32)
        return launch_half<float, ENTRY_VJP>(1, b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status,
                                             nullptr, nullptr, nullptr, ws, ws_bytes, stream);
    return launch_half<double, ENTRY_VJP>(1, b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, nullptr,
                                          nullptr, nullptr, ws, ws_bytes, stream);
}

int32_t dsim_vjp_kept(const dsim_batch* b, const dsim_params* p, const void* q, const void* v, const void* tau,
                      const void* g_vnext, const void* g_lam, const int8_t* mode, int32_t* status, void* g_q,
                      void* g_v, void* g_tau, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(b, p);
    if (rc) return rc;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!q || !v || !tau || !status || !mode || !g_vnext || !g_q || !g_v || !g_tau) return DSIM_ERR_ARG;
    int8_t* md = const_cast<int8_t*>(mode);  // read only by the derivative launch
    if (p->precision == DSIM_F32)
        return launch_half<float, ENTRY_VJP>(2, b, p, q, v, tau, g_vnext, g_lam, nullptr, nullptr, md, status, g_q,
                                             g_v, g_tau, ws, ws_bytes, stream);
    return launch_half<double, ENTRY_VJP>(2, b, p, q, v, tau, g_vnext, g_lam, nullptr, nullptr, md, status, g_q,
                                          g_v, g_tau, ws, ws_bytes, stream);
}

int32_t dsim_jacobian_kept(const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                           const void* tau, const int8_t* mode, int32_t* status, void* dvdq, void* dvdv,
                           void* dvdtau, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(b, p);
    if (rc) return rc;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!q || !v || !tau || !status || !mode || !dvdq || !dvdv || !dvdtau || !b->jac_off) return DSIM_ERR_ARG;
    int8_t* md = const_cast<int8_t*>(mode);  // read only by the derivative launch
    if (p->precision == DSIM_F32)
        return launch_half<float, ENTRY_JAC>(2, b, p, q, v, tau, nullptr, nullptr, nullptr, nullptr, md, status,
                                             dvdq, dvdv, dvdtau, ws, ws_bytes, stream);
    return launch_half<double, ENTRY_JAC>(2, b, p, q, v, tau, nullptr, nullptr, nullptr, nullptr, md, status, dvdq,
                                          dvdv, dvdtau, ws, ws_bytes, stream);
}

int32_t dsim_step_vjp_params(const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                             const void* tau, const void* g_vnext, const void* g_lam, void* v_next, void* lam,
                             int8_t* mode, int32_t* status, void* g_q, void* g_v, void* g_tau, void* g_params,
                             void* ws, size_t ws_bytes, void* stream) {
    if (!g_vnext || !g_q || !g_v || !g_tau || !g_params) return DSIM_ERR_ARG;
    return dispatch<ENTRY_PVJP>(b, p, q, v, tau, g_vnext, g_lam, v_next, lam, mode, status, g_q, g_v, g_tau,
                                g_params, nullptr, ws, ws_bytes, stream);
}

int32_t dsim_step_integrate(const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                            const void* tau, void* q_next, void* v_next, void* lam, int8_t* mode, int32_t* status,
                            void* stream) {
    if (!q_next) return DSIM_ERR_ARG;
    return dispatch<ENTRY_SINT>(b, p, q, v, tau, nullptr, nullptr, v_next, lam, mode, status, q_next, nullptr,
                                nullptr, nullptr, nullptr, nullptr, 0, stream);
}

int32_t dsim_step_integrate_vjp(const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                                const void* tau, const void* a_qnext, const void* a_vnext, void* v_next, void* lam,
                                int8_t* mode, int32_t* status, void* a_q, void* a_v, void* g_tau, void* ws,
                                size_t ws_bytes, void* stream) {
    if (!a_qnext || !a_vnext || !a_q || !a_v || !g_tau) return DSIM_ERR_ARG;
    return dispatch<ENTRY_RVJP>(b, p, q, v, tau, a_vnext, a_qnext, v_next, lam, mode, status, a_q, a_v, g_tau,
                                nullptr, nullptr, ws, ws_bytes, stream);
}

int32_t dsim_step_integrate_keep(const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                                 const void* tau, void* q_next, void* v_next, void* lam, int8_t* mode,
                                 int32_t* status, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_common(b, p);
    if (rc) return rc;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!q || !v || !tau || !q_next || !v_next || !status || !mode || !lam) return DSIM_ERR_ARG;
    if (p->precision == DSIM_F32)
        return keep_integrate<float>(b, p, q, v, tau, q_next, v_next, lam, mode, status, ws, ws_bytes, stream);
    return keep_integrate<double>(b, p, q, v, tau, q_next, v_next, lam, mode, status, ws, ws_bytes, stream);
}

int32_t dsim_step_integrate_vjp_kept(const dsim_batch* b, const dsim_params* p, const void* q, const void* v,
                                     const void* tau, const void* a_qnext, const void* a_vnext, const int8_t* mode,
                                     int32_t* status, void* a_q, void* a_v, void* g_tau, void* ws, size_t ws_bytes,
                                     void* stream) {
    int rc = check_common(b, p);
    if (rc) return rc;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!q || !v || !tau || !status || !mode || !a_qnext || !a_vnext || !a_q || !a_v || !g_tau) return DSIM_ERR_ARG;
    int8_t* md = const_cast<int8_t*>(mode);  // read only by the derivative launch
    if (p->precision == DSIM_F32)
        return launch_half<float, ENTRY_RVJP>(2, b, p, q, v, tau, a_vnext, a_qnext, nullptr, nullptr, md, status, a_q,
                                              a_v, g_tau, ws, ws_bytes, stream);
    return launch_half<double, ENTRY_RVJP>(2, b, p, q, v, tau, a_vnext, a_qnext, nullptr, nullptr, md, status, a_q,
                                           a_v, g_tau, ws, ws_bytes, stream);
}

int32_t dsim_tangent_to_ambient(const dsim_batch* b, int32_t precision, const void* q, const void* g_tangent,
                                void* g_ambient, void* stream) {
    if (!b || b->n_env < 0 || (precision != DSIM_F32 && precision != DSIM_F64)) return DSIM_ERR_ARG;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!q || !g_tangent || !g_ambient || !b->body_off || !b->dof_off || !b->cfg_off || !b->jtype)
        return DSIM_ERR_ARG;
    if (precision == DSIM_F32)
        hipLaunchKernelGGL(ambient_kernel<float>, dim3(b->n_env), dim3(64), 0, static_cast<hipStream_t>(stream),
                           view<float>(b), static_cast<const float*>(q), static_cast<const float*>(g_tangent),
                           static_cast<float*>(g_ambient));
    else
        hipLaunchKernelGGL(ambient_kernel<double>, dim3(b->n_env), dim3(64), 0, static_cast<hipStream_t>(stream),
                           view<double>(b), static_cast<const double*>(q), static_cast<const double*>(g_tangent),
                           static_cast<double*>(g_ambient));
    return hipGetLastError() == hipSuccess ? DSIM_SUCCESS : DSIM_ERR_LAUNCH;
}

int32_t dsim_ambient_to_tangent(const dsim_batch* b, int32_t precision, const void* q, const void* g_ambient,
                                void* g_tangent, void* stream) {
    if (!b || b->n_env < 0 || (precision != DSIM_F32 && precision != DSIM_F64)) return DSIM_ERR_ARG;
    if (b->n_env == 0) return DSIM_SUCCESS;
    if (!q || !g_tangent || !g_ambient || !b->body_off || !b->dof_off || !b->cfg_off || !b->jtype)
        return DSIM_ERR_ARG;
    if (precision == DSIM_F32)
        hipLaunchKernelGGL(tangent_kernel<float>, dim3(b->n_env), dim3(64), 0, static_cast<hipStream_t>(stream),
                           view<float>(b), static_cast<const float*>(q), static_cast<const float*>(g_ambient),
                           static_cast<float*>(g_tangent));
    else
        hipLaunchKernelGGL(tangent_kernel<double>, dim3(b->n_env), dim3(64), 0, static_cast<hipStream_t>(stream),
                           view<double>(b), static_cast<const double*>(q), static_cast<const double*>(g_ambient),
                           static_cast<double*>(g_tangent));
    return hipGetLastError() == hipSuccess ? DSIM_SUCCESS : DSIM_ERR_LAUNCH;
}

}  // extern "C"
