// dsim_host.cpp -- a host (CPU) build of the library's kernel code, for tests.
//
// The kernels are written as "work items strided over the team, then a team
// barrier" (dsim_core.h), so the same source runs on the CPU with a team of
// one thread.  This file instantiates that build: every environment of a
// batch whose arrays are HOST memory is run through run_env exactly as one
// workgroup of the GPU launch would run it, in the same launch order (the
// two passes of the step launch over all environments -- in the derivative
// entries the first as the ASM and NCP launches, the second as the FBK
// launch -- then the derivative launch for the derivative entries).  It is a verification tool (address checking of each
// scratch region, the solver's behaviour on chosen environments), never a
// path of the library: the package has no CPU fallback.
//
// With region_alloc != 0 every region that carve() hands out gets an
// allocation of its own of exactly its size, so that an address checker
// (a host-only build with AddressSanitizer) sees the bounds of each region
// instead of one slab.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#define DSIM_HOST_BUILD 1
#include "../../include/dsim.h"
#include "../../paper_2409_07107_amd/csrc/dsim_pipeline.h"

using namespace dsim;

namespace {

std::vector<void*> g_regions;

void* region_alloc(size_t bytes) {
    void* p = std::malloc(bytes ? bytes : 1);
    std::memset(p, 0xA5, bytes ? bytes : 1);  // uninitialised reads show as garbage
    g_regions.push_back(p);
    return p;
}

void free_regions() {
    for (void* p : g_regions) std::free(p);
    g_regions.clear();
}

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

// One pass of env_kernel<R, entry> over the listed environments.
template <class R>
int pass(const dsim_batch* b, const dsim_params* p, int entry, const R* q, const R* v, const R* tau, const R* gbar,
         const R* gbar2, R* v_next, R* lam, int8_t* mode, int32_t* status, R* o1, R* o2, R* o3, R* o4, R* o5,
         double* ld, int e0, int e1, int region, int solve_pass = 0) {
    const BatchView<R> B = view<R>(b);
    Params P = params_of(p);
    P.pass = solve_pass;
    const Dims D = dims_of(b);
    Env<R> E;
    const size_t bytes = carve<R>(nullptr, D, entry, E);
    std::vector<char> slab;
    Team T;
    T.tid = 0;
    T.nt = 1;
    T.lane = 0;
    T.wave = 0;
    T.wsize = 1;
    for (int blk = e0; blk < e1; ++blk) {
        const int e = b->order ? b->order[blk] : blk;
        if (e < 0 || e >= b->n_env) continue;
        if (b->body_off[e + 1] - b->body_off[e] > D.NB || b->dof_off[e + 1] - b->dof_off[e] > D.NV ||
            b->contact_off[e + 1] - b->contact_off[e] > D.NC) {
            status[e] = ST_SIZE;
            continue;
        }
        if (solve_pass == 1 && !(status[e] & (ST_NCP | ST_POLISH))) continue;
        if (region) {
            host_region_alloc = region_alloc;
            carve<R>(reinterpret_cast<char*>(16), D, entry, E);
            host_region_alloc = nullptr;
        } else {
            slab.assign(bytes, char(0xA5));
            carve<R>(slab.data(), D, entry, E);
        }
        run_env<R>(T, E, B, P, D, entry, e, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4,
                   o5, ld);
        if (region) free_regions();
    }
    return 0;
}

template <class R>
int run(const dsim_batch* b, const dsim_params* p, int entry, const void* q, const void* v, const void* tau,
        const void* gbar, const void* gbar2, void* v_next, void* lam, int8_t* mode, int32_t* status, void* o1,
        void* o2, void* o3, void* o4, void* o5, void* ws, int e0, int e1, int region) {
    auto c = [](const void* x) { return static_cast<const R*>(x); };
    auto w = [](void* x) { return static_cast<R*>(x); };
    double* ld = static_cast<double*>(ws);
    if (!entry_has_derivative(entry)) {
        for (int sp = 0; sp < 2; ++sp)
            pass<R>(b, p, entry, c(q), c(v), c(tau), c(gbar), c(gbar2), w(v_next), w(lam), mode, status, w(o1),
                    w(o2), w(o3), w(o4), w(o5), ld, e0, e1, region, sp);
        return 0;
    }
    // the first step pass as the ASM and NCP launches, then the fallback pass
    // (FBK)
    for (int ent : {int(ENTRY_ASM), int(ENTRY_NCP)})
        pass<R>(b, p, ent, c(q), c(v), c(tau), nullptr, nullptr, w(v_next), w(lam), mode, status, nullptr, nullptr,
                nullptr, nullptr, nullptr, ld, e0, e1, region, 0);
    pass<R>(b, p, ENTRY_FBK, c(q), c(v), c(tau), nullptr, nullptr, w(v_next), w(lam), mode, status, nullptr,
            nullptr, nullptr, nullptr, nullptr, ld, e0, e1, region, 1);
    return pass<R>(b, p, entry, c(q), c(v), c(tau), c(gbar), c(gbar2), w(v_next), w(lam), mode, status, w(o1), w(o2),
                   w(o3), w(o4), w(o5), ld, e0, e1, region);
}

}  // namespace

extern "C" {

// Bytes of one team's scratch (as dsim_lds_bytes) and of the derivative
// entries' hand-over workspace (as dsim_workspace_bytes), host build.
size_t dsim_host_team_bytes(const dsim_batch* b, const dsim_params* p, int entry) {
    const Dims d = dims_of(b);
    if (p->precision == DSIM_F32) {
        Env<float> E;
        return carve<float>(nullptr, d, entry, E);
    }
    Env<double> E;
    return carve<double>(nullptr, d, entry, E);
}

size_t dsim_host_workspace_bytes(const dsim_batch* b, const dsim_params* p) {
    const Dims d = dims_of(b);
    const size_t rec = p->precision == DSIM_F32 ? handover_layout<float>(d).bytes : handover_layout<double>(d).bytes;
    const size_t imp = ((size_t(b->n_env) * kLdStride + 1) & ~size_t(1)) * sizeof(double);
    return imp + size_t(b->n_env) * rec;
}

// Runs `entry` (a dsim_entry) on launch blocks e0 .. e1-1 (environments, or
// positions of b->order) with every pointer in HOST memory; the argument
// meaning follows the library's entry of the same kind.
int dsim_host_run(const dsim_batch* b, const dsim_params* p, int entry, const void* q, const void* v,
                  const void* tau, const void* gbar, const void* gbar2, void* v_next, void* lam, int8_t* mode,
                  int32_t* status, void* o1, void* o2, void* o3, void* o4, void* o5, void* ws, int e0, int e1,
                  int region_alloc) {
    if (p->precision == DSIM_F32)
        return run<float>(b, p, entry, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5, ws,
                          e0, e1, region_alloc);
    return run<double>(b, p, entry, q, v, tau, gbar, gbar2, v_next, lam, mode, status, o1, o2, o3, o4, o5, ws, e0,
                       e1, region_alloc);
}

}  // extern "C"
