// dsim_core.h -- types, small spatial-algebra helpers and the per-environment
// scratch of the contact step and its derivatives.
//
// One team of threads (a workgroup on gfx950) processes one environment at a
// time.  Every phase is written as "work items strided over the team, then a
// team barrier", so that the same source also builds as plain host C++ with a
// team of one thread (a debugging build; the library itself runs on the GPU).
//
// Spatial vectors are world-aligned and taken about a reference point `org`
// (the world position of body 0), ordered (angular; linear) for motions and
// (moment; force) for forces.
//
// Precision: the tree recursions (kinematics, inertias, the tree-sparse
// factorisation of M, inverse dynamics and its partial derivatives) and the
// reduced contact system run in FP64 in both forms; the dense products of the
// Delassus operator and of the Jacobian assembly, the Gauss-Seidel sweeps and
// the large per-environment matrices use the working precision R (float in
// the FP32 form).
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <limits.h>

#ifdef DSIM_HOST_BUILD
#include <cmath>
#include <cstdio>
#define DSIM_HD
#define DSIM_INLINE inline
using std::cos;
using std::fabs;
using std::sin;
using std::sqrt;
#else
#include <hip/hip_runtime.h>
// Every per-environment function is inlined into its kernel: a function
// compiled on its own sees the LDS buffers behind Env's pointers as generic
// (flat) addresses and reaches LDS with flat loads and stores, several times
// slower than the LDS instructions the kernel body gets.
#define DSIM_HD __host__ __device__ __attribute__((always_inline))
#define DSIM_INLINE inline
#endif

namespace dsim {

// --------------------------------------------------------------------------
// team of threads
// --------------------------------------------------------------------------
struct Team {
    int tid, nt;     // thread id within the team, team size
    int lane, wave;  // lane within the wavefront, wavefront id
    int wsize;       // wavefront size (64 on gfx950)
#ifdef DSIM_HOST_BUILD
    void sync() const {}
    void wave_sync() const {}
#else
    __device__ void sync() const { __syncthreads(); }
    __device__ void wave_sync() const {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
#endif
};

// Wavefront 0 of a team working alone: the same code as for a whole team,
// with the wavefront's barrier in place of the team's.  Chains of small
// dependent steps (the refinement's Newton iterations and factorisations)
// run on it, so that each step costs a wavefront barrier instead of a
// workgroup barrier; the other wavefronts wait at the next team barrier.
struct WaveTeam : Team {
#ifdef DSIM_HOST_BUILD
    void sync() const {}
#else
    __device__ void sync() const { wave_sync(); }
#endif
};

// The wavefront-0 view of team T (called by the threads of wavefront 0).
DSIM_HD inline WaveTeam wave_team(const Team& T) {
    WaveTeam W;
    W.tid = T.lane;
    W.nt = T.nt < T.wsize ? T.nt : T.wsize;
    W.lane = T.lane;
    W.wave = 0;
    W.wsize = T.wsize;
    return W;
}

// Slots of the team reductions: three per wavefront of the largest team
// (512 threads, 8 wavefronts; team_max2 stores a pair per wavefront and the
// natural map's sum one more); the host build (a debugging build whose team
// threads are plain threads) uses two per thread.
#ifdef DSIM_HOST_BUILD
constexpr int kRedSlots = 2 * 512;
#else
constexpr int kRedSlots = 3 * 8;
#endif

// Maximum of (v, i) over the team: the larger value wins, equal values go to
// the smaller index, so that a strided scan in increasing index order
// followed by this reduction picks what one serial scan with a strict
// comparison picks.  Threads without a candidate pass (-1, INT_MAX).  Every
// thread gets the result.  The slots are reused: a caller separates two
// calls by at least one team barrier after the first call returns.
template <class TT>
DSIM_HD inline void team_argmax(const TT& T, double* redv, int* redi, double& v, int& i) {
#ifdef DSIM_HOST_BUILD
    redv[T.tid] = v;
    redi[T.tid] = i;
    T.sync();
    v = redv[0];
    i = redi[0];
    for (int w = 1; w < T.nt; ++w)
        if (redv[w] > v || (redv[w] == v && redi[w] < i)) {
            v = redv[w];
            i = redi[w];
        }
#else
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(i, off, 64);
        if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
        }
    }
    if (T.lane == 0) {
        redv[T.wave] = v;
        redi[T.wave] = i;
    }
    T.sync();
    const int nw = (T.nt + 63) >> 6;
    v = redv[0];
    i = redi[0];
    for (int w = 1; w < nw; ++w)
        if (redv[w] > v || (redv[w] == v && redi[w] < i)) {
            v = redv[w];
            i = redi[w];
        }
#endif
}

// Maxima of two values over the team (NaN never wins), returned to every
// thread; the same slot reuse rule as team_argmax.
template <class TT>
DSIM_HD inline void team_max2(const TT& T, double* redv, double& a, double& b) {
#ifdef DSIM_HOST_BUILD
    redv[2 * T.tid] = a;
    redv[2 * T.tid + 1] = b;
    T.sync();
    a = redv[0];
    b = redv[1];
    for (int w = 1; w < T.nt; ++w) {
        a = redv[2 * w] > a ? redv[2 * w] : a;
        b = redv[2 * w + 1] > b ? redv[2 * w + 1] : b;
    }
#else
    for (int off = 32; off >= 1; off >>= 1) {
        const double oa = __shfl_xor(a, off, 64);
        const double ob = __shfl_xor(b, off, 64);
        a = oa > a ? oa : a;
        b = ob > b ? ob : b;
    }
    if (T.lane == 0) {
        redv[2 * T.wave] = a;
        redv[2 * T.wave + 1] = b;
    }
    T.sync();
    const int nw = (T.nt + 63) >> 6;
    a = redv[0];
    b = redv[1];
    for (int w = 1; w < nw; ++w) {
        a = redv[2 * w] > a ? redv[2 * w] : a;
        b = redv[2 * w + 1] > b ? redv[2 * w + 1] : b;
    }
#endif
}

// status bits and modes (mirror include/dsim.h)
enum { ST_NCP = 1, ST_RANK = 2, ST_DEGEN = 4, ST_NONFINITE = 8, ST_POLISH = 16, ST_SIZE = 32 };
enum { BRK = 0, STK = 1, SLD = 2 };
// entries: the step; the step and its full Jacobian; the step and its VJP;
// the step followed by q+ = q (+) dt v+; the adjoint of that fused map; the
// step, its VJP and the gradients in the body masses and friction
// coefficients; the step, its Jacobian and the parameter columns
enum { ENTRY_STEP = 0, ENTRY_JAC = 1, ENTRY_VJP = 2, ENTRY_SINT = 3, ENTRY_RVJP = 4, ENTRY_PVJP = 5, ENTRY_PJAC = 6 };
// The first pass of a derivative entry's step as two launches (internal, not
// entries of the C ABI): the tree recursions and the contact system (G, g,
// the inverses of G's diagonal blocks, v_f, a_f) written to the hand-over
// record (ASM), then the contact solve from that record in a much smaller
// on-chip layout, so that more environment teams share a compute unit while
// they iterate (NCP).  The fallback pass of a derivative entry starts from
// the same record (FBK: the NCP layout with the fallback solvers' second
// k x k matrix).
enum { ENTRY_ASM = 7, ENTRY_NCP = 8, ENTRY_FBK = 9 };
// FP64 impulses handed from the step launch to the derivative launch: one
// slot of 3 x (maximum contacts) per environment, followed by the work its
// contact solve executed (read back for the flop count): Gauss-Seidel
// sweeps of the first pass, Levenberg-Marquardt iterations and linear
// solves and ADMM iterations of the fallback pass
constexpr int kLdWork = 63;
// then whether the first pass left the environment unsolved (1) or not (0)
constexpr int kLdFallback = 67;
constexpr int kLdStride = 68;

DSIM_HD inline bool entry_has_derivative(int entry) {
    return entry == ENTRY_JAC || entry == ENTRY_VJP || entry == ENTRY_RVJP || entry == ENTRY_PVJP ||
           entry == ENTRY_PJAC;
}
// entries that assemble the full Jacobian (they need the T and CZ buffers)
DSIM_HD inline bool entry_is_jacobian(int entry) { return entry == ENTRY_JAC || entry == ENTRY_PJAC; }

template <class R>
struct BatchView {
    int n_env;
    const int32_t *body_off, *dof_off, *cfg_off, *contact_off, *jac_off;
    const int32_t *parent, *jtype, *cbody;
    const R *axis, *jrot, *jpos, *mass, *com, *inertia, *cpoint, *mu;
    const int32_t* order;  // optional launch list (block index -> environment)
    const int32_t* pjac_off;  // offsets of the parameter Jacobians
    const R* cradius;         // sphere radius per contact (nullptr: all points)
};

struct Params {
    double dt, gx, gy, gz;
    int gap_mode, ncp_sweeps, ncp_rounds, newton_iters;
    double ncp_tol, rank_tol, mode_eps;
    double kp, kd;  // Baumgarte gains (gap mode 1)
    int pass;       // step launches: 0 the first pass, 1 the fallback pass of the solve
};

struct Dims {
    int NB, NV, NC, K;  // maxima over the batch (K = 3 NC)
};

// Bitwise equality of two floating-point values (NaN payloads and the sign
// of zero included).
template <class T>
DSIM_HD inline bool same_bits(T a, T b) {
    if constexpr (sizeof(T) == 4) {
        uint32_t x, y;
        __builtin_memcpy(&x, &a, 4);
        __builtin_memcpy(&y, &b, 4);
        return x == y;
    } else {
        static_assert(sizeof(T) == 8, "float or double");
        uint64_t x, y;
        __builtin_memcpy(&x, &a, 8);
        __builtin_memcpy(&y, &b, 8);
        return x == y;
    }
}

// --------------------------------------------------------------------------
// small vector helpers (3-vectors, spatial 6-vectors)
// --------------------------------------------------------------------------
template <class T>
DSIM_HD inline void cross3(const T* a, const T* b, T* o) {
    T x = a[1] * b[2] - a[2] * b[1];
    T y = a[2] * b[0] - a[0] * b[2];
    T z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
template <class T>
DSIM_HD inline T dot3(const T* a, const T* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <class T>
DSIM_HD inline T dot6(const T* a, const T* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}
// motion x motion: (w, v) x (w', v') = (w x w', w x v' + v x w')
template <class T>
DSIM_HD inline void mxm(const T* a, const T* b, T* o) {
    T t0[3], t1[3], t2[3];
    cross3(a, b, t0);
    cross3(a, b + 3, t1);
    cross3(a + 3, b, t2);
    o[0] = t0[0]; o[1] = t0[1]; o[2] = t0[2];
    o[3] = t1[0] + t2[0]; o[4] = t1[1] + t2[1]; o[5] = t1[2] + t2[2];
}
// motion x* force: (w, v) x* (n, f) = (w x n + v x f, w x f)
template <class T>
DSIM_HD inline void mxf(const T* a, const T* f, T* o) {
    T t0[3], t1[3], t2[3];
    cross3(a, f, t0);
    cross3(a + 3, f + 3, t1);
    cross3(a, f + 3, t2);
    o[0] = t0[0] + t1[0]; o[1] = t0[1] + t1[1]; o[2] = t0[2] + t1[2];
    o[3] = t2[0]; o[4] = t2[1]; o[5] = t2[2];
}
// spatial inertia about the reference point, 10 parameters
// I = (m, h[3] = m c, Ibar[6] = xx yy zz xy xz yz about the point):
// I (w, v) = (Ibar w + h x v, m v - h x w)
template <class T>
DSIM_HD inline void iapply(const T* I, const T* m, T* o) {
    const T* w = m;
    const T* v = m + 3;
    T hv[3], hw[3];
    cross3(I + 1, v, hv);
    cross3(I + 1, w, hw);
    o[0] = I[4] * w[0] + I[7] * w[1] + I[8] * w[2] + hv[0];
    o[1] = I[7] * w[0] + I[5] * w[1] + I[9] * w[2] + hv[1];
    o[2] = I[8] * w[0] + I[9] * w[1] + I[6] * w[2] + hv[2];
    o[3] = I[0] * v[0] - hw[0];
    o[4] = I[0] * v[1] - hw[1];
    o[5] = I[0] * v[2] - hw[2];
}
template <class T>
DSIM_HD inline void mat3mul(const T* A, const T* B, T* C) {  // row-major
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
template <class T>
DSIM_HD inline void mat3vec(const T* A, const T* x, T* y) {
    T a = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    T b = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    T c = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
    y[0] = a; y[1] = b; y[2] = c;
}

// --------------------------------------------------------------------------
// per-environment scratch (carved from LDS, or a device workspace)
// --------------------------------------------------------------------------
template <class R>
struct Env {
    int nb, nv, nq, nc, k;
    int e, b0, d0, q0, c0;  // env index and global offsets
    // small int header: [0] levels, [1] m (reduced size), [2] sticking
    // contacts, [4] rank, [5] status, [6] refinement ok, [9..13] refinement
    // control, [10] non-finite output, [14] sweep state repeated
    int* hdr;
    int *parent, *jtype, *dof0, *ndof, *cfg0, *lorder, *lstart, *dbody, *dpar, *cbody, *cmode, *lmode;
    int *vctc, *vcmp, *rperm, *cperm;  // reduced variables: contact, component; pivots
    uint64_t* bmask;                   // per body: dofs that move it (its own and its ancestors')
    // FP64 tree quantities
    double *Rw, *pw, *S, *V, *Vp, *Acc, *Fc, *Iw, *Ic, *Bc, *Ec, *xw, *org;
    double* crad;  // per contact: 0 for a body-fixed point, else the sphere radius
    double *v, *tau, *bias, *af, *vf, *vn, *ap, *Mx, *Mi;
    double *IcS, *BtS, *EtS, *aj, *wj, *cj, *Yq, *Yv;
    double* gint;  // adjoint of q carried through the position update
    double* scr;  // FP64 solve scratch, max(K, NV) x NV
    // working-precision quantities
    R *mu, *Winv, *J, *KT, *g, *Lam, *sig, *Lam0;
    R* sig0;      // step entries: sigma and modes at the end of the previous
    int* lmode0;  // sweep round (with Lam0, the impulses)
    R *dTq, *dTv, *E, *T, *P, *Q;
    // FP64 contact system; reduced variables: row and column vectors, diagonal
    double *vrow, *vcol, *vdiag;
    double *Gd, *gd, *Ld, *Ld1, *dfr;
    double *A, *Z, *Ysc, *rhs, *X, *ytmp, *dsig, *dsc;
    double* A2;  // step entries: a second k x k FP64 matrix for the damped Newton fallback of the solve
    double* redv;  // team reductions: one (value, index) slot per wavefront
    int* redi;
};

#ifdef DSIM_HOST_BUILD
// Host build only: when set, every region carve() hands out comes from this
// allocator with exactly its own size (so that an address checker sees each
// region's bounds); the byte count is unchanged.
inline void* (*host_region_alloc)(size_t) = nullptr;
#endif

template <class T>
DSIM_HD inline T* take(char*& p, size_t n, size_t& total) {
    size_t bytes = (n * sizeof(T) + 15) & ~size_t(15);
#ifdef DSIM_HOST_BUILD
    if (host_region_alloc) {
        total += bytes;
        return static_cast<T*>(host_region_alloc(n * sizeof(T)));
    }
#endif
    T* r = reinterpret_cast<T*>(p);
    p += bytes;
    total += bytes;
    return r;
}

// The layout of the NCP and FBK launches: the contact system, the solver's
// state and the reduced system only (the tree quantities stay in the
// hand-over record), and for FBK the fallback's second k x k matrix.  Every
// other pointer is null.
template <class R>
DSIM_HD inline size_t carve_ncp(char* base, const Dims& d, Env<R>& E, bool fallback) {
    size_t tot = 0;
    char* p = base;
    const int NV = d.NV, NC = d.NC, K = d.K, KK = K * K;
    E = Env<R>{};
    E.hdr = take<int>(p, 16, tot);
    E.cmode = take<int>(p, NC, tot);
    E.lmode = take<int>(p, NC, tot);
    E.lmode0 = take<int>(p, NC, tot);
    E.vctc = take<int>(p, K, tot);
    E.vcmp = take<int>(p, K, tot);
    E.rperm = take<int>(p, K, tot);
    E.cperm = take<int>(p, K, tot);
    E.vf = take<double>(p, NV, tot);
    E.af = take<double>(p, NV, tot);
    E.vn = take<double>(p, NV, tot);
    E.ap = take<double>(p, NV, tot);
    E.mu = take<R>(p, NC, tot);
    E.Winv = take<R>(p, 9 * NC, tot);
    E.g = take<R>(p, K, tot);
    E.Lam = take<R>(p, K, tot);
    E.sig = take<R>(p, K, tot);
    E.Lam0 = take<R>(p, K, tot);
    E.sig0 = take<R>(p, K, tot);
    E.vrow = take<double>(p, 3 * K, tot);
    E.vcol = take<double>(p, 3 * K, tot);
    E.vdiag = take<double>(p, K, tot);
    E.Gd = take<double>(p, KK, tot);
    E.gd = take<double>(p, K, tot);
    E.Ld = take<double>(p, K, tot);
    E.Ld1 = take<double>(p, K, tot);
    E.dfr = take<double>(p, 4 * NC, tot);
    E.A = take<double>(p, KK, tot);
    E.A2 = fallback ? take<double>(p, KK, tot) : nullptr;
    E.rhs = take<double>(p, K, tot);
    E.X = take<double>(p, K, tot);
    E.ytmp = take<double>(p, K, tot);
    E.dsig = take<double>(p, K, tot);
    E.dsc = take<double>(p, 12, tot);
    E.redv = take<double>(p, kRedSlots, tot);
    E.redi = take<int>(p, kRedSlots, tot);
    return tot;
}

// Carves the scratch of one environment team out of `base` (nullptr: only
// sizes).  Returns the number of bytes.
template <class R>
DSIM_HD inline size_t carve(char* base, const Dims& d, int entry, Env<R>& E) {
    if (entry == ENTRY_NCP || entry == ENTRY_FBK) return carve_ncp<R>(base, d, E, entry == ENTRY_FBK);
    size_t tot = 0;
    char* p = base;
    const int NB = d.NB, NV = d.NV, NC = d.NC, K = d.K;
    E.hdr = take<int>(p, 16, tot);
    E.parent = take<int>(p, NB, tot);
    E.jtype = take<int>(p, NB, tot);
    E.dof0 = take<int>(p, NB, tot);
    E.ndof = take<int>(p, NB, tot);
    E.cfg0 = take<int>(p, NB, tot);
    E.lorder = take<int>(p, NB, tot);
    E.lstart = take<int>(p, NB + 1, tot);
    E.dbody = take<int>(p, NV, tot);
    E.dpar = take<int>(p, NV, tot);
    E.cbody = take<int>(p, NC, tot);
    E.cmode = take<int>(p, NC, tot);
    E.lmode = take<int>(p, NC, tot);
    E.vctc = take<int>(p, K, tot);
    E.vcmp = take<int>(p, K, tot);
    E.rperm = take<int>(p, K, tot);
    E.cperm = take<int>(p, K, tot);
    E.bmask = take<uint64_t>(p, NB, tot);
    E.Rw = take<double>(p, 9 * NB, tot);
    E.pw = take<double>(p, 3 * NB, tot);
    E.S = take<double>(p, 6 * NV, tot);
    const bool deriv = entry_has_derivative(entry);
    if (deriv) {
        E.V = take<double>(p, 6 * NB, tot);
        E.Acc = take<double>(p, 6 * NB, tot);
        E.Fc = take<double>(p, 6 * NB, tot);
        E.Iw = take<double>(p, 10 * NB, tot);
        E.Ic = take<double>(p, 10 * NB, tot);
    }
    E.xw = take<double>(p, 3 * NC, tot);
    E.crad = take<double>(p, NC, tot);
    E.org = take<double>(p, 3, tot);
    E.v = take<double>(p, NV, tot);
    E.tau = take<double>(p, NV, tot);
    E.bias = take<double>(p, NV, tot);
    E.af = take<double>(p, NV, tot);
    E.vf = take<double>(p, NV, tot);
    E.vn = take<double>(p, NV, tot);
    E.ap = take<double>(p, NV, tot);
    // Buffers with disjoint lifetimes share storage.
    //  * derivative entries (the step's quantities come from the hand-over
    //    record; M^-1 is read there, in device memory, and not copied):
    //    mx holds the composites B_b and X_b until dtau/dq, dtau/dv and E
    //    are formed, then (Jacobian) CZ and P = I + T J; the union holds the
    //    per-dof derivative vectors, then the columns of the reduced solve
    //    and the transposed-solve vector, then Q = P M^-1; Gd holds
    //    Z = A^-1 B, then T = -K C Z when it fits.
    //  * step-only entries: the factors of M, then the FP64 product J M^-1,
    //    then (once the Delassus operator is formed) the reduced-system
    //    matrix A; and one region for the body velocities, accelerations,
    //    forces and inertias of the dynamics (dead once RNEA and the mass
    //    matrix are done), then M^-1 (dead once J M^-1 is formed), then Gd.
    //    Four teams of a 36-dof tree with 8 contacts then fit one
    //    compute unit's LDS.
    const int NN = NV * NV, KK = K * K;
    double* un = nullptr;
    double* gda = nullptr;
    double* ax = nullptr;
    // FP64 step entries whose J storage (dead once the Delassus matrix is
    // formed) holds the reduced matrix A and the reduced-variable vectors:
    // those live there, and K^T is the FP64 product J M^-1 itself, kept in
    // mx through the solve
    const bool in_j = !deriv && sizeof(R) == sizeof(double) && size_t(K) * NV >= size_t(KK) + 7 * size_t(K);
    if (!deriv) {
        size_t mx = size_t(NN > K * NV ? NN : K * NV);
        if (mx < size_t(KK)) mx = size_t(KK);
        // the fallback's second k x k matrix follows A in mx, or (J layout)
        // Gd in the shared region
        if (!in_j && mx < size_t(2) * KK) mx = size_t(2) * KK;
        E.Mx = take<double>(p, mx, tot);
        E.scr = E.Mx;
        ax = E.Mx;
        size_t ur = size_t(38) * NB;
        if (ur < size_t(NN)) ur = size_t(NN);
        if (ur < size_t(KK)) ur = size_t(KK);
        if (in_j && ur < size_t(2) * KK) ur = size_t(2) * KK;
        double* u = take<double>(p, ur, tot);
        E.V = u;
        E.Acc = u + 6 * NB;
        E.Fc = u + 12 * NB;
        E.Iw = u + 18 * NB;
        E.Ic = u + 28 * NB;
        E.Mi = u;
        gda = u;
    } else {
        const size_t cmp = size_t(54) * NB * sizeof(double);
        const size_t czb = entry_is_jacobian(entry) ? size_t(KK > NN ? KK : NN) * sizeof(R) : 0;
        const size_t b = cmp > czb ? cmp : czb;
        E.Mx = take<double>(p, (b + sizeof(double) - 1) / sizeof(double), tot);
        E.Mi = nullptr;  // set to the hand-over record's copy
    }
    if (deriv) {
        size_t u = size_t(45) * NV;
        if (u < size_t(KK)) u = size_t(KK);
        if (u < size_t(K)) u = size_t(K);
        const size_t qd = (size_t(NN) * sizeof(R) + sizeof(double) - 1) / sizeof(double);
        if (u < qd) u = qd;
        un = take<double>(p, u, tot);
        E.scr = un;
    }
    E.mu = take<R>(p, NC, tot);
    E.Winv = take<R>(p, 9 * NC, tot);
    E.J = take<R>(p, K * NV, tot);
    if (in_j) {
        E.KT = reinterpret_cast<R*>(E.Mx);
        ax = reinterpret_cast<double*>(E.J);
    } else {
        E.KT = take<R>(p, K * NV, tot);
    }
    E.g = take<R>(p, K, tot);
    E.Lam = take<R>(p, K, tot);
    E.sig = take<R>(p, K, tot);
    E.Lam0 = take<R>(p, K, tot);
    if (!deriv) {
        E.sig0 = take<R>(p, K, tot);
        E.lmode0 = take<int>(p, NC, tot);
    } else {
        E.sig0 = nullptr;
        E.lmode0 = nullptr;
    }
    if (in_j) {
        E.vrow = ax + KK;
        E.vcol = E.vrow + 3 * K;
        E.vdiag = E.vcol + 3 * K;
    } else {
        E.vrow = take<double>(p, 3 * K, tot);
        E.vcol = take<double>(p, 3 * K, tot);
        E.vdiag = take<double>(p, K, tot);
    }
    E.Gd = gda ? gda : take<double>(p, KK, tot);
    E.gd = take<double>(p, K, tot);
    E.Ld = take<double>(p, K, tot);
    E.Ld1 = take<double>(p, K, tot);
    E.dfr = take<double>(p, 4 * NC, tot);
    E.A = ax ? ax : take<double>(p, KK, tot);
    E.A2 = deriv ? nullptr : (in_j ? E.Gd + KK : E.Mx + KK);
    E.rhs = take<double>(p, K, tot);
    E.X = take<double>(p, K, tot);
    E.ytmp = take<double>(p, K, tot);
    E.dsig = take<double>(p, K, tot);
    E.dsc = take<double>(p, 12, tot);
    E.redv = take<double>(p, kRedSlots, tot);
    E.redi = take<int>(p, kRedSlots, tot);
    if (deriv) {
        E.Vp = take<double>(p, 6 * NB, tot);
        E.gint = take<double>(p, NV, tot);
        double* d = un;
        E.IcS = d; d += 6 * NV;
        E.BtS = d; d += 6 * NV;
        E.EtS = d; d += 3 * NV;
        E.aj = d; d += 6 * NV;
        E.wj = d; d += 6 * NV;
        E.cj = d; d += 6 * NV;
        E.Yq = d; d += 6 * NV;
        E.Yv = d; d += 6 * NV;
        E.Bc = E.Mx;
        E.Ec = E.Mx + 36 * NB;
        E.Ysc = un;
        E.Q = reinterpret_cast<R*>(un);
        E.P = reinterpret_cast<R*>(E.Mx);
        E.dTq = take<R>(p, NN, tot);
        E.dTv = take<R>(p, NN, tot);
        E.E = take<R>(p, K * NV, tot);
        E.Z = E.Gd;
        if (entry_is_jacobian(entry))
            E.T = (size_t(NV) * K * sizeof(R) <= size_t(KK) * sizeof(double)) ? reinterpret_cast<R*>(E.Gd)
                                                                                : take<R>(p, NV * K, tot);
        else
            E.T = nullptr;
    }
    return tot;
}

// --------------------------------------------------------------------------
// hand-over record of the step launch
// --------------------------------------------------------------------------

// In a derivative entry the step launch also writes, per environment, the
// step's quantities that the derivative phases read: placements, motion
// subspaces, velocities, spatial and composite inertias, contact points,
// M^-1, the contact rows J and K^T = J M^-1, sigma, the reduced variables and
// the factorised reduced matrix, v+ and a+.  The derivative launch loads them
// instead of recomputing the step (the recomputation, latency-bound at one
// team per compute unit, was most of that launch).  Byte offsets within one
// record, sized by the launch's maxima.
struct Handover {
    size_t Rw, pw, S, V, Iw, Ic, xw, Mi, dsig, vrow, vcol, vdiag, dfr, A, vn, ap, J, KT;
    size_t rperm, cperm, vctc, vcmp, hdr;
    size_t Gd, gd, vf, af, Winv;  // the contact system, from the ASM launch to the NCP launch
    size_t bytes;
};

template <class R>
DSIM_HD inline Handover handover_layout(const Dims& d) {
    const size_t NB = d.NB, NV = d.NV, NC = d.NC, K = d.K;
    Handover h;
    size_t o = 0;
    auto at = [&o](size_t bytes) {
        const size_t r = o;
        o += (bytes + 15) & ~size_t(15);
        return r;
    };
    const size_t D8 = sizeof(double);
    h.Rw = at(9 * NB * D8);
    h.pw = at(3 * NB * D8);
    h.S = at(6 * NV * D8);
    h.V = at(6 * NB * D8);
    h.Iw = at(10 * NB * D8);
    h.Ic = at(10 * NB * D8);
    h.xw = at(3 * NC * D8);
    h.Mi = at(NV * NV * D8);
    h.dsig = at(K * D8);
    h.vrow = at(3 * K * D8);
    h.vcol = at(3 * K * D8);
    h.vdiag = at(K * D8);
    h.dfr = at(4 * NC * D8);
    h.A = at(K * K * D8);
    h.vn = at(NV * D8);
    h.ap = at(NV * D8);
    h.J = at(K * NV * sizeof(R));
    h.KT = at(K * NV * sizeof(R));
    h.rperm = at(K * sizeof(int));
    h.cperm = at(K * sizeof(int));
    h.vctc = at(K * sizeof(int));
    h.vcmp = at(K * sizeof(int));
    h.hdr = at(4 * sizeof(int));
    h.Gd = at(K * K * D8);
    h.gd = at(K * D8);
    h.vf = at(NV * D8);
    h.af = at(NV * D8);
    h.Winv = at(9 * NC * sizeof(R));
    h.bytes = o;
    return h;
}

// Start of the records in a derivative entry's workspace: after the FP64
// impulses (kLdStride doubles per environment), 16-byte aligned.
DSIM_HD inline char* handover_base(double* ld, int n_env) {
    return reinterpret_cast<char*>(ld + ((size_t(n_env) * kLdStride + 1) & ~size_t(1)));
}

template <class T>
DSIM_HD inline void team_put(const Team& Tm, char* rec, size_t off, const T* src, int n) {
    T* dst = reinterpret_cast<T*>(rec + off);
    for (int i = Tm.tid; i < n; i += Tm.nt) dst[i] = src[i];
}

template <class T>
DSIM_HD inline void team_get(const Team& Tm, const char* rec, size_t off, T* dst, int n) {
    const T* src = reinterpret_cast<const T*>(rec + off);
    for (int i = Tm.tid; i < n; i += Tm.nt) dst[i] = src[i];
}

}  // namespace dsim
