// dsim_core.h -- per-environment pipeline of the contact step and its
// derivatives, executed by one team of threads (one workgroup on gfx950).
//
// Every phase is written as "work items strided over the team, then a team
// barrier", so that the same source also builds as plain host C++ with a team
// of one thread (a debugging build; the library itself only runs on the GPU).
//
// Spatial vectors are world-frame and taken about the world origin, ordered
// (angular; linear) for motions and (moment; force) for forces.
#pragma once

#include <stddef.h>
#include <stdint.h>

#ifdef DSIM_HOST_BUILD
#include <cmath>
#define DSIM_HD
using std::sqrt;
using std::fabs;
using std::sin;
using std::cos;
#else
#include <hip/hip_runtime.h>
#define DSIM_HD __host__ __device__
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

// status bits and modes (mirrors include/dsim.h)
enum { ST_NCP = 1, ST_RANK = 2, ST_DEGEN = 4, ST_NONFINITE = 8, ST_POLISH = 16 };
enum { BRK = 0, STK = 1, SLD = 2 };
enum { ENTRY_STEP = 0, ENTRY_JAC = 1, ENTRY_VJP = 2 };

template <class R>
struct BatchView {
    int n_env;
    const int32_t *body_off, *dof_off, *cfg_off, *contact_off, *jac_off;
    const int32_t *parent, *jtype, *cbody;
    const R *axis, *jrot, *jpos, *mass, *com, *inertia, *cpoint, *mu;
};

struct Params {
    double dt, gx, gy, gz;
    int gap_mode, ncp_sweeps, ncp_rounds, newton_iters;
    double ncp_tol, rank_tol, mode_eps;
};

struct Dims {
    int NB, NV, NC, K;  // maxima over the batch (K = 3 NC)
};

// --------------------------------------------------------------------------
// small vector helpers
// --------------------------------------------------------------------------
template <class R>
DSIM_HD inline void cross3(const R* a, const R* b, R* o) {
    R x = a[1] * b[2] - a[2] * b[1];
    R y = a[2] * b[0] - a[0] * b[2];
    R z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
template <class R>
DSIM_HD inline R dot3(const R* a, const R* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <class R>
DSIM_HD inline R dot6(const R* a, const R* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}
// motion x motion: (w, v) x (w', v') = (w x w', w x v' + v x w')
template <class R>
DSIM_HD inline void mxm(const R* a, const R* b, R* o) {
    R t0[3], t1[3], t2[3];
    cross3(a, b, t0);
    cross3(a, b + 3, t1);
    cross3(a + 3, b, t2);
    o[0] = t0[0]; o[1] = t0[1]; o[2] = t0[2];
    o[3] = t1[0] + t2[0]; o[4] = t1[1] + t2[1]; o[5] = t1[2] + t2[2];
}
// motion x* force: (w, v) x* (n, f) = (w x n + v x f, w x f)
template <class R>
DSIM_HD inline void mxf(const R* a, const R* f, R* o) {
    R t0[3], t1[3], t2[3];
    cross3(a, f, t0);
    cross3(a + 3, f + 3, t1);
    cross3(a, f + 3, t2);
    o[0] = t0[0] + t1[0]; o[1] = t0[1] + t1[1]; o[2] = t0[2] + t1[2];
    o[3] = t2[0]; o[4] = t2[1]; o[5] = t2[2];
}
// spatial inertia about the world origin, parameters
// I10 = (m, h[3] = m c, Ibar[6] = xx yy zz xy xz yz about the origin):
// I (w, v) = (Ibar w + h x v, m v - h x w)
template <class R>
DSIM_HD inline void iapply(const R* I, const R* m, R* o) {
    const R* w = m;
    const R* v = m + 3;
    R hv[3], hw[3];
    cross3(I + 1, v, hv);
    cross3(I + 1, w, hw);
    o[0] = I[4] * w[0] + I[7] * w[1] + I[8] * w[2] + hv[0];
    o[1] = I[7] * w[0] + I[5] * w[1] + I[9] * w[2] + hv[1];
    o[2] = I[8] * w[0] + I[9] * w[1] + I[6] * w[2] + hv[2];
    o[3] = I[0] * v[0] - hw[0];
    o[4] = I[0] * v[1] - hw[1];
    o[5] = I[0] * v[2] - hw[2];
}
template <class R>
DSIM_HD inline void mat3mul(const R* A, const R* B, R* C) {  // row-major
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
template <class R>
DSIM_HD inline void mat3vec(const R* A, const R* x, R* y) {
    R a = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    R b = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    R c = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
    y[0] = a; y[1] = b; y[2] = c;
}

// --------------------------------------------------------------------------
// per-environment scratch (carved from LDS, or a device workspace)
// --------------------------------------------------------------------------
template <class R>
struct Env {
    int nb, nv, nq, nc, k;
    int e, b0, d0, q0, c0;  // env index and global offsets
    int* hdr;               // small int header: [0] nlev, [1] m, [2] nstk, [3] nsld, [4] rank, [5] status, [6] ok
    int *parent, *jtype, *dof0, *ndof, *cfg0, *lorder, *lstart, *dbody, *dpar, *cbody, *cmode, *vctc, *vcmp,
        *lmode, *rperm, *cperm;
    uint64_t* bmask;
    R *Rw, *pw, *S, *V, *Vp, *Acc, *Fc, *Iw, *Ic, *Bc, *Ec, *xw, *mu, *Winv;
    R *v, *tau, *bias, *af, *vf, *vn, *ap;
    R *Mx, *J, *KT, *G, *g, *Lam, *sig, *Lam0;
    R *IcS, *BtS, *EtS, *aj, *wj, *cj, *Yq, *Yv;
    R *dTq, *dTv, *E, *Minv, *T, *P, *Q;
    R *vrow, *vcol;      // per reduced variable: row and column vectors (3 each)
    R *vdiag;            // per reduced variable: diagonal term
    R *sfr;              // per contact sliding frame: u (2), w, r1 (3)
    double *A, *Z, *Ysc, *rhs, *X, *ytmp, *dsig;
};

template <class T>
DSIM_HD inline T* take(char*& p, size_t n, size_t& total) {
    size_t bytes = (n * sizeof(T) + 15) & ~size_t(15);
    T* r = reinterpret_cast<T*>(p);
    p += bytes;
    total += bytes;
    return r;
}

// Carves the scratch of one environment team out of `base` (nullptr: only
// sizes).  Returns the number of bytes.
template <class R>
DSIM_HD inline size_t carve(char* base, const Dims& d, int entry, Env<R>& E) {
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
    E.Rw = take<R>(p, 9 * NB, tot);
    E.pw = take<R>(p, 3 * NB, tot);
    E.S = take<R>(p, 6 * NV, tot);
    E.V = take<R>(p, 6 * NB, tot);
    E.Acc = take<R>(p, 6 * NB, tot);
    E.Fc = take<R>(p, 6 * NB, tot);
    E.Iw = take<R>(p, 10 * NB, tot);
    E.Ic = take<R>(p, 10 * NB, tot);
    E.xw = take<R>(p, 3 * NC, tot);
    E.mu = take<R>(p, NC, tot);
    E.Winv = take<R>(p, 9 * NC, tot);
    E.v = take<R>(p, NV, tot);
    E.tau = take<R>(p, NV, tot);
    E.bias = take<R>(p, NV, tot);
    E.af = take<R>(p, NV, tot);
    E.vf = take<R>(p, NV, tot);
    E.vn = take<R>(p, NV, tot);
    E.ap = take<R>(p, NV, tot);
    E.Mx = take<R>(p, NV * NV, tot);
    E.J = take<R>(p, K * NV, tot);
    E.KT = take<R>(p, K * NV, tot);
    E.G = take<R>(p, K * K, tot);
    E.g = take<R>(p, K, tot);
    E.Lam = take<R>(p, K, tot);
    E.sig = take<R>(p, K, tot);
    E.Lam0 = take<R>(p, K, tot);
    E.vrow = take<R>(p, 3 * K, tot);
    E.vcol = take<R>(p, 3 * K, tot);
    E.vdiag = take<R>(p, K, tot);
    E.sfr = take<R>(p, 8 * NC, tot);
    E.A = take<double>(p, K * K, tot);
    E.rhs = take<double>(p, K, tot);
    E.X = take<double>(p, K, tot);
    E.ytmp = take<double>(p, K, tot);
    E.dsig = take<double>(p, K, tot);
    if (entry != ENTRY_STEP) {
        E.Vp = take<R>(p, 6 * NB, tot);
        E.Bc = take<R>(p, 36 * NB, tot);
        E.Ec = take<R>(p, 18 * NB, tot);
        E.IcS = take<R>(p, 6 * NV, tot);
        E.BtS = take<R>(p, 6 * NV, tot);
        E.EtS = take<R>(p, 3 * NV, tot);
        E.aj = take<R>(p, 6 * NV, tot);
        E.wj = take<R>(p, 6 * NV, tot);
        E.cj = take<R>(p, 6 * NV, tot);
        E.Yq = take<R>(p, 6 * NV, tot);
        E.Yv = take<R>(p, 6 * NV, tot);
        E.dTq = take<R>(p, NV * NV, tot);
        E.dTv = take<R>(p, NV * NV, tot);
        E.E = take<R>(p, K * NV, tot);
        E.Minv = take<R>(p, NV * NV, tot);
        E.T = take<R>(p, NV * K, tot);
        E.P = take<R>(p, (NV * NV > K * K ? NV * NV : K * K), tot);
        E.Q = take<R>(p, NV * NV, tot);
        E.Z = take<double>(p, K * K, tot);
        E.Ysc = take<double>(p, K * K, tot);
    }
    return tot;
}

// --------------------------------------------------------------------------
// model tables and kinematics
// --------------------------------------------------------------------------
template <class R>
DSIM_HD void load_env(const Team& T, Env<R>& E, const BatchView<R>& B, int e, const R* v, const R* tau) {
    E.e = e;
    E.b0 = B.body_off[e];
    E.d0 = B.dof_off[e];
    E.q0 = B.cfg_off[e];
    E.c0 = B.contact_off[e];
    E.nb = B.body_off[e + 1] - E.b0;
    E.nv = B.dof_off[e + 1] - E.d0;
    E.nq = B.cfg_off[e + 1] - E.q0;
    E.nc = B.contact_off[e + 1] - E.c0;
    E.k = 3 * E.nc;
    if (T.tid == 0) {
        int nb = E.nb;
        int dof = 0, cfg = 0;
        int depth[64];
        for (int b = 0; b < nb; ++b) {
            int par = B.parent[E.b0 + b];
            int jt = B.jtype[E.b0 + b];
            E.parent[b] = par;
            E.jtype[b] = jt;
            E.dof0[b] = dof;
            E.cfg0[b] = cfg;
            int nd = (jt == 1) ? 6 : 1;
            E.ndof[b] = nd;
            uint64_t m = (par >= 0) ? E.bmask[par] : 0ull;
            for (int i = 0; i < nd; ++i) {
                E.dbody[dof + i] = b;
                E.dpar[dof + i] = (i > 0) ? dof + i - 1 : (par >= 0 ? E.dof0[par] + E.ndof[par] - 1 : -1);
                m |= 1ull << (dof + i);
            }
            E.bmask[b] = m;
            depth[b] = (par >= 0) ? depth[par] + 1 : 0;
            dof += nd;
            cfg += (jt == 1) ? 7 : 1;
        }
        // bodies grouped by depth (level order), parents before children
        int maxd = 0;
        for (int b = 0; b < nb; ++b) maxd = depth[b] > maxd ? depth[b] : maxd;
        int nlev = nb ? maxd + 1 : 0;
        int pos = 0;
        for (int L = 0; L < nlev; ++L) {
            E.lstart[L] = pos;
            for (int b = 0; b < nb; ++b)
                if (depth[b] == L) E.lorder[pos++] = b;
        }
        E.lstart[nlev] = pos;
        E.hdr[0] = nlev;
        for (int i = 1; i < 16; ++i) E.hdr[i] = 0;
    }
    for (int i = T.tid; i < E.nv; i += T.nt) {
        E.v[i] = v[E.d0 + i];
        E.tau[i] = tau[E.d0 + i];
    }
    for (int c = T.tid; c < E.nc; c += T.nt) {
        E.cbody[c] = B.cbody[E.c0 + c];
        E.mu[c] = B.mu[E.c0 + c];
    }
    T.sync();
}

// World placement, motion subspace and velocity of body b (parent done).
template <class R>
DSIM_HD void fk_body(Env<R>& E, const BatchView<R>& B, const R* q, int b) {
    const int gb = E.b0 + b;
    const int par = E.parent[b];
    R* Rw = E.Rw + 9 * b;
    R* pw = E.pw + 3 * b;
    const R* qq = q + E.q0 + E.cfg0[b];
    if (E.jtype[b] == 1) {
        R x = qq[3], y = qq[4], z = qq[5], w = qq[6];
        Rw[0] = 1 - 2 * (y * y + z * z); Rw[1] = 2 * (x * y - z * w);     Rw[2] = 2 * (x * z + y * w);
        Rw[3] = 2 * (x * y + z * w);     Rw[4] = 1 - 2 * (x * x + z * z); Rw[5] = 2 * (y * z - x * w);
        Rw[6] = 2 * (x * z - y * w);     Rw[7] = 2 * (y * z + x * w);     Rw[8] = 1 - 2 * (x * x + y * y);
        pw[0] = qq[0]; pw[1] = qq[1]; pw[2] = qq[2];
        const int d = E.dof0[b];
        for (int c = 0; c < 3; ++c) {
            R* Sl = E.S + 6 * (d + c);      // linear body-frame axis c
            R* Sa = E.S + 6 * (d + 3 + c);  // angular body-frame axis c
            R ax[3] = {Rw[c], Rw[3 + c], Rw[6 + c]};
            Sl[0] = 0; Sl[1] = 0; Sl[2] = 0;
            Sl[3] = ax[0]; Sl[4] = ax[1]; Sl[5] = ax[2];
            R pxa[3];
            cross3(pw, ax, pxa);
            Sa[0] = ax[0]; Sa[1] = ax[1]; Sa[2] = ax[2];
            Sa[3] = pxa[0]; Sa[4] = pxa[1]; Sa[5] = pxa[2];
        }
    } else {
        const R* a = B.axis + 3 * gb;
        const R th = qq[0];
        const R s = sin(th), c = cos(th), omc = 1 - c;
        // Rodrigues rotation about the unit axis a
        R Rot[9] = {c + omc * a[0] * a[0],        omc * a[0] * a[1] - s * a[2], omc * a[0] * a[2] + s * a[1],
                    omc * a[1] * a[0] + s * a[2], c + omc * a[1] * a[1],        omc * a[1] * a[2] - s * a[0],
                    omc * a[2] * a[0] - s * a[1], omc * a[2] * a[1] + s * a[0], c + omc * a[2] * a[2]};
        R Rj[9];
        mat3mul(B.jrot + 9 * gb, Rot, Rj);
        const R* jp = B.jpos + 3 * gb;
        if (par < 0) {
            for (int i = 0; i < 9; ++i) Rw[i] = Rj[i];
            pw[0] = jp[0]; pw[1] = jp[1]; pw[2] = jp[2];
        } else {
            mat3mul(E.Rw + 9 * par, Rj, Rw);
            R t[3];
            mat3vec(E.Rw + 9 * par, jp, t);
            pw[0] = E.pw[3 * par] + t[0];
            pw[1] = E.pw[3 * par + 1] + t[1];
            pw[2] = E.pw[3 * par + 2] + t[2];
        }
        R ax[3];
        mat3vec(Rw, a, ax);
        R* Sd = E.S + 6 * E.dof0[b];
        R pxa[3];
        cross3(pw, ax, pxa);
        Sd[0] = ax[0]; Sd[1] = ax[1]; Sd[2] = ax[2];
        Sd[3] = pxa[0]; Sd[4] = pxa[1]; Sd[5] = pxa[2];
    }
}

// Body velocities V_b = V_parent + sum_d S_d x_d for a velocity vector x.
template <class R>
DSIM_HD void body_velocity(Env<R>& E, const R* x, R* Vout, int b) {
    const int par = E.parent[b];
    R* Vb = Vout + 6 * b;
    for (int i = 0; i < 6; ++i) Vb[i] = (par >= 0) ? Vout[6 * par + i] : R(0);
    for (int j = 0; j < E.ndof[b]; ++j) {
        const int d = E.dof0[b] + j;
        const R* Sd = E.S + 6 * d;
        for (int i = 0; i < 6; ++i) Vb[i] += Sd[i] * x[d];
    }
}

template <class R>
DSIM_HD void kinematics(const Team& T, Env<R>& E, const BatchView<R>& B, const R* q) {
    const int nlev = E.hdr[0];
    for (int L = 0; L < nlev; ++L) {
        const int s = E.lstart[L], n = E.lstart[L + 1] - s;
        for (int i = T.tid; i < n; i += T.nt) {
            const int b = E.lorder[s + i];
            fk_body(E, B, q, b);
            body_velocity(E, E.v, E.V, b);
        }
        T.sync();
    }
    // world inertias and contact points
    for (int b = T.tid; b < E.nb; b += T.nt) {
        const int gb = E.b0 + b;
        const R* Rw = E.Rw + 9 * b;
        const R m = B.mass[gb];
        R c[3];
        mat3vec(Rw, B.com + 3 * gb, c);
        c[0] += E.pw[3 * b]; c[1] += E.pw[3 * b + 1]; c[2] += E.pw[3 * b + 2];
        const R* in = B.inertia + 6 * gb;
        R Ib[9] = {in[0], in[3], in[4], in[3], in[1], in[5], in[4], in[5], in[2]};
        R t[9], Iw[9];
        mat3mul(Rw, Ib, t);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Iw[3 * i + j] = t[3 * i] * Rw[3 * j] + t[3 * i + 1] * Rw[3 * j + 1] + t[3 * i + 2] * Rw[3 * j + 2];
        const R cc = dot3(c, c);
        R* I = E.Iw + 10 * b;
        I[0] = m;
        I[1] = m * c[0]; I[2] = m * c[1]; I[3] = m * c[2];
        I[4] = Iw[0] + m * (cc - c[0] * c[0]);
        I[5] = Iw[4] + m * (cc - c[1] * c[1]);
        I[6] = Iw[8] + m * (cc - c[2] * c[2]);
        I[7] = Iw[1] - m * c[0] * c[1];
        I[8] = Iw[2] - m * c[0] * c[2];
        I[9] = Iw[5] - m * c[1] * c[2];
        for (int i = 0; i < 10; ++i) E.Ic[10 * b + i] = I[i];
    }
    for (int c = T.tid; c < E.nc; c += T.nt) {
        const int b = E.cbody[c];
        R x[3];
        mat3vec(E.Rw + 9 * b, B.cpoint + 3 * (E.c0 + c), x);
        E.xw[3 * c] = x[0] + E.pw[3 * b];
        E.xw[3 * c + 1] = x[1] + E.pw[3 * b + 1];
        E.xw[3 * c + 2] = x[2] + E.pw[3 * b + 2];
    }
    T.sync();
    // composite inertias (children listed after parents)
    for (int i = T.tid; i < 10; i += T.nt)
        for (int b = E.nb - 1; b > 0; --b) {
            const int par = E.parent[b];
            if (par >= 0) E.Ic[10 * par + i] += E.Ic[10 * b + i];
        }
    T.sync();
}

// Composite-rigid-body mass matrix: M[j][k] = S_j . (Ic_{body(k)} S_k) for
// j on the ancestor chain of k.  Written to the lower triangle of Mx.
template <class R>
DSIM_HD void mass_matrix(const Team& T, Env<R>& E) {
    const int n = E.nv;
    for (int i = T.tid; i < n * n; i += T.nt) E.Mx[i] = 0;
    T.sync();
    for (int k = T.tid; k < n; k += T.nt) {
        R F[6];
        iapply(E.Ic + 10 * E.dbody[k], E.S + 6 * k, F);
        for (int j = k; j >= 0; j = E.dpar[j]) E.Mx[k * n + j] = dot6(E.S + 6 * j, F);
    }
    T.sync();
}

// Recursive Newton-Euler in world coordinates.  acc: per-dof accelerations
// (nullptr = 0); fscale: world contact forces are Lam * fscale (0 = none).
// Leaves body accelerations in Acc and composite forces in Fc; writes the
// generalised forces to out (if not null).
template <class R>
DSIM_HD void rnea(const Team& T, Env<R>& E, const Params& P, const R* acc, R fscale, R* out) {
    const int nlev = E.hdr[0];
    for (int L = 0; L < nlev; ++L) {
        const int s = E.lstart[L], n = E.lstart[L + 1] - s;
        for (int i = T.tid; i < n; i += T.nt) {
            const int b = E.lorder[s + i];
            const int par = E.parent[b];
            R* Ab = E.Acc + 6 * b;
            const R* Vb = E.V + 6 * b;
            if (par >= 0) {
                for (int c = 0; c < 6; ++c) Ab[c] = E.Acc[6 * par + c];
            } else {
                Ab[0] = 0; Ab[1] = 0; Ab[2] = 0;
                Ab[3] = R(-P.gx); Ab[4] = R(-P.gy); Ab[5] = R(-P.gz);
            }
            R Vrel[6];
            for (int c = 0; c < 6; ++c) Vrel[c] = Vb[c] - (par >= 0 ? E.V[6 * par + c] : R(0));
            R vp[6];
            mxm(Vb, Vrel, vp);
            for (int c = 0; c < 6; ++c) Ab[c] += vp[c];
            if (acc) {
                for (int j = 0; j < E.ndof[b]; ++j) {
                    const int d = E.dof0[b] + j;
                    for (int c = 0; c < 6; ++c) Ab[c] += E.S[6 * d + c] * acc[d];
                }
            }
            R IA[6], IV[6], VxIV[6];
            const R* I = E.Iw + 10 * b;
            iapply(I, Ab, IA);
            iapply(I, Vb, IV);
            mxf(Vb, IV, VxIV);
            R* F = E.Fc + 6 * b;
            for (int c = 0; c < 6; ++c) F[c] = IA[c] + VxIV[c];
        }
        T.sync();
    }
    if (fscale != R(0)) {
        if (T.tid == 0) {
            for (int c = 0; c < E.nc; ++c) {
                const int b = E.cbody[c];
                R f[3] = {E.Lam[3 * c] * fscale, E.Lam[3 * c + 1] * fscale, E.Lam[3 * c + 2] * fscale};
                R xf[3];
                cross3(E.xw + 3 * c, f, xf);
                R* F = E.Fc + 6 * b;
                F[0] -= xf[0]; F[1] -= xf[1]; F[2] -= xf[2];
                F[3] -= f[0]; F[4] -= f[1]; F[5] -= f[2];
            }
        }
        T.sync();
    }
    for (int i = T.tid; i < 6; i += T.nt)
        for (int b = E.nb - 1; b > 0; --b) {
            const int par = E.parent[b];
            if (par >= 0) E.Fc[6 * par + i] += E.Fc[6 * b + i];
        }
    T.sync();
    if (out)
        for (int d = T.tid; d < E.nv; d += T.nt) out[d] = dot6(E.S + 6 * d, E.Fc + 6 * E.dbody[d]);
    T.sync();
}

// Tree-sparse factorisation M = L^T D L (L unit lower triangular with the
// sparsity of the dof ancestor chains), in place in Mx: strictly lower part
// holds L, the diagonal holds D.  Eliminates from the leaves up, so no fill
// appears outside the chains.
template <class R>
DSIM_HD void ltdl(const Team& T, Env<R>& E) {
    const int n = E.nv;
    R* M = E.Mx;
    R* tmp = E.ap;  // scratch row
    for (int k = n - 1; k >= 0; --k) {
        for (int i = T.tid; i < k; i += T.nt) tmp[i] = M[k * n + i];
        T.sync();
        const R dk = M[k * n + k];
        for (int i = T.tid; i < k; i += T.nt) {
            // dofs below k on its ancestor chain: those that move body(k)
            if (!((E.bmask[E.dbody[k]] >> i) & 1ull)) continue;
            const R a = tmp[i] / dk;
            M[k * n + i] = a;
            for (int j = i; j >= 0; j = E.dpar[j]) M[i * n + j] -= a * tmp[j];
        }
        T.sync();
    }
}

// Solve M x = b in place with the factors (one thread per right-hand side).
template <class R>
DSIM_HD inline void ltdl_solve(const Env<R>& E, R* x, int stride) {
    const int n = E.nv;
    const R* M = E.Mx;
    for (int i = n - 1; i >= 0; --i) {
        const R xi = x[i * stride];
        for (int j = E.dpar[i]; j >= 0; j = E.dpar[j]) x[j * stride] -= M[i * n + j] * xi;
    }
    for (int i = 0; i < n; ++i) x[i * stride] /= M[i * n + i];
    for (int i = 0; i < n; ++i) {
        R s = x[i * stride];
        for (int j = E.dpar[i]; j >= 0; j = E.dpar[j]) s -= M[i * n + j] * x[j * stride];
        x[i * stride] = s;
    }
}

// --------------------------------------------------------------------------
// contacts: Jacobian, Delassus operator
// --------------------------------------------------------------------------
template <class R>
DSIM_HD void contact_jacobian(const Team& T, Env<R>& E) {
    const int n = E.nv, k = E.k;
    for (int idx = T.tid; idx < k * n; idx += T.nt) {
        const int row = idx / n, d = idx - row * n;
        const int c = row / 3, r = row - 3 * c;
        const int b = E.cbody[c];
        R val = 0;
        if ((E.bmask[b] >> d) & 1ull) {
            const R* Sd = E.S + 6 * d;
            R wx[3];
            cross3(Sd, E.xw + 3 * c, wx);
            val = Sd[3 + r] + wx[r];
        }
        E.J[idx] = val;
    }
    T.sync();
}

// K^T = J M^-1 (k x n), G = J M^-1 J^T, g = J v_f (+ phi/dt)
template <class R>
DSIM_HD void delassus(const Team& T, Env<R>& E, const Params& P) {
    const int n = E.nv, k = E.k;
    for (int idx = T.tid; idx < k * n; idx += T.nt) E.KT[idx] = E.J[idx];
    T.sync();
    for (int r = T.tid; r < k; r += T.nt) ltdl_solve(E, E.KT + r * n, 1);
    T.sync();
    for (int idx = T.tid; idx < k * k; idx += T.nt) {
        const int a = idx / k, c = idx - a * k;
        if (c > a) continue;
        R s = 0;
        const R* x = E.KT + a * n;
        const R* y = E.J + c * n;
        for (int i = 0; i < n; ++i) s += x[i] * y[i];
        E.G[a * k + c] = s;
        E.G[c * k + a] = s;
    }
    for (int r = T.tid; r < k; r += T.nt) {
        R s = 0;
        const R* x = E.J + r * n;
        for (int i = 0; i < n; ++i) s += x[i] * E.vf[i];
        if (P.gap_mode == 1 && (r % 3) == 2) s += E.xw[r] / R(P.dt);
        E.g[r] = s;
    }
    T.sync();
    // inverse of each 3x3 diagonal block (local solves)
    for (int c = T.tid; c < E.nc; c += T.nt) {
        const R* G = E.G;
        R W[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) W[3 * i + j] = G[(3 * c + i) * k + 3 * c + j];
        R tr = W[0] + W[4] + W[8];
        R eps = tr * R(1e-12);
        W[0] += eps; W[4] += eps; W[8] += eps;
        R c00 = W[4] * W[8] - W[5] * W[7], c01 = W[5] * W[6] - W[3] * W[8], c02 = W[3] * W[7] - W[4] * W[6];
        R det = W[0] * c00 + W[1] * c01 + W[2] * c02;
        R id = R(1) / det;
        R* Wi = E.Winv + 9 * c;
        Wi[0] = c00 * id;
        Wi[1] = (W[2] * W[7] - W[1] * W[8]) * id;
        Wi[2] = (W[1] * W[5] - W[2] * W[4]) * id;
        Wi[3] = c01 * id;
        Wi[4] = (W[0] * W[8] - W[2] * W[6]) * id;
        Wi[5] = (W[2] * W[3] - W[0] * W[5]) * id;
        Wi[6] = c02 * id;
        Wi[7] = (W[1] * W[6] - W[0] * W[7]) * id;
        Wi[8] = (W[0] * W[4] - W[1] * W[3]) * id;
    }
    T.sync();
}

// --------------------------------------------------------------------------
// NCP: block Gauss-Seidel with local solves, then Newton on the mode-fixed
// equations through the reduced system.
// --------------------------------------------------------------------------

// Unit slip direction t solving (s I + r Wt) t = bt for s > 0, with Wt given
// by its eigen-decomposition (l1 >= l2 >= 0, unit eigenvector (e0, e1) of l1)
// and bt by its coordinates beta in that basis.  |t(s)| decreases in s;
// Newton on 1/|t(s)| = 1 (the trust-region secular equation).
template <class R>
DSIM_HD inline void slip_direction(R l1, R l2, R e0, R e1, R beta1, R beta2, R r, R& t0, R& t1) {
    const R p1 = r * l1, p2 = r * (l2 > R(0) ? l2 : R(0));
    const R tiny = R(1e-30);
    R sv = 0;
    if (p2 <= R(1e-12) * (p1 + tiny)) sv = fabs(beta2);
    if (p1 + sv <= tiny) sv = fabs(beta1) + fabs(beta2);
    for (int it = 0; it < 40; ++it) {
        const R d1 = sv + p1, d2 = sv + p2;
        const R q1 = beta1 / d1, q2 = d2 > tiny ? beta2 / d2 : R(0);
        const R n2 = q1 * q1 + q2 * q2;
        const R nrm = sqrt(n2);
        if (!(nrm > R(0))) break;
        const R psi = R(1) / nrm - R(1);
        const R dn2 = q1 * q1 / d1 + (d2 > tiny ? q2 * q2 / d2 : R(0));
        const R dpsi = dn2 / (n2 * nrm);
        if (!(dpsi > R(0))) break;
        R sn = sv - psi / dpsi;
        if (sn <= R(0)) sn = R(0.5) * sv;
        const R ds = fabs(sn - sv);
        sv = sn;
        if (ds <= R(4) * R(sizeof(R) == 4 ? 1.2e-7 : 2.3e-16) * (sv + p1)) break;
    }
    const R d1 = sv + p1, d2 = sv + p2;
    const R q1 = d1 > tiny ? beta1 / d1 : R(0), q2 = d2 > tiny ? beta2 / d2 : R(0);
    const R u0 = e0 * q1 - e1 * q2, u1 = e1 * q1 + e0 * q2;
    const R nu = sqrt(u0 * u0 + u1 * u1);
    if (nu > R(0)) { t0 = u0 / nu; t1 = u1 / nu; } else { t0 = 1; t1 = 0; }
}

// One-contact problem sigma = W Lam + b.  Separation if the normal free
// velocity is non-negative, else the sticking impulse if it lies in the
// cone, else the sliding impulse on the cone boundary.
//
// Sliding: sigma_N = 0 gives Lam_N = -(b_N + W_NT . Lam_T) / W_NN, so
// sigma_T = Wt Lam_T + bt with the Schur complement Wt = W_TT - W_TN W_NT^T / W_NN
// and bt = b_T - W_TN b_N / W_NN.  With Lam_T = -r t (|t| = 1, r = mu Lam_N)
// and sigma_T = s t (s > 0):  (s I + r Wt) t = bt, which fixes t(r); r itself
// solves g(r) = r (W_NN - mu W_NT . t(r)) + mu b_N = 0, with g(0) = mu b_N < 0:
// bracketed, then refined by regula falsi (Illinois variant).
template <class R>
DSIM_HD inline int local_solve(const R* W, const R* Wi, const R* b, R mu, R* lam) {
    if (b[2] >= R(0)) {
        lam[0] = lam[1] = lam[2] = 0;
        return BRK;
    }
    R s[3];
    mat3vec(Wi, b, s);
    s[0] = -s[0]; s[1] = -s[1]; s[2] = -s[2];
    const R nt = sqrt(s[0] * s[0] + s[1] * s[1]);
    if (s[2] > R(0) && nt <= mu * s[2]) {
        lam[0] = s[0]; lam[1] = s[1]; lam[2] = s[2];
        return STK;
    }
    const R wnn = W[8];
    if (mu <= R(0) || !(wnn > R(0))) {
        lam[0] = 0; lam[1] = 0;
        lam[2] = wnn > R(0) ? -b[2] / wnn : R(0);
        return SLD;
    }
    const R w00 = W[0] - W[2] * W[6] / wnn;
    const R w11 = W[4] - W[5] * W[7] / wnn;
    const R w01 = R(0.5) * ((W[1] - W[2] * W[7] / wnn) + (W[3] - W[5] * W[6] / wnn));
    const R bt0 = b[0] - W[2] * b[2] / wnn, bt1 = b[1] - W[5] * b[2] / wnn;
    // eigen-decomposition of the symmetric 2x2 Wt; (e0, e1) is the larger of
    // (l1 - w11, w01) and (w01, l1 - w00), both solutions of (Wt - l1 I) e = 0
    const R disc = sqrt(R(0.25) * (w00 - w11) * (w00 - w11) + w01 * w01);
    const R l1 = R(0.5) * (w00 + w11) + disc, l2 = R(0.5) * (w00 + w11) - disc;
    R e0 = l1 - w11, e1 = w01;
    {
        const R f0 = w01, f1 = l1 - w00;
        if (f0 * f0 + f1 * f1 > e0 * e0 + e1 * e1) { e0 = f0; e1 = f1; }
        const R nn = sqrt(e0 * e0 + e1 * e1);
        if (nn > R(0)) { e0 /= nn; e1 /= nn; } else { e0 = 1; e1 = 0; }
    }
    const R beta1 = e0 * bt0 + e1 * bt1, beta2 = -e1 * bt0 + e0 * bt1;
    R t0 = 1, t1 = 0;
    auto gfun = [&](R r) -> R {
        slip_direction(l1, l2, e0, e1, beta1, beta2, r, t0, t1);
        return r * (wnn - mu * (W[6] * t0 + W[7] * t1)) + mu * b[2];
    };
    R rlo = 0, glo = mu * b[2];
    R rhi = -mu * b[2] / wnn, ghi = gfun(rhi);
    for (int it = 0; it < 60 && !(ghi > R(0)); ++it) {
        rlo = rhi; glo = ghi;
        rhi *= R(2);
        ghi = gfun(rhi);
    }
    R r = rhi;
    if (ghi > R(0)) {
        int side = 0;
        const R rtol = R(sizeof(R) == 4 ? 1e-7 : 1e-15);
        for (int it = 0; it < 100; ++it) {
            r = (rlo * ghi - rhi * glo) / (ghi - glo);
            if (!(r > rlo && r < rhi)) r = R(0.5) * (rlo + rhi);
            const R gr = gfun(r);
            if (gr > R(0)) {
                rhi = r; ghi = gr;
                if (side == 1) glo *= R(0.5);
                side = 1;
            } else {
                rlo = r; glo = gr;
                if (side == -1) ghi *= R(0.5);
                side = -1;
            }
            if (rhi - rlo <= rtol * rhi || gr == R(0)) break;
        }
    }
    gfun(r);
    lam[0] = -r * t0;
    lam[1] = -r * t1;
    lam[2] = r / mu;
    return SLD;
}

// `sweeps` block Gauss-Seidel sweeps, run by wavefront 0 (sigma = G Lam + g
// is kept up to date in LDS; each contact update is computed redundantly by
// all lanes, then the lanes update sigma row-parallel).
template <class R>
DSIM_HD void nsgs(const Team& T, Env<R>& E, int sweeps) {
    const int k = E.k, nc = E.nc;
    if (T.wave == 0) {
        for (int s = 0; s < sweeps; ++s) {
            for (int c = 0; c < nc; ++c) {
                const int o = 3 * c;
                R W[9];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) W[3 * i + j] = E.G[(o + i) * k + o + j];
                R L[3] = {E.Lam[o], E.Lam[o + 1], E.Lam[o + 2]};
                R b[3];
                for (int i = 0; i < 3; ++i) b[i] = E.sig[o + i] - (W[3 * i] * L[0] + W[3 * i + 1] * L[1] + W[3 * i + 2] * L[2]);
                R Ln[3];
                int md = local_solve(W, E.Winv + 9 * c, b, E.mu[c], Ln);
                R d0 = Ln[0] - L[0], d1 = Ln[1] - L[1], d2 = Ln[2] - L[2];
                T.wave_sync();
                for (int r = T.lane; r < k; r += T.wsize)
                    E.sig[r] += E.G[r * k + o] * d0 + E.G[r * k + o + 1] * d1 + E.G[r * k + o + 2] * d2;
                if (T.lane == 0) {
                    E.Lam[o] = Ln[0]; E.Lam[o + 1] = Ln[1]; E.Lam[o + 2] = Ln[2];
                    E.lmode[c] = md;
                }
                T.wave_sync();
            }
        }
    }
    T.sync();
}

template <class R>
DSIM_HD void update_sigma(const Team& T, Env<R>& E) {
    const int k = E.k;
    for (int r = T.tid; r < k; r += T.nt) {
        R s = E.g[r];
        for (int c = 0; c < k; ++c) s += E.G[r * k + c] * E.Lam[c];
        E.sig[r] = s;
    }
    T.sync();
}

// Reduced variables of the mode set in E.cmode (Section III.C, Appendix B):
// sticking contacts first (3 each), then sliding contacts (2 each, in the
// tangent plane of the cone R = [Lam/|Lam|, e_z x sigma_T/|sigma_T|]).  Row
// vectors select the equation rows; the sliding rows are scaled so that the
// coefficients stay bounded (first row: e_z, second row w u_perp with
// w = mu Lam_N / (mu Lam_N + |sigma_T|) and diagonal 1 - w).
template <class R>
DSIM_HD void reduced_vars(const Team& T, Env<R>& E) {
    if (T.tid == 0) {
        int m = 0, nstk = 0, nsld = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int c = 0; c < E.nc; ++c) {
                const int md = E.cmode[c];
                if (pass == 0 && md == STK) {
                    for (int a = 0; a < 3; ++a) {
                        E.vctc[m] = c;
                        E.vcmp[m] = a;
                        for (int i = 0; i < 3; ++i) {
                            E.vrow[3 * m + i] = (i == a) ? R(1) : R(0);
                            E.vcol[3 * m + i] = (i == a) ? R(1) : R(0);
                        }
                        E.vdiag[m] = 0;
                        ++m;
                    }
                    ++nstk;
                } else if (pass == 1 && md == SLD) {
                    const int o = 3 * c;
                    R s0 = E.sig[o], s1 = E.sig[o + 1];
                    R ns = sqrt(s0 * s0 + s1 * s1);
                    R u0 = ns > R(0) ? s0 / ns : R(1), u1 = ns > R(0) ? s1 / ns : R(0);
                    R L0 = E.Lam[o], L1 = E.Lam[o + 1], L2 = E.Lam[o + 2];
                    R nl = sqrt(L0 * L0 + L1 * L1 + L2 * L2);
                    R mln = E.mu[c] * L2;
                    R w = (mln + ns) > R(0) ? mln / (mln + ns) : R(1);
                    R* f = E.sfr + 8 * c;
                    f[0] = u0; f[1] = u1; f[2] = w;
                    f[3] = L0 / nl; f[4] = L1 / nl; f[5] = L2 / nl;
                    // variable along r1 = Lam/|Lam|: row e_z
                    E.vctc[m] = c; E.vcmp[m] = 0;
                    E.vrow[3 * m] = 0; E.vrow[3 * m + 1] = 0; E.vrow[3 * m + 2] = 1;
                    E.vcol[3 * m] = f[3]; E.vcol[3 * m + 1] = f[4]; E.vcol[3 * m + 2] = f[5];
                    E.vdiag[m] = 0;
                    ++m;
                    // variable along r2 = e_z x u: row w u_perp, diagonal 1 - w
                    E.vctc[m] = c; E.vcmp[m] = 1;
                    E.vrow[3 * m] = -w * u1; E.vrow[3 * m + 1] = w * u0; E.vrow[3 * m + 2] = 0;
                    E.vcol[3 * m] = -u1; E.vcol[3 * m + 1] = u0; E.vcol[3 * m + 2] = 0;
                    E.vdiag[m] = 1 - w;
                    ++m;
                    ++nsld;
                }
            }
        E.hdr[1] = m;
        E.hdr[2] = nstk;
        E.hdr[3] = nsld;
    }
    T.sync();
}

// A = rows^T G cols + diag (FP64), m x m row-major.
template <class R>
DSIM_HD void build_A(const Team& T, Env<R>& E) {
    const int m = E.hdr[1], k = E.k;
    for (int idx = T.tid; idx < m * m; idx += T.nt) {
        const int i = idx / m, j = idx - i * m;
        const int ci = 3 * E.vctc[i], cj = 3 * E.vctc[j];
        const R* ri = E.vrow + 3 * i;
        const R* cv = E.vcol + 3 * j;
        double s = 0;
        for (int a = 0; a < 3; ++a) {
            if (ri[a] == R(0)) continue;
            double t = 0;
            for (int b = 0; b < 3; ++b) t += double(E.G[(ci + a) * k + cj + b]) * double(cv[b]);
            s += double(ri[a]) * t;
        }
        if (i == j) s += double(E.vdiag[i]);
        E.A[idx] = s;
    }
    T.sync();
}

// In-place elimination of A with pivoting.  Sticking variables first, with
// symmetric (diagonal) pivoting: the sticking block is G_SS, symmetric
// positive semidefinite, so this is a pivoted LDL^T (square-root-free
// Cholesky) of it.  Then complete pivoting on the Schur complement of the
// sliding block.  Pivots below rank_tol times the largest initial pivot end
// the elimination; the remaining variables are set to zero by the solves
// (basic solution).  Leaves L (unit, below the diagonal) and U in A, the row
// and column permutations in rperm/cperm, the rank in hdr[4].
template <class R>
DSIM_HD void factor_A(const Team& T, Env<R>& E, double rank_tol) {
    const int m = E.hdr[1];
    const int nst = 3 * E.hdr[2];
    double* A = E.A;
    if (T.tid == 0) {
        for (int i = 0; i < m; ++i) { E.rperm[i] = i; E.cperm[i] = i; }
        E.hdr[4] = m;
    }
    T.sync();
    double scale = 0;
    for (int i = 0; i < m * m; ++i) { double a = fabs(A[i]); scale = a > scale ? a : scale; }
    const double tol = rank_tol * (scale > 0 ? scale : 1.0);
    int rank = 0;
    bool stick_phase = nst > 0;
    for (int p = 0; p < m; ++p) {
        // pivot choice (every thread computes the same, reading A)
        int pr = -1, pc = -1;
        double best = -1;
        if (stick_phase && p < nst) {
            for (int i = p; i < nst; ++i) {
                double a = fabs(A[i * m + i]);
                if (a > best) { best = a; pr = i; pc = i; }
            }
            // sticking block exhausted: its remaining rows and columns are
            // (numerically) zero, continue with complete pivoting
            if (best <= tol) stick_phase = false;
        }
        if (!(stick_phase && p < nst)) {
            best = -1;
            for (int i = p; i < m; ++i)
                for (int j = p; j < m; ++j) {
                    double a = fabs(A[i * m + j]);
                    if (a > best) { best = a; pr = i; pc = j; }
                }
        }
        if (best <= tol || pr < 0) break;
        T.sync();
        // swap rows p <-> pr and columns p <-> pc
        if (pr != p)
            for (int j = T.tid; j < m; j += T.nt) { double t = A[p * m + j]; A[p * m + j] = A[pr * m + j]; A[pr * m + j] = t; }
        T.sync();
        if (pc != p)
            for (int i = T.tid; i < m; i += T.nt) { double t = A[i * m + p]; A[i * m + p] = A[i * m + pc]; A[i * m + pc] = t; }
        if (T.tid == 0) {
            int t = E.rperm[p]; E.rperm[p] = E.rperm[pr]; E.rperm[pr] = t;
            t = E.cperm[p]; E.cperm[p] = E.cperm[pc]; E.cperm[pc] = t;
        }
        T.sync();
        const double piv = A[p * m + p];
        for (int i = p + 1 + T.tid; i < m; i += T.nt) A[i * m + p] /= piv;
        T.sync();
        const int rem = m - p - 1;
        for (int idx = T.tid; idx < rem * rem; idx += T.nt) {
            const int i = p + 1 + idx / rem, j = p + 1 + idx % rem;
            A[i * m + j] -= A[i * m + p] * A[p * m + j];
        }
        T.sync();
        rank = p + 1;
    }
    if (T.tid == 0) E.hdr[4] = rank;
    T.sync();
}

// Solve A x = b for one right-hand side (one thread), b permuted by rperm,
// free variables zero, result scattered by cperm.  x and b may alias only
// through the scratch y.
DSIM_HD inline void lu_solve(const double* A, int m, int rank, const int* rperm, const int* cperm,
                             const double* b, int bstride, double* y, double* x, int xstride) {
    for (int i = 0; i < m; ++i) y[i] = b[rperm[i] * bstride];
    for (int i = 0; i < rank; ++i) {
        double s = y[i];
        for (int j = 0; j < i; ++j) s -= A[i * m + j] * y[j];
        y[i] = s;
    }
    for (int i = rank; i < m; ++i) y[i] = 0;
    for (int i = rank - 1; i >= 0; --i) {
        double s = y[i];
        for (int j = i + 1; j < rank; ++j) s -= A[i * m + j] * y[j];
        y[i] = s / A[i * m + i];
    }
    for (int i = 0; i < m; ++i) x[cperm[i] * xstride] = y[i];
}

}  // namespace dsim
