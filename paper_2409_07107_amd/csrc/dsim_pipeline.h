// dsim_pipeline.h -- one environment's step (eq. 3-5 and the NCP), its full
// Jacobian (eq. FD_grads, eq. 10-12, Appendix B and D) and its
// vector-Jacobian product.
#pragma once

#include "dsim_core.h"
#include "dsim_ncp.h"
#include "dsim_tree.h"

namespace dsim {

// The step: kinematics, dynamics, factorisation, contacts (step_assemble),
// then NCP and v+ (step_finish).  With a hand-over record (`rec`, laid out by
// `H`), each quantity the derivative phases read is also written there once
// it is final, before its storage is reused.
template <class R>
DSIM_HD void step_assemble(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, const R* q,
                           const Handover* H, char* rec) {
    const int nb = E.nb, n = E.nv, k = E.k, nc = E.nc;
    kinematics(T, E, B, q);
    mass_matrix(T, E);
    rnea(T, E, P, nullptr, 0.0, E.bias);
    if (rec) {
        // the body velocities and inertias share storage with M^-1
        team_put(T, rec, H->Rw, E.Rw, 9 * nb);
        team_put(T, rec, H->pw, E.pw, 3 * nb);
        team_put(T, rec, H->S, E.S, 6 * n);
        team_put(T, rec, H->V, E.V, 6 * nb);
        team_put(T, rec, H->Iw, E.Iw, 10 * nb);
        team_put(T, rec, H->Ic, E.Ic, 10 * nb);
        team_put(T, rec, H->xw, E.xw, 3 * nc);
        T.sync();
    }
    ltdl(T, E);
    tree_inverse(T, E);
    // free motion a_f = M^-1 (tau - b), v_f = v + dt a_f
    for (int i = T.tid; i < n; i += T.nt) {
        double s = 0;
        for (int j = 0; j < n; ++j) s += E.Mi[i * n + j] * (E.tau[j] - E.bias[j]);
        E.af[i] = s;
        E.vf[i] = E.v[i] + P.dt * s;
    }
    T.sync();
    if (rec) {
        // M^-1 shares storage with the Delassus matrices
        team_put(T, rec, H->Mi, E.Mi, n * n);
        T.sync();
    }
    if (k > 0) {
        contact_jacobian(T, E);
        delassus(T, E, P);
    }
    if (rec) {
        // the FP64 solve reuses J's storage
        team_put(T, rec, H->J, E.J, k * n);
        T.sync();
    }
}

// The contact system of the step for the NCP launch: K^T, G (FP64), g
// (FP64), the inverses of G's diagonal blocks, v_f and a_f.
template <class R>
DSIM_HD void put_contact_system(const Team& T, const Env<R>& E, const Handover& H, char* rec) {
    const int n = E.nv, k = E.k;
    team_put(T, rec, H.KT, E.KT, k * n);
    team_put(T, rec, H.Gd, E.Gd, k * k);
    team_put(T, rec, H.gd, E.gd, k);
    team_put(T, rec, H.vf, E.vf, n);
    team_put(T, rec, H.af, E.af, n);
    team_put(T, rec, H.Winv, E.Winv, 9 * E.nc);
}

// The NCP launch's start: sizes and friction coefficients of environment e,
// and the contact system from its record; g in working precision is the
// rounding of its FP64 value, as the Delassus assembly forms it.
// K^T stays in the record (E.KT points there).
template <class R>
DSIM_HD void load_contact_system(const Team& T, Env<R>& E, const BatchView<R>& B, int e, const Handover& H,
                                 char* rec) {
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
    const int n = E.nv, k = E.k;
    if (T.tid == 0)
        for (int i = 0; i < 16; ++i) E.hdr[i] = 0;
    for (int c = T.tid; c < E.nc; c += T.nt) E.mu[c] = B.mu[E.c0 + c];
    team_get(T, rec, H.Gd, E.Gd, k * k);
    team_get(T, rec, H.gd, E.gd, k);
    team_get(T, rec, H.vf, E.vf, n);
    team_get(T, rec, H.af, E.af, n);
    team_get(T, rec, H.Winv, E.Winv, 9 * E.nc);
    E.KT = reinterpret_cast<R*>(rec + H.KT);
    T.sync();
    for (int r = T.tid; r < k; r += T.nt) E.g[r] = R(E.gd[r]);
    T.sync();
}

template <class R>
DSIM_HD void step_finish(const Team& T, Env<R>& E, const Params& P, const Handover* H, char* rec,
                         const R* lam_start) {
    const int n = E.nv, k = E.k, nc = E.nc;
    solve_ncp(T, E, P, lam_start);
    // v+ = v_f + M^-1 J^T Lam and a+ = a_f + M^-1 J^T Lam / dt
    for (int i = T.tid; i < n; i += T.nt) {
        double s = 0;
        for (int c = 0; c < k; ++c) s += double(E.KT[c * n + i]) * E.Ld[c];
        E.vn[i] = E.vf[i] + s;
        E.ap[i] = E.af[i] + s / P.dt;
    }
    T.sync();
    if (rec) {
        // (the NCP launch reads K^T in place)
        if (static_cast<const void*>(E.KT) != static_cast<const void*>(rec + H->KT))
            team_put(T, rec, H->KT, E.KT, k * n);
        team_put(T, rec, H->dsig, E.dsig, k);
        team_put(T, rec, H->vrow, E.vrow, 3 * k);
        team_put(T, rec, H->vcol, E.vcol, 3 * k);
        team_put(T, rec, H->vdiag, E.vdiag, k);
        team_put(T, rec, H->dfr, E.dfr, 4 * nc);
        team_put(T, rec, H->A, E.A, k * k);
        team_put(T, rec, H->vn, E.vn, n);
        team_put(T, rec, H->ap, E.ap, n);
        team_put(T, rec, H->rperm, E.rperm, k);
        team_put(T, rec, H->cperm, E.cperm, k);
        team_put(T, rec, H->vctc, E.vctc, k);
        team_put(T, rec, H->vcmp, E.vcmp, k);
        if (T.tid == 0) {
            int* h = reinterpret_cast<int*>(rec + H->hdr);
            h[0] = E.hdr[1];
            h[1] = E.hdr[2];
            h[2] = E.hdr[4];
        }
    }
    residual_and_flags(T, E, P);
}

template <class R>
DSIM_HD void step_forward(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, const R* q,
                          const Handover* H, char* rec, const R* lam_start) {
    step_assemble(T, E, B, P, q, H, rec);
    step_finish(T, E, P, H, rec, lam_start);
}

// The step's quantities for the derivative, loaded from the record the step
// launch of the same call wrote (its FP64 impulses from `ld`, its modes from
// `mode`): bit for bit what the step computed.
template <class R>
DSIM_HD void load_step(const Team& T, Env<R>& E, const Handover& H, const char* rec, const double* ld,
                       const int8_t* mode) {
    const int nb = E.nb, n = E.nv, k = E.k, nc = E.nc;
    team_get(T, rec, H.Rw, E.Rw, 9 * nb);
    team_get(T, rec, H.pw, E.pw, 3 * nb);
    team_get(T, rec, H.S, E.S, 6 * n);
    team_get(T, rec, H.V, E.V, 6 * nb);
    team_get(T, rec, H.Iw, E.Iw, 10 * nb);
    team_get(T, rec, H.Ic, E.Ic, 10 * nb);
    team_get(T, rec, H.xw, E.xw, 3 * nc);
    // M^-1 is read where the step left it (each entry once per product)
    E.Mi = reinterpret_cast<double*>(const_cast<char*>(rec) + H.Mi);
    team_get(T, rec, H.J, E.J, k * n);
    team_get(T, rec, H.KT, E.KT, k * n);
    team_get(T, rec, H.dsig, E.dsig, k);
    team_get(T, rec, H.vrow, E.vrow, 3 * k);
    team_get(T, rec, H.vcol, E.vcol, 3 * k);
    team_get(T, rec, H.vdiag, E.vdiag, k);
    team_get(T, rec, H.dfr, E.dfr, 4 * nc);
    team_get(T, rec, H.A, E.A, k * k);
    team_get(T, rec, H.vn, E.vn, n);
    team_get(T, rec, H.ap, E.ap, n);
    team_get(T, rec, H.rperm, E.rperm, k);
    team_get(T, rec, H.cperm, E.cperm, k);
    team_get(T, rec, H.vctc, E.vctc, k);
    team_get(T, rec, H.vcmp, E.vcmp, k);
    const double* l = ld + size_t(E.e) * kLdStride;
    for (int r = T.tid; r < k; r += T.nt) {
        E.Ld[r] = l[r];
        E.Lam[r] = R(l[r]);
    }
    for (int c = T.tid; c < nc; c += T.nt) E.cmode[c] = mode[E.c0 + c];
    if (T.tid == 0) {
        const int* h = reinterpret_cast<const int*>(rec + H.hdr);
        E.hdr[1] = h[0];
        E.hdr[2] = h[1];
        E.hdr[4] = h[2];
    }
    T.sync();
}

template <class R>
DSIM_HD void write_step(const Team& T, Env<R>& E, R* v_next, R* lam, int8_t* mode, int32_t* status) {
    bool bad = false;
    for (int i = T.tid; i < E.nv; i += T.nt) {
        v_next[E.d0 + i] = R(E.vn[i]);
        if (!(E.vn[i] == E.vn[i]) || fabs(E.vn[i]) > 1e300) bad = true;
    }
    for (int r = T.tid; r < E.k; r += T.nt) lam[3 * E.c0 + r] = E.Lam[r];
    for (int c = T.tid; c < E.nc; c += T.nt) mode[E.c0 + c] = int8_t(E.cmode[c]);
    if (bad) E.hdr[10] = 1;
    T.sync();
    if (T.tid == 0) status[E.e] = E.hdr[5] | (E.hdr[10] ? ST_NONFINITE : 0);
}

// --------------------------------------------------------------------------
// derivative phases (FP64 tree quantities)
// --------------------------------------------------------------------------

// Per body: B_b (6x6, column mm = B_b e_mm) with
//   B_b w = I_b (w x V_b) + w x* (I_b V_b) + V_b x* (I_b w),
// the change of the body's inertial force under a perturbation w of its
// velocity that is not a rigid transport; and X_b (6x3): the change of the
// contact forces on body b when the body turns by w (the force stays fixed in
// the world while its point moves): X_b w = sum_c (x_c x (w x f_c), w x f_c),
// f_c = Lam_c / dt.  Then composites over subtrees.
template <class R>
DSIM_HD void composites(const Team& T, Env<R>& E, const Params& P) {
    for (int b = T.tid; b < E.nb; b += T.nt) {
        const double* I = E.Iw + 10 * b;
        const double* Vb = E.V + 6 * b;
        double IV[6];
        iapply(I, Vb, IV);
        double* Bm = E.Bc + 36 * b;
        for (int mm = 0; mm < 6; ++mm) {
            double e[6] = {0, 0, 0, 0, 0, 0};
            e[mm] = 1;
            double wxV[6], t1[6], t2[6], Ie[6], t3[6];
            mxm(e, Vb, wxV);
            iapply(I, wxV, t1);
            mxf(e, IV, t2);
            iapply(I, e, Ie);
            mxf(Vb, Ie, t3);
            for (int r = 0; r < 6; ++r) Bm[6 * r + mm] = t1[r] + t2[r] + t3[r];
        }
        double* X = E.Ec + 18 * b;
        for (int i = 0; i < 18; ++i) X[i] = 0;
    }
    T.sync();
    if (T.tid == 0) {
        const double inv = 1.0 / P.dt;
        for (int c = 0; c < E.nc; ++c) {
            const int b = E.cbody[c];
            const double f[3] = {E.Ld[3 * c] * inv, E.Ld[3 * c + 1] * inv, E.Ld[3 * c + 2] * inv};
            const double* x = E.xw + 3 * c;
            double* X = E.Ec + 18 * b;
            // a sphere's contact point moves with its centre, not as a point
            // of the body: turning by w moves it by w x (r n) more, so the
            // actual moment change gains (w x r n) x f; X holds the rigid
            // transport minus the actual change, hence the extra
            // -(w x r n) x f = w (f . r n) - r n (f . w)  (n = e_z)
            const double rad = E.crad[c];
            for (int mm = 0; mm < 3; ++mm) {
                double e[3] = {0, 0, 0};
                e[mm] = 1;
                double gg[3], xg[3];
                cross3(e, f, gg);
                cross3(x, gg, xg);
                for (int r = 0; r < 3; ++r) {
                    X[3 * r + mm] += xg[r];
                    X[3 * (r + 3) + mm] += gg[r];
                }
                if (rad != 0.0) {
                    X[3 * mm + mm] += rad * f[2];
                    X[3 * 2 + mm] -= rad * f[mm];
                }
            }
        }
    }
    T.sync();
    for (int i = T.tid; i < 54; i += T.nt)
        for (int b = E.nb - 1; b > 0; --b) {
            const int par = E.parent[b];
            if (par < 0) continue;
            if (i < 36)
                E.Bc[36 * par + i] += E.Bc[36 * b + i];
            else
                E.Ec[18 * par + i - 36] += E.Ec[18 * b + i - 36];
        }
    T.sync();
}

// Partial derivatives of the generalised forces tau = ID(q, v, a+) - J^T Lam/dt
// (a+ = (v+ - v)/dt, Lam held fixed) in q along the tangent perturbations and
// in v (Section III.A: the terms dUFD/dq, dUFD/dv of eq. FD_grads, with the
// contact-point term of Section III.D for points fixed on the bodies).
//
// Moving joint j by dq_j turns its subtree by the world twist xi = S_j.
// Quantities of the subtree are carried along (a rigid transport, which does
// not change tau_k for k in the subtree) except for the parent's motion:
// the body velocities gain w_j = -xi x V_parent and the accelerations
// a_j + w_j x V_i with a_j = -xi x A_parent - w_j x V_parent; contact forces,
// fixed in the world, change by X w.  Hence, with composites over subtree(k),
//   dtau_k/dq_j = S_k . (Ic_k a_j + Bc_k w_j + Xc_k omega_j)   (joint j moves body(k))
//   dtau_k/dq_j = S_k . (xi x* Fc_j + Ic_j a_j + Bc_j w_j + Xc_j omega_j)
//                                                   (body(k) a strict ancestor)
// and for v, with c_j = -S_j x V_parent + V_body(j) x S_j,
//   dtau_k/dv_j = S_k . (Bc S_j + Ic c_j) over the deeper subtree.
template <class R>
DSIM_HD void id_partials(const Team& T, Env<R>& E, const Params& P) {
    const int n = E.nv;
    for (int d = T.tid; d < n; d += T.nt) {
        const int b = E.dbody[d];
        const int par = E.parent[b];
        const double* Sd = E.S + 6 * d;
        iapply(E.Ic + 10 * b, Sd, E.IcS + 6 * d);
        const double* Bm = E.Bc + 36 * b;
        const double* X = E.Ec + 18 * b;
        for (int c = 0; c < 6; ++c) {
            double s = 0;
            for (int r = 0; r < 6; ++r) s += Bm[6 * r + c] * Sd[r];
            E.BtS[6 * d + c] = s;
        }
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int r = 0; r < 6; ++r) s += X[3 * r + c] * Sd[r];
            E.EtS[3 * d + c] = s;
        }
        double Vl[6], Al[6];
        if (par >= 0) {
            for (int c = 0; c < 6; ++c) {
                Vl[c] = E.V[6 * par + c];
                Al[c] = E.Acc[6 * par + c];
            }
        } else {
            for (int c = 0; c < 6; ++c) Vl[c] = 0;
            Al[0] = 0; Al[1] = 0; Al[2] = 0;
            Al[3] = -P.gx; Al[4] = -P.gy; Al[5] = -P.gz;
        }
        double w[6], a[6], t[6], cj[6];
        mxm(Sd, Vl, t);
        for (int c = 0; c < 6; ++c) w[c] = -t[c];
        mxm(Sd, Al, a);
        mxm(w, Vl, t);
        for (int c = 0; c < 6; ++c) a[c] = -a[c] - t[c];
        mxm(E.V + 6 * b, Sd, t);
        for (int c = 0; c < 6; ++c) cj[c] = w[c] + t[c];
        for (int c = 0; c < 6; ++c) {
            E.aj[6 * d + c] = a[c];
            E.wj[6 * d + c] = w[c];
            E.cj[6 * d + c] = cj[c];
        }
        double y[6], u[6];
        mxf(Sd, E.Fc + 6 * b, y);
        iapply(E.Ic + 10 * b, a, u);
        for (int c = 0; c < 6; ++c) y[c] += u[c];
        for (int r = 0; r < 6; ++r) {
            double s = 0, s2 = 0;
            for (int c = 0; c < 6; ++c) {
                s += Bm[6 * r + c] * w[c];
                s2 += Bm[6 * r + c] * Sd[c];
            }
            y[r] += s + X[3 * r] * Sd[0] + X[3 * r + 1] * Sd[1] + X[3 * r + 2] * Sd[2];
            u[r] = s2;
        }
        for (int c = 0; c < 6; ++c) E.Yq[6 * d + c] = y[c];
        iapply(E.Ic + 10 * b, cj, t);
        for (int c = 0; c < 6; ++c) E.Yv[6 * d + c] = u[c] + t[c];
    }
    T.sync();
    for (int idx = T.tid; idx < n * n; idx += T.nt) {
        const int kk = idx / n, j = idx - kk * n;
        const int bk = E.dbody[kk], bj = E.dbody[j];
        double dq = 0, dv = 0;
        if ((E.bmask[bk] >> j) & 1ull) {
            dq = dot6(E.IcS + 6 * kk, E.aj + 6 * j) + dot6(E.BtS + 6 * kk, E.wj + 6 * j) +
                 dot3(E.EtS + 3 * kk, E.S + 6 * j);
            dv = dot6(E.BtS + 6 * kk, E.S + 6 * j) + dot6(E.IcS + 6 * kk, E.cj + 6 * j);
        } else if ((E.bmask[bj] >> kk) & 1ull) {
            dq = dot6(E.S + 6 * kk, E.Yq + 6 * j);
            dv = dot6(E.S + 6 * kk, E.Yv + 6 * j);
        }
        E.dTq[idx] = R(dq);
        E.dTv[idx] = R(dv);
    }
    T.sync();
}

// E = d(J(q) v+)/dq at fixed v+ (Section III.C: the forward-kinematics
// velocity term at (q, v+), with the contact-point motion of Section III.D):
// for joint j moving the contact body, the point velocity changes by
// xi x (u_body - u_parent) + omega_parent x (xi applied to the point), where
// u are point velocities under v+; plus (1/dt) J_N in gap mode 1.
template <class R>
DSIM_HD void velocity_partials(const Team& T, Env<R>& E, const Params& P) {
    const int nlev = E.hdr[0];
    for (int L = 0; L < nlev; ++L) {
        const int s = E.lstart[L], n = E.lstart[L + 1] - s;
        for (int i = T.tid; i < n; i += T.nt) body_velocity(E, E.vn, E.Vp, E.lorder[s + i]);
        T.sync();
    }
    const int n = E.nv, k = E.k;
    for (int idx = T.tid; idx < k * n; idx += T.nt) {
        const int row = idx / n, j = idx - row * n;
        const int c = row / 3, r = row - 3 * c;
        const int b = E.cbody[c];
        double val = 0;
        if ((E.bmask[b] >> j) & 1ull) {
            const double* x = E.xw + 3 * c;
            const double* Sj = E.S + 6 * j;
            const int par = E.parent[E.dbody[j]];
            double ui[3], ul[3] = {0, 0, 0}, wl[3] = {0, 0, 0};
            const double* Vi = E.Vp + 6 * b;
            cross3(Vi, x, ui);
            for (int a = 0; a < 3; ++a) ui[a] += Vi[3 + a];
            if (par >= 0) {
                const double* Vl = E.Vp + 6 * par;
                cross3(Vl, x, ul);
                for (int a = 0; a < 3; ++a) {
                    ul[a] += Vl[3 + a];
                    wl[a] = Vl[a];
                }
            }
            const double du[3] = {ui[0] - ul[0], ui[1] - ul[1], ui[2] - ul[2]};
            double dx[3], t1[3], t2[3];
            cross3(Sj, x, dx);
            for (int a = 0; a < 3; ++a) dx[a] += Sj[3 + a];
            cross3(Sj, du, t1);
            cross3(wl, dx, t2);
            val = t1[r] + t2[r];
            // a sphere's contact point moves with the centre: it is displaced
            // by xi_ang x (r n) more than a point of the body, which the body
            // rotation carries into the point velocity (n = e_z)
            const double rad = E.crad[c];
            double sn[3] = {0, 0, 0};
            if (rad != 0.0) {
                const double rn[3] = {0, 0, rad};
                double ex[3];
                cross3(Sj, rn, sn);
                cross3(Vi, sn, ex);
                val += ex[r];
            }
            if (P.gap_mode == 1 && r == 2) {
                // d/dq of phi/dt - kp [phi/dt]_- (slope 0 at phi = 0) ...
                const double phi = x[2] + E.org[2];
                val += (1.0 - (phi < 0 ? P.kp : 0.0)) * dx[2] / P.dt;
                // ... and of -kd (J(q) v)_N at fixed v (E.V: body velocities at v)
                if (P.kd != 0.0) {
                    double vi[3], vl[3] = {0, 0, 0}, w0[3] = {0, 0, 0};
                    const double* Wi = E.V + 6 * b;
                    cross3(Wi, x, vi);
                    for (int a = 0; a < 3; ++a) vi[a] += Wi[3 + a];
                    if (par >= 0) {
                        const double* Wl = E.V + 6 * par;
                        cross3(Wl, x, vl);
                        for (int a = 0; a < 3; ++a) {
                            vl[a] += Wl[3 + a];
                            w0[a] = Wl[a];
                        }
                    }
                    const double dv[3] = {vi[0] - vl[0], vi[1] - vl[1], vi[2] - vl[2]};
                    double s1[3], s2[3], s3[3];
                    cross3(Sj, dv, s1);
                    cross3(w0, dx, s2);
                    cross3(Wi, sn, s3);  // sphere term at v (zero for points)
                    val -= P.kd * (s1[2] + s2[2] + s3[2]);
                }
            }
        }
        E.E[idx] = R(val);
    }
    T.sync();
}

// Z = A^-1 B (FP64, basic solution), one thread per column of B; B selects
// the equation rows of each reduced variable (its row vector).  Column rho of
// Z is stored contiguously.
template <class R>
DSIM_HD void reduced_solve(const Team& T, Env<R>& E) {
    const int m = E.hdr[1], k = E.k, rank = E.hdr[4];
    for (int rho = T.tid; rho < k; rho += T.nt) {
        double* y = E.Ysc + rho * m;
        double* z = E.Z + rho * m;
        for (int i = 0; i < m; ++i) {
            const int vi = E.rperm[i];
            const int a = rho - 3 * E.vctc[vi];
            y[i] = (a >= 0 && a < 3) ? E.vrow[3 * vi + a] : 0.0;
        }
        for (int i = 0; i < rank; ++i) {
            double s = y[i];
            for (int j = 0; j < i; ++j) s -= E.A[i * m + j] * y[j];
            y[i] = s;
        }
        for (int i = rank; i < m; ++i) y[i] = 0;
        for (int i = rank - 1; i >= 0; --i) {
            double s = y[i];
            for (int j = i + 1; j < rank; ++j) s -= E.A[i * m + j] * y[j];
            y[i] = s / E.A[i * m + i];
        }
        for (int i = 0; i < m; ++i) z[E.cperm[i]] = y[i];
    }
    T.sync();
}

// Shared by the Jacobian and the VJP: inverse dynamics at a+ with the contact
// forces, composites, the partial derivatives of inverse dynamics and of the
// contact velocities.
template <class R>
DSIM_HD void derivative_partials(const Team& T, Env<R>& E, const Params& P) {
    rnea(T, E, P, E.ap, 1.0 / P.dt, nullptr);
    composites(T, E, P);
    id_partials(T, E, P);
    velocity_partials(T, E, P);
}

// Full Jacobian (Appendix D, eq. total_derivation, impulse form):
//   D0 = [-dt M^-1 dtau/dq, I - dt M^-1 dtau/dv, dt M^-1]
//   dv+/dtheta = D0 + M^-1 J^T dLam,  dLam = -C A^-1 B (J D0 + [E, 0, 0])
// regrouped as  T = -K C Z (K = M^-1 J^T, Z = A^-1 B), P = I + T J,
// Q = P M^-1:  dv+/dq = -dt Q dtau/dq + T E,  dv+/dv = P - dt Q dtau/dv,
// dv+/dtau = dt Q.  One FP64 factorisation of A serves all 3 n columns.
template <class R>
DSIM_HD void jacobian(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, R* dvdq, R* dvdv,
                      R* dvdtau) {
    const int n = E.nv, k = E.k;
    derivative_partials(T, E, P);
    const int m = E.hdr[1];
    R* CZ = E.P;  // k x k, reused before P is formed
    if (m > 0) {
        reduced_solve(T, E);
        for (int idx = T.tid; idx < k * k; idx += T.nt) {
            const int row = idx / k, rho = idx - row * k;
            const int c = row / 3, a = row - 3 * c;
            double s = 0;
            for (int i = 0; i < m; ++i)
                if (E.vctc[i] == c) s += E.vcol[3 * i + a] * E.Z[rho * m + i];
            CZ[idx] = R(s);
        }
        T.sync();
        for (int idx = T.tid; idx < n * k; idx += T.nt) {
            const int i = idx / k, rho = idx - i * k;
            double s = 0;
            for (int c = 0; c < k; ++c) s += double(E.KT[c * n + i]) * double(CZ[c * k + rho]);
            E.T[idx] = R(-s);
        }
    } else {
        for (int idx = T.tid; idx < n * k; idx += T.nt) E.T[idx] = 0;
    }
    T.sync();
    for (int idx = T.tid; idx < n * n; idx += T.nt) {
        const int i = idx / n, j = idx - i * n;
        double s = (i == j) ? 1.0 : 0.0;
        for (int r = 0; r < k; ++r) s += double(E.T[i * k + r]) * double(E.J[r * n + j]);
        E.P[idx] = R(s);
    }
    T.sync();
    // Q = P M^-1 with the FP64 M^-1 of the step
    for (int idx = T.tid; idx < n * n; idx += T.nt) {
        const int i = idx / n, j = idx - i * n;
        double s = 0;
        for (int l = 0; l < n; ++l) s += double(E.P[i * n + l]) * E.Mi[l * n + j];
        E.Q[idx] = R(s);
    }
    T.sync();
    const R dt = R(P.dt);
    const int off = B.jac_off[E.e];
    for (int idx = T.tid; idx < n * n; idx += T.nt) {
        const int i = idx / n, j = idx - i * n;
        // FP64 sums of the working-precision operands: on gfx950 an FP64
        // FMA issues at the rate of an unpacked FP32 one, and the sums of
        // the assembly cancel
        double sq = 0, sv = 0, se = 0;
        for (int l = 0; l < n; ++l) {
            const double ql = double(E.Q[i * n + l]);
            sq += ql * double(E.dTq[l * n + j]);
            sv += ql * double(E.dTv[l * n + j]);
        }
        for (int r = 0; r < k; ++r) se += double(E.T[i * k + r]) * double(E.E[r * n + j]);
        // Baumgarte damping: the normal rows of the contact equation also
        // depend on v through -kd J_N v (Appendix D)
        double sd = 0;
        if (P.gap_mode == 1 && P.kd != 0.0)
            for (int r = 2; r < k; r += 3) sd += double(E.T[i * k + r]) * double(E.J[r * n + j]);
        dvdq[off + idx] = R(-P.dt * sq + se);
        dvdv[off + idx] = R(double(E.P[idx]) - P.dt * sv - P.kd * sd);
        dvdtau[off + idx] = R(P.dt * double(E.Q[idx]));
    }
    T.sync();
}

// --------------------------------------------------------------------------
// position update q+ = q (+) dt v+ (symplectic Euler) and its adjoint
// --------------------------------------------------------------------------

// sin(t)/t, (1 - cos t)/t^2, (t - sin t)/t^3 and sin(t/2)/t for t = |w|,
// by their Taylor series near 0 (truncation below 1e-17 for t < 1e-2).
DSIM_HD inline void exp_coeffs(const double* w, double& a, double& b, double& c, double& h) {
    const double t2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    if (t2 < 1e-4) {
        a = 1.0 - t2 / 6.0 * (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0));
        b = 0.5 - t2 / 24.0 * (1.0 - t2 / 30.0 * (1.0 - t2 / 56.0));
        c = 1.0 / 6.0 - t2 / 120.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0));
        h = 0.5 - t2 / 48.0 * (1.0 - t2 / 80.0 * (1.0 - t2 / 168.0));
        return;
    }
    const double t = sqrt(t2);
    a = sin(t) / t;
    b = (1.0 - cos(t)) / t2;
    c = (t - sin(t)) / (t2 * t);
    h = sin(0.5 * t) / t;
}

// X = Exp(xi) for a body twist xi = (linear rho, angular phi): rotation Rx
// (row-major) and translation tx = V(phi) rho.
DSIM_HD inline void exp_se3(const double* xi, double* Rx, double* tx) {
    const double* rho = xi;
    const double* phi = xi + 3;
    double a, b, c, h;
    exp_coeffs(phi, a, b, c, h);
    const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
    double K2[9];
    mat3mul(K, K, K2);
    double V[9];
    for (int i = 0; i < 9; ++i) {
        const double id = (i % 4 == 0) ? 1.0 : 0.0;
        Rx[i] = id + a * K[i] + b * K2[i];
        V[i] = id + b * K[i] + c * K2[i];
    }
    mat3vec(V, rho, tx);
}

// q+ = q (+) dt v+ for every joint of the environment (v+ = E.vn).  A free
// flyer composes its placement with Exp(dt v+) on the right: p+ = p + R t,
// quat+ = quat * exp(dt omega) (renormalised); a revolute angle adds dt v+.
template <class R>
DSIM_HD void integrate(const Team& T, Env<R>& E, const Params& P, const R* q, R* qn) {
    for (int b = T.tid; b < E.nb; b += T.nt) {
        const int c0 = E.q0 + E.cfg0[b], d0 = E.dof0[b];
        if (E.jtype[b] == 1) {
            double xi[6], Rx[9], tx[3];
            for (int i = 0; i < 6; ++i) xi[i] = P.dt * E.vn[d0 + i];
            exp_se3(xi, Rx, tx);
            double a, bb, c, h;
            exp_coeffs(xi + 3, a, bb, c, h);
            const double* Rw = E.Rw + 9 * b;  // R(quat) from the kinematics
            double dp[3];
            mat3vec(Rw, tx, dp);
            for (int i = 0; i < 3; ++i) qn[c0 + i] = R(double(q[c0 + i]) + dp[i]);
            const double x = q[c0 + 3], y = q[c0 + 4], z = q[c0 + 5], w = q[c0 + 6];
            const double ex = h * xi[3], ey = h * xi[4], ez = h * xi[5];
            const double ew = cos(0.5 * sqrt(xi[3] * xi[3] + xi[4] * xi[4] + xi[5] * xi[5]));
            // quaternion product (x y z w) * (ex ey ez ew)
            double nx = w * ex + ew * x + (y * ez - z * ey);
            double ny = w * ey + ew * y + (z * ex - x * ez);
            double nz = w * ez + ew * z + (x * ey - y * ex);
            double nw = w * ew - (x * ex + y * ey + z * ez);
            const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz + nw * nw);
            qn[c0 + 3] = R(nx * inv);
            qn[c0 + 4] = R(ny * inv);
            qn[c0 + 5] = R(nz * inv);
            qn[c0 + 6] = R(nw * inv);
        } else {
            qn[c0] = R(double(q[c0]) + P.dt * E.vn[d0]);
        }
    }
    T.sync();
}

// Adjoint of the position update at (q, v+) for a tangent adjoint aq of q+:
// with X = Exp(xi), xi = dt v+, a perturbation q (+) d and v+ + dv gives
// q+ (+) (Ad_{X^-1} d + dt Jr(xi) dv) to first order, Jr the right Jacobian
// of the exponential, Jr(xi) = sum_k (-ad_xi)^k / (k+1)!.  Adds
// dt Jr^T aq to gv (the adjoint of v+) and writes Ad_{X^-1}^T aq to gq.
template <class R>
DSIM_HD void integrate_adjoint(const Team& T, Env<R>& E, const Params& P, const R* aq, double* gv, double* gq) {
    for (int b = T.tid; b < E.nb; b += T.nt) {
        const int d0 = E.dof0[b];
        if (E.jtype[b] == 1) {
            double xi[6], a[6], Rx[9], tx[3];
            for (int i = 0; i < 6; ++i) {
                xi[i] = P.dt * E.vn[d0 + i];
                a[i] = double(aq[E.d0 + d0 + i]);
            }
            exp_se3(xi, Rx, tx);
            // Ad_{X^-1}^T a = (Rx a_lin, tx x (Rx a_lin) + Rx a_ang)
            double rl[3], ra[3], txr[3];
            mat3vec(Rx, a, rl);
            mat3vec(Rx, a + 3, ra);
            cross3(tx, rl, txr);
            for (int i = 0; i < 3; ++i) {
                gq[d0 + i] = rl[i];
                gq[d0 + 3 + i] = txr[i] + ra[i];
            }
            // Jr^T a = sum_k M^k a / (k+1)!, M = (-ad_xi)^T:
            // M (x_lin, x_ang) = (phi x x_lin, rho x x_lin + phi x x_ang)
            double term[6], sum[6];
            for (int i = 0; i < 6; ++i) term[i] = sum[i] = a[i];
            double na = 0;
            for (int i = 0; i < 6; ++i) na = fmax(na, fabs(a[i]));
            for (int kk = 1; kk < 60; ++kk) {
                double l[3], r1[3], r2[3];
                cross3(xi + 3, term, l);
                cross3(xi, term, r1);
                cross3(xi + 3, term + 3, r2);
                double tm = 0;
                for (int i = 0; i < 3; ++i) {
                    term[i] = l[i] / (kk + 1);
                    term[3 + i] = (r1[i] + r2[i]) / (kk + 1);
                    tm = fmax(tm, fmax(fabs(term[i]), fabs(term[3 + i])));
                }
                for (int i = 0; i < 6; ++i) sum[i] += term[i];
                if (tm <= 1e-18 * na) break;
            }
            for (int i = 0; i < 6; ++i) gv[d0 + i] += P.dt * sum[i];
        } else {
            const double a = double(aq[E.d0 + d0]);
            gq[d0] = a;
            gv[d0] += P.dt * a;
        }
    }
    T.sync();
}

// Reverse mode: the transpose of the Jacobian above applied to gbar,
//   tg = T^T gbar = -B^T A^-T C^T (K^T gbar),  pg = P^T gbar = gbar + J^T tg,
//   qg = Q^T gbar = M^-1 pg,
//   g_tau = dt qg,  g_v = pg - dt dtau/dv^T qg,  g_q = -dt dtau/dq^T qg + E^T tg.
// The transposed solve is the exact transpose of the basic-solution operator
// of the forward derivative, so both agree for rank-deficient A.
//
// With aqn != nullptr (the adjoint of the fused step and position update),
// gbar is the adjoint of v+ coming from later steps and aqn the tangent
// adjoint of q+: the adjoint of the position update is applied first and its
// q part added to gq.
template <class R>
DSIM_HD void vjp(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, const R* gbar, const R* aqn,
                 const R* glam, R* gq, R* gv, R* gtau) {
    const int n = E.nv, k = E.k, m = E.hdr[1], rank = E.hdr[4];
    derivative_partials(T, E, P);
    double* gb = E.bias;  // gbar (the bias is no longer needed)
    double* pg = E.af;    // P^T gbar, then M^-1 P^T gbar
    double* pk = E.vf;    // P^T gbar kept
    double* tg = E.scr;   // T^T gbar (k)
    for (int i = T.tid; i < n; i += T.nt) gb[i] = double(gbar[E.d0 + i]);
    T.sync();
    if (aqn) integrate_adjoint(T, E, P, aqn, gb, E.gint);
    if (T.tid == 0) {
        double* sp = E.rhs;
        double* z = E.ytmp;
        double* y = E.X;
        for (int i = 0; i < m; ++i) {
            const int c = E.vctc[i];
            double s = 0;
            for (int a = 0; a < 3; ++a) {
                double ka = 0;
                for (int j = 0; j < n; ++j) ka += double(E.KT[(3 * c + a) * n + j]) * gb[j];
                // an adjoint of the impulses enters beside K^T gbar: dLam = C X
                if (glam) ka += double(glam[3 * E.c0 + 3 * c + a]);
                s += E.vcol[3 * i + a] * ka;
            }
            sp[i] = s;
        }
        for (int j = 0; j < rank; ++j) {
            double s = sp[E.cperm[j]];
            for (int i = 0; i < j; ++i) s -= E.A[i * m + j] * z[i];
            z[j] = s / E.A[j * m + j];
        }
        for (int i = rank - 1; i >= 0; --i) {
            double s = z[i];
            for (int j = i + 1; j < rank; ++j) s -= E.A[j * m + i] * z[j];
            z[i] = s;
        }
        for (int i = 0; i < m; ++i) y[E.rperm[i]] = (i < rank) ? z[i] : 0.0;
        for (int r = 0; r < k; ++r) tg[r] = 0;
        for (int i = 0; i < m; ++i) {
            const int c = E.vctc[i];
            for (int a = 0; a < 3; ++a) tg[3 * c + a] -= E.vrow[3 * i + a] * y[i];
        }
    }
    T.sync();
    for (int j = T.tid; j < n; j += T.nt) {
        double s = gb[j];
        for (int r = 0; r < k; ++r) s += double(E.J[r * n + j]) * tg[r];
        pk[j] = s;
    }
    T.sync();
    for (int i = T.tid; i < n; i += T.nt) {
        double s = 0;
        for (int j = 0; j < n; ++j) s += E.Mi[i * n + j] * pk[j];
        pg[i] = s;
    }
    T.sync();
    for (int j = T.tid; j < n; j += T.nt) {
        double sq = 0, sv = 0, se = 0;
        for (int l = 0; l < n; ++l) {
            sq += double(E.dTq[l * n + j]) * pg[l];
            sv += double(E.dTv[l * n + j]) * pg[l];
        }
        for (int r = 0; r < k; ++r) se += double(E.E[r * n + j]) * tg[r];
        double sd = 0;  // Baumgarte damping (Appendix D): -kd J_N^T tg
        if (P.gap_mode == 1 && P.kd != 0.0)
            for (int r = 2; r < k; r += 3) sd += double(E.J[r * n + j]) * tg[r];
        gq[E.d0 + j] = R(-P.dt * sq + se + (aqn ? E.gint[j] : 0.0));
        gv[E.d0 + j] = R(pk[j] - P.dt * sv - P.kd * sd);
        gtau[E.d0 + j] = R(P.dt * pg[j]);
    }
    T.sync();
}

// Generalised force of the physical parameter `col` of body-or-contact
// layout [n_b masses, 6 n_b rotational inertias, n_c friction
// coefficients] (the order of the parameter columns), at fixed (v+, Lam),
// for the ID-side parameters: per body b,
//  * mass m_b (centre of mass and rotational inertia about it fixed):
//    F = I' A_b + V_b x* I' V_b with I' the unit point mass at the centre
//    of mass, A_b and V_b the body's acceleration (gravity included) at a+
//    and velocity at v;
//  * rotational inertia component k (xx yy zz xy xz yz about the centre of
//    mass, body frame): with the world-frame unit change dI = R E_k R^T
//    (E_k = e_i e_i^T, or e_i e_j^T + e_j e_i^T), F = (dI alpha + omega x
//    dI omega, 0).
// The generalised force on dof l is S_l . F for the dofs that move b.
DSIM_HD inline void param_force(const double* Iw, const double* Rw, const double* A, const double* V, int k,
                                double* F) {
    if (k < 0) {
        const double c[3] = {Iw[1] / Iw[0], Iw[2] / Iw[0], Iw[3] / Iw[0]};
        const double Ip[10] = {1.0, c[0], c[1], c[2], c[1] * c[1] + c[2] * c[2], c[0] * c[0] + c[2] * c[2],
                               c[0] * c[0] + c[1] * c[1], -c[0] * c[1], -c[0] * c[2], -c[1] * c[2]};
        double iv[6], vxiv[6];
        iapply(Ip, A, F);
        iapply(Ip, V, iv);
        mxf(V, iv, vxiv);
        for (int a = 0; a < 6; ++a) F[a] += vxiv[a];
        return;
    }
    // component k: (i, j) = (0,0) (1,1) (2,2) (0,1) (0,2) (1,2)
    const int i = k < 3 ? k : (k == 5 ? 1 : 0);
    const int j = k < 3 ? k : (k == 3 ? 1 : 2);
    // body-frame angular acceleration and velocity: R^T alpha, R^T omega
    double a[3], w[3];
    for (int r = 0; r < 3; ++r) {
        a[r] = Rw[r] * A[0] + Rw[3 + r] * A[1] + Rw[6 + r] * A[2];
        w[r] = Rw[r] * V[0] + Rw[3 + r] * V[1] + Rw[6 + r] * V[2];
    }
    // E_k x in the body frame
    double ea[3] = {0, 0, 0}, ew[3] = {0, 0, 0};
    ea[i] += a[j];
    ew[i] += w[j];
    if (i != j) {
        ea[j] += a[i];
        ew[j] += w[i];
    }
    double wxe[3];
    cross3(w, ew, wxe);
    const double t[3] = {ea[0] + wxe[0], ea[1] + wxe[1], ea[2] + wxe[2]};
    for (int r = 0; r < 3; ++r) {
        F[r] = Rw[3 * r] * t[0] + Rw[3 * r + 1] * t[1] + Rw[3 * r + 2] * t[2];
        F[3 + r] = 0;
    }
}

// Slip direction of a sliding contact at the solution (sigma_T / |sigma_T|,
// or opposite the friction impulse before any slip).
template <class R>
DSIM_HD inline void slip_dir(const Env<R>& E, int c, double& u0, double& u1) {
    const double s0 = E.dsig[3 * c], s1 = E.dsig[3 * c + 1];
    const double ns = sqrt(s0 * s0 + s1 * s1);
    u0 = 1.0;
    u1 = 0.0;
    if (ns > 0) {
        u0 = s0 / ns;
        u1 = s1 / ns;
    } else {
        const double l0 = E.Ld[3 * c], l1 = E.Ld[3 * c + 1];
        const double nl = sqrt(l0 * l0 + l1 * l1);
        if (nl > 0) {
            u0 = -l0 / nl;
            u1 = -l1 / nl;
        }
    }
}

// Gradients of gbar . v+ in the physical parameters, after `vjp` (which
// leaves pg = M^-1 P^T gbar, so that gbar^T dv+/dtau = dt pg^T).
//
// The step's residual depends on a parameter at fixed (v+, Lam) through
// inverse dynamics or through the sliding cone, never through both, so
// each gradient is a generalised force paired with dt pg:
//  * masses and rotational inertias: the forces of `param_force`, paired
//    with -dt pg over the dofs that move the body, i.e. -dt V_b(pg) . F
//    with V_b(x) the body velocity for joint velocities x;
//  * friction coefficient mu_c of a sliding contact: the tangential rows
//    Lam_T + mu Lam_N u = 0 change like a tangential impulse -Lam_N u dmu
//    applied outside the mode equations, i.e. a generalised force
//    -J_c^T (Lam_N u, 0) / dt; the gradient is -Lam_N u . (J_c pg)_T.  It
//    is zero for breaking and sticking contacts.
// Output per environment at 7 b0 + c0: [n_b masses, 6 n_b inertias (xx yy
// zz xy xz yz per body), n_c friction coefficients].
template <class R>
DSIM_HD void param_grads(const Team& T, Env<R>& E, const Params& P, R* gp) {
    const int n = E.nv, nb = E.nb;
    const double* pg = E.af;
    R* out = gp + 7 * size_t(E.b0) + E.c0;
    for (int idx = T.tid; idx < 7 * nb; idx += T.nt) {
        const int b = idx < nb ? idx : (idx - nb) / 6;
        const int k = idx < nb ? -1 : (idx - nb) % 6;
        double F[6];
        param_force(E.Iw + 10 * b, E.Rw + 9 * b, E.Acc + 6 * b, E.V + 6 * b, k, F);
        double w[6] = {0, 0, 0, 0, 0, 0};
        const uint64_t mask = E.bmask[b];
        for (int j = 0; j < n; ++j)
            if ((mask >> j) & 1ull)
                for (int a = 0; a < 6; ++a) w[a] += E.S[6 * j + a] * pg[j];
        out[idx] = R(-P.dt * dot6(w, F));
    }
    for (int c = T.tid; c < E.nc; c += T.nt) {
        double g = 0;
        if (E.cmode[c] == SLD) {
            double u0, u1;
            slip_dir(E, c, u0, u1);
            double j0 = 0, j1 = 0;
            for (int j = 0; j < n; ++j) {
                j0 += double(E.J[(3 * c) * n + j]) * pg[j];
                j1 += double(E.J[(3 * c + 1) * n + j]) * pg[j];
            }
            g = -E.Ld[3 * c + 2] * (u0 * j0 + u1 * j1);
        }
        out[7 * nb + c] = R(g);
    }
    T.sync();
}

// Forward-mode columns of the physical parameters, after `jacobian` (Q =
// P M^-1 is still formed): with the generalised forces of `param_grads`,
//   d v+ / d (m_b or I_b,k) = -dt Q S^T F      (dofs that move b)
//   d v+ / d mu_c           = -Q J_c^T (Lam_N u, 0)   (sliding contacts)
// written row-major n x (7 n_b + n_c) at pjac_off[e], columns in the order
// of `param_grads`.  Each thread forms the force of its column on the fly.
template <class R>
DSIM_HD void param_columns(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, R* dvdp) {
    const int n = E.nv, nb = E.nb, nc = E.nc, np = 7 * nb + nc;
    const int off = B.pjac_off[E.e];
    for (int idx = T.tid; idx < n * np; idx += T.nt) {
        const int i = idx / np, col = idx - i * np;
        double s = 0;
        if (col < 7 * nb) {
            const int b = col < nb ? col : (col - nb) / 6;
            const int k = col < nb ? -1 : (col - nb) % 6;
            double F[6];
            param_force(E.Iw + 10 * b, E.Rw + 9 * b, E.Acc + 6 * b, E.V + 6 * b, k, F);
            const uint64_t mask = E.bmask[b];
            for (int l = 0; l < n; ++l)
                if ((mask >> l) & 1ull) s += double(E.Q[i * n + l]) * dot6(E.S + 6 * l, F);
            s *= -P.dt;
        } else {
            const int cc = col - 7 * nb;
            if (E.cmode[cc] == SLD) {
                double u0, u1;
                slip_dir(E, cc, u0, u1);
                for (int l = 0; l < n; ++l)
                    s += double(E.Q[i * n + l]) *
                         (u0 * double(E.J[(3 * cc) * n + l]) + u1 * double(E.J[(3 * cc + 1) * n + l]));
                s *= -E.Ld[3 * cc + 2];
            }
        }
        dvdp[off + idx] = R(s);
    }
    T.sync();
}

// The step's FP64 impulses and the work its contact solve executed, into
// the environment's slot of `ld`.
template <class R>
DSIM_HD void write_work(const Team& T, const Env<R>& E, const Params& P, double* ld) {
    double* l = ld + size_t(E.e) * kLdStride;
    for (int r = T.tid; r < E.k; r += T.nt) l[r] = E.Ld[r];
    if (T.tid == 0) {
        // executed solver work: the first pass writes its sweeps and
        // clears the fallback's counts, the fallback pass (run only
        // for the environments the first left unsolved) writes its own
        if (P.pass == 0) {
            l[kLdWork] = double(E.hdr[7]);
            l[kLdFallback] = (E.hdr[5] & (ST_NCP | ST_POLISH)) ? 1.0 : 0.0;
        }
        l[kLdWork + 1] = double(E.hdr[8]);
        l[kLdWork + 2] = double(E.hdr[3]);
        l[kLdWork + 3] = double(E.hdr[15]);
    }
}

// Full pipeline of one environment.
//
// The step entries (STEP, SINT) solve the step and write its outputs, and
// the FP64 impulses to `ld` when given.  The derivative entries (JAC, VJP,
// RVJP) run after a step launch over the same environments: they restore
// the step from `ld` and the written modes, then differentiate it.  The
// first step pass of a derivative entry is the ASM launch (the step up to
// its contact system, into the record) followed by the NCP launch (the rest
// of the step from the record), and its fallback pass the FBK launch (from
// the same record): the same arithmetic as the step launches.
template <class R>
DSIM_HD void run_env(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, const Dims& D, int entry,
                     int e, const R* q, const R* v, const R* tau, const R* gbar, const R* gbar2, R* v_next, R* lam,
                     int8_t* mode, int32_t* status, R* o1, R* o2, R* o3, R* o4, R* o5, double* ld) {
    // hand-over record of this environment (derivative entries only)
    const Handover H = handover_layout<R>(D);
    char* rec = ld ? handover_base(ld, B.n_env) + size_t(e) * H.bytes : nullptr;
    if (entry == ENTRY_NCP || entry == ENTRY_FBK) {
        // no tree quantities in this launch's layout: sizes, friction
        // coefficients and the contact system only
        load_contact_system(T, E, B, e, H, rec);
        step_finish(T, E, P, &H, rec, static_cast<const R*>(lam));
        write_step(T, E, v_next, lam, mode, status);
        write_work(T, E, P, ld);
        T.sync();
        return;
    }
    load_env(T, E, B, e, q, v, tau);
    if (entry == ENTRY_ASM) {
        step_assemble(T, E, B, P, q, &H, rec);
        put_contact_system(T, E, H, rec);
    } else if (!entry_has_derivative(entry)) {
        step_forward(T, E, B, P, q, rec ? &H : nullptr, rec, static_cast<const R*>(lam));
        write_step(T, E, v_next, lam, mode, status);
        if (ld) write_work(T, E, P, ld);
        if (entry == ENTRY_SINT) integrate(T, E, P, q, o1);
    } else {
        load_step(T, E, H, rec, ld, mode);
        if (entry == ENTRY_JAC) jacobian(T, E, B, P, o1, o2, o3);
        if (entry == ENTRY_PJAC) {
            jacobian(T, E, B, P, o1, o2, o3);
            param_columns(T, E, B, P, o4);
        }
        // the VJP entries take the impulse adjoint in gbar2; the rollout
        // adjoint takes the position adjoint there
        if (entry == ENTRY_VJP) vjp(T, E, B, P, gbar, static_cast<const R*>(nullptr), gbar2, o1, o2, o3);
        if (entry == ENTRY_RVJP) vjp(T, E, B, P, gbar, gbar2, static_cast<const R*>(nullptr), o1, o2, o3);
        if (entry == ENTRY_PVJP) {
            vjp(T, E, B, P, gbar, static_cast<const R*>(nullptr), gbar2, o1, o2, o3);
            param_grads(T, E, P, o4);
        }
        // a NaN or Inf in the derivative outputs sets the status bit that
        // the step sets for its own outputs
        const int n = E.nv, np = 7 * E.nb + E.nc;
        bool bad = false;
        auto scan = [&](const R* p, size_t off, int cnt) {
            if (!p) return;
            for (int i = T.tid; i < cnt; i += T.nt) {
                const double x = double(p[off + i]);
                if (!(x == x) || fabs(x) > 1e300) bad = true;
            }
        };
        if (entry == ENTRY_JAC || entry == ENTRY_PJAC) {
            const size_t off = size_t(B.jac_off[e]);
            scan(o1, off, n * n);
            scan(o2, off, n * n);
            scan(o3, off, n * n);
            if (entry == ENTRY_PJAC) scan(o4, size_t(B.pjac_off[e]), n * np);
        } else {
            scan(o1, size_t(E.d0), n);
            scan(o2, size_t(E.d0), n);
            scan(o3, size_t(E.d0), n);
            if (entry == ENTRY_PVJP) scan(o4, 7 * size_t(E.b0) + E.c0, np);
        }
        if (T.tid == 0) E.hdr[11] = 0;
        T.sync();
        if (bad) E.hdr[11] = 1;
        T.sync();
        if (T.tid == 0 && E.hdr[11]) status[e] |= ST_NONFINITE;
    }
    T.sync();
}

}  // namespace dsim
