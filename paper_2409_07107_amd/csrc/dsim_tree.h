// dsim_tree.h -- FP64 recursions over the kinematic tree (Section II.C):
// kinematics, composite inertias, the mass matrix, inverse dynamics, the
// tree-sparse factorisation of M, the contact Jacobian and the Delassus
// operator (eq. 5).
#pragma once

#include "dsim_core.h"

namespace dsim {

// Model tables of environment e: parents, coordinates, dof chains, levels.
template <class R>
DSIM_HD void load_env(const Team& T, Env<R>& E, const BatchView<R>& B, int e, const R* q, const R* v,
                      const R* tau) {
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
    // the model tables are read by the team at once; the serial pass below
    // then works from LDS
    for (int b = T.tid; b < E.nb; b += T.nt) {
        E.parent[b] = B.parent[E.b0 + b];
        E.jtype[b] = B.jtype[E.b0 + b];
    }
    T.sync();
    if (T.tid == 0) {
        const int nb = E.nb;
        int dof = 0, cfg = 0;
        int depth[64];
        for (int b = 0; b < nb; ++b) {
            const int par = E.parent[b];
            const int jt = E.jtype[b];
            E.dof0[b] = dof;
            E.cfg0[b] = cfg;
            const int nd = (jt == 1) ? 6 : 1;
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
        const int nlev = nb ? maxd + 1 : 0;
        int pos = 0;
        for (int L = 0; L < nlev; ++L) {
            E.lstart[L] = pos;
            for (int b = 0; b < nb; ++b)
                if (depth[b] == L) E.lorder[pos++] = b;
        }
        E.lstart[nlev] = pos;
        for (int i = 0; i < 16; ++i) E.hdr[i] = 0;
        E.hdr[0] = nlev;
        // reference point: the world position of body 0
        const R* o = (nb > 0 && E.jtype[0] == 1) ? q + E.q0 : B.jpos + 3 * E.b0;
        for (int i = 0; i < 3; ++i) E.org[i] = nb > 0 ? double(o[i]) : 0.0;
    }
    for (int i = T.tid; i < E.nv; i += T.nt) {
        E.v[i] = double(v[E.d0 + i]);
        E.tau[i] = double(tau[E.d0 + i]);
    }
    for (int c = T.tid; c < E.nc; c += T.nt) {
        E.cbody[c] = B.cbody[E.c0 + c];
        E.mu[c] = B.mu[E.c0 + c];
        E.crad[c] = B.cradius ? double(B.cradius[E.c0 + c]) : 0.0;
    }
    T.sync();
}

// Placement, motion subspace (world-aligned, about org) of body b, parent done.
template <class R>
DSIM_HD void fk_body(Env<R>& E, const BatchView<R>& B, const R* q, int b) {
    const int gb = E.b0 + b;
    const int par = E.parent[b];
    double* Rw = E.Rw + 9 * b;
    double* pw = E.pw + 3 * b;
    const R* qq = q + E.q0 + E.cfg0[b];
    if (E.jtype[b] == 1) {
        const double x = qq[3], y = qq[4], z = qq[5], w = qq[6];
        Rw[0] = 1 - 2 * (y * y + z * z); Rw[1] = 2 * (x * y - z * w);     Rw[2] = 2 * (x * z + y * w);
        Rw[3] = 2 * (x * y + z * w);     Rw[4] = 1 - 2 * (x * x + z * z); Rw[5] = 2 * (y * z - x * w);
        Rw[6] = 2 * (x * z - y * w);     Rw[7] = 2 * (y * z + x * w);     Rw[8] = 1 - 2 * (x * x + y * y);
        for (int i = 0; i < 3; ++i) pw[i] = double(qq[i]) - E.org[i];
        const int d = E.dof0[b];
        for (int c = 0; c < 3; ++c) {
            double* Sl = E.S + 6 * (d + c);      // linear body-frame axis c
            double* Sa = E.S + 6 * (d + 3 + c);  // angular body-frame axis c
            const double ax[3] = {Rw[c], Rw[3 + c], Rw[6 + c]};
            double pxa[3];
            cross3(pw, ax, pxa);
            for (int i = 0; i < 3; ++i) {
                Sl[i] = 0;
                Sl[3 + i] = ax[i];
                Sa[i] = ax[i];
                Sa[3 + i] = pxa[i];
            }
        }
    } else {
        double a[3], jr[9], jp[3];
        for (int i = 0; i < 3; ++i) a[i] = double(B.axis[3 * gb + i]);
        for (int i = 0; i < 9; ++i) jr[i] = double(B.jrot[9 * gb + i]);
        for (int i = 0; i < 3; ++i) jp[i] = double(B.jpos[3 * gb + i]);
        const double th = double(qq[0]);
        const double s = sin(th), c = cos(th), omc = 1 - c;
        // Rodrigues rotation about the unit axis a
        const double Rot[9] = {c + omc * a[0] * a[0],        omc * a[0] * a[1] - s * a[2], omc * a[0] * a[2] + s * a[1],
                               omc * a[1] * a[0] + s * a[2], c + omc * a[1] * a[1],        omc * a[1] * a[2] - s * a[0],
                               omc * a[2] * a[0] - s * a[1], omc * a[2] * a[1] + s * a[0], c + omc * a[2] * a[2]};
        double Rj[9];
        mat3mul(jr, Rot, Rj);
        if (par < 0) {
            for (int i = 0; i < 9; ++i) Rw[i] = Rj[i];
            for (int i = 0; i < 3; ++i) pw[i] = jp[i] - E.org[i];
        } else {
            mat3mul(E.Rw + 9 * par, Rj, Rw);
            double t[3];
            mat3vec(E.Rw + 9 * par, jp, t);
            for (int i = 0; i < 3; ++i) pw[i] = E.pw[3 * par + i] + t[i];
        }
        double ax[3], pxa[3];
        mat3vec(Rw, a, ax);  // the axis is invariant under the joint rotation
        cross3(pw, ax, pxa);
        double* Sd = E.S + 6 * E.dof0[b];
        for (int i = 0; i < 3; ++i) {
            Sd[i] = ax[i];
            Sd[3 + i] = pxa[i];
        }
    }
}

// V_b = V_parent + sum_d S_d x_d for a joint-velocity vector x.
template <class R>
DSIM_HD void body_velocity(Env<R>& E, const double* x, double* Vout, int b) {
    const int par = E.parent[b];
    double* Vb = Vout + 6 * b;
    for (int i = 0; i < 6; ++i) Vb[i] = (par >= 0) ? Vout[6 * par + i] : 0.0;
    for (int j = 0; j < E.ndof[b]; ++j) {
        const int d = E.dof0[b] + j;
        const double* Sd = E.S + 6 * d;
        for (int i = 0; i < 6; ++i) Vb[i] += Sd[i] * x[d];
    }
}

// Placements, motion subspaces and velocities level by level; spatial
// inertias about org; contact points; composite inertias.
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
    for (int b = T.tid; b < E.nb; b += T.nt) {
        const int gb = E.b0 + b;
        const double* Rw = E.Rw + 9 * b;
        const double m = double(B.mass[gb]);
        double cl[3], c[3];
        for (int i = 0; i < 3; ++i) cl[i] = double(B.com[3 * gb + i]);
        mat3vec(Rw, cl, c);
        for (int i = 0; i < 3; ++i) c[i] += E.pw[3 * b + i];
        double in[6];
        for (int i = 0; i < 6; ++i) in[i] = double(B.inertia[6 * gb + i]);
        const double Ib[9] = {in[0], in[3], in[4], in[3], in[1], in[5], in[4], in[5], in[2]};
        double t[9], Iw[9];
        mat3mul(Rw, Ib, t);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                Iw[3 * i + j] = t[3 * i] * Rw[3 * j] + t[3 * i + 1] * Rw[3 * j + 1] + t[3 * i + 2] * Rw[3 * j + 2];
        const double cc = dot3(c, c);
        double* I = E.Iw + 10 * b;
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
        double xl[3], x[3];
        for (int i = 0; i < 3; ++i) xl[i] = double(B.cpoint[3 * (E.c0 + c) + i]);
        mat3vec(E.Rw + 9 * b, xl, x);
        for (int i = 0; i < 3; ++i) E.xw[3 * c + i] = x[i] + E.pw[3 * b + i];
        // a sphere touches the plane z = 0 at its lowest point
        E.xw[3 * c + 2] -= E.crad[c];
    }
    T.sync();
    // composite inertias (children are listed after their parents)
    for (int i = T.tid; i < 10; i += T.nt)
        for (int b = E.nb - 1; b > 0; --b) {
            const int par = E.parent[b];
            if (par >= 0) E.Ic[10 * par + i] += E.Ic[10 * b + i];
        }
    T.sync();
}

// Composite-rigid-body mass matrix: M[j][k] = S_j . (Ic_{body(k)} S_k) for j
// on the dof ancestor chain of k, written to the lower triangle of Mx.
template <class R>
DSIM_HD void mass_matrix(const Team& T, Env<R>& E) {
    const int n = E.nv;
    for (int i = T.tid; i < n * n; i += T.nt) E.Mx[i] = 0;
    T.sync();
    for (int k = T.tid; k < n; k += T.nt) {
        double F[6];
        iapply(E.Ic + 10 * E.dbody[k], E.S + 6 * k, F);
        for (int j = k; j >= 0; j = E.dpar[j]) E.Mx[k * n + j] = dot6(E.S + 6 * j, F);
    }
    T.sync();
}

// Recursive Newton-Euler in world-aligned coordinates about org.  acc:
// per-dof accelerations (nullptr = 0); contact forces Lam * fscale applied
// at the contact points (fscale = 0: none).  Leaves body accelerations in
// Acc, composite forces in Fc, the generalised forces in out (if given).
template <class R>
DSIM_HD void rnea(const Team& T, Env<R>& E, const Params& P, const double* acc, double fscale, double* out) {
    const int nlev = E.hdr[0];
    for (int L = 0; L < nlev; ++L) {
        const int s = E.lstart[L], n = E.lstart[L + 1] - s;
        for (int i = T.tid; i < n; i += T.nt) {
            const int b = E.lorder[s + i];
            const int par = E.parent[b];
            double* Ab = E.Acc + 6 * b;
            const double* Vb = E.V + 6 * b;
            if (par >= 0) {
                for (int c = 0; c < 6; ++c) Ab[c] = E.Acc[6 * par + c];
            } else {
                // gravity as an upward acceleration of the world
                Ab[0] = 0; Ab[1] = 0; Ab[2] = 0;
                Ab[3] = -P.gx; Ab[4] = -P.gy; Ab[5] = -P.gz;
            }
            double Vrel[6], vp[6];
            for (int c = 0; c < 6; ++c) Vrel[c] = Vb[c] - (par >= 0 ? E.V[6 * par + c] : 0.0);
            mxm(Vb, Vrel, vp);
            for (int c = 0; c < 6; ++c) Ab[c] += vp[c];
            if (acc) {
                for (int j = 0; j < E.ndof[b]; ++j) {
                    const int d = E.dof0[b] + j;
                    for (int c = 0; c < 6; ++c) Ab[c] += E.S[6 * d + c] * acc[d];
                }
            }
            double IA[6], IV[6], VxIV[6];
            const double* I = E.Iw + 10 * b;
            iapply(I, Ab, IA);
            iapply(I, Vb, IV);
            mxf(Vb, IV, VxIV);
            double* F = E.Fc + 6 * b;
            for (int c = 0; c < 6; ++c) F[c] = IA[c] + VxIV[c];
        }
        T.sync();
    }
    if (fscale != 0.0) {
        if (T.tid == 0) {
            for (int c = 0; c < E.nc; ++c) {
                const int b = E.cbody[c];
                const double f[3] = {E.Ld[3 * c] * fscale, E.Ld[3 * c + 1] * fscale, E.Ld[3 * c + 2] * fscale};
                double xf[3];
                cross3(E.xw + 3 * c, f, xf);
                double* F = E.Fc + 6 * b;
                for (int i = 0; i < 3; ++i) {
                    F[i] -= xf[i];
                    F[3 + i] -= f[i];
                }
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
// L, diagonal D.  Eliminating from the leaves up creates no fill outside the
// chains.
template <class R>
DSIM_HD void ltdl(const Team& T, Env<R>& E) {
    const int n = E.nv;
    double* M = E.Mx;
    double* tmp = E.ap;  // scratch row
    for (int k = n - 1; k >= 0; --k) {
        for (int i = T.tid; i < k; i += T.nt) tmp[i] = M[k * n + i];
        T.sync();
        const double dk = M[k * n + k];
        for (int i = T.tid; i < k; i += T.nt) {
            // dofs below k on its ancestor chain: those that move body(k)
            if (!((E.bmask[E.dbody[k]] >> i) & 1ull)) continue;
            const double a = tmp[i] / dk;
            M[k * n + i] = a;
            for (int j = i; j >= 0; j = E.dpar[j]) M[i * n + j] -= a * tmp[j];
        }
        T.sync();
    }
}

// Solve M x = b in place with the factors (one thread per right-hand side).
template <class R>
DSIM_HD inline void ltdl_solve(const Env<R>& E, double* x, int stride) {
    const int n = E.nv;
    const double* M = E.Mx;
    for (int i = n - 1; i >= 0; --i) {
        const double xi = x[i * stride];
        for (int j = E.dpar[i]; j >= 0; j = E.dpar[j]) x[j * stride] -= M[i * n + j] * xi;
    }
    for (int i = 0; i < n; ++i) x[i * stride] /= M[i * n + i];
    for (int i = 0; i < n; ++i) {
        double s = x[i * stride];
        for (int j = E.dpar[i]; j >= 0; j = E.dpar[j]) s -= M[i * n + j] * x[j * stride];
        x[i * stride] = s;
    }
}

// M^-1 (FP64, n x n) from the factors, all columns at once: X = I, then the
// L^T pass (for i from the leaves: X[j][:] -= L[i][j] X[i][:] over the chain
// of i, parallel over the chain and the columns), the D pass, and the L pass
// (for i from the root: X[i][:] -= sum_j L[i][j] X[j][:], parallel over the
// columns).  n team barriers per pass instead of serial per-column solves.
template <class R>
DSIM_HD void tree_inverse(const Team& T, Env<R>& E) {
    const int n = E.nv;
    const double* M = E.Mx;
    double* X = E.Mi;
    for (int idx = T.tid; idx < n * n; idx += T.nt) X[idx] = ((idx / n) == (idx % n)) ? 1.0 : 0.0;
    T.sync();
    for (int i = n - 1; i >= 0; --i) {
        // chain of i: j < i with bit j in bmask(body(i)); items (j, column c)
        const uint64_t chain = E.bmask[E.dbody[i]] & ((i > 0) ? ((1ull << i) - 1ull) : 0ull);
        if (chain) {
            for (int idx = T.tid; idx < i * n; idx += T.nt) {
                const int j = idx / n, c = idx - j * n;
                if ((chain >> j) & 1ull) X[j * n + c] -= M[i * n + j] * X[i * n + c];
            }
            T.sync();
        }
    }
    for (int idx = T.tid; idx < n * n; idx += T.nt) X[idx] /= M[(idx / n) * n + (idx / n)];
    T.sync();
    for (int i = 0; i < n; ++i) {
        const int pj = E.dpar[i];
        if (pj < 0) continue;
        for (int c = T.tid; c < n; c += T.nt) {
            double s = X[i * n + c];
            for (int j = pj; j >= 0; j = E.dpar[j]) s -= M[i * n + j] * X[j * n + c];
            X[i * n + c] = s;
        }
        T.sync();
    }
}

// Contact Jacobian (Appendix C, eq. contact_jaco with a static ground and a
// world-aligned frame): row (c, r) = world velocity component r of the
// body-fixed contact point c per unit joint velocity.
template <class R>
DSIM_HD void contact_jacobian(const Team& T, Env<R>& E) {
    const int n = E.nv, k = E.k;
    for (int idx = T.tid; idx < k * n; idx += T.nt) {
        const int row = idx / n, d = idx - row * n;
        const int c = row / 3, r = row - 3 * c;
        const int b = E.cbody[c];
        double val = 0;
        if ((E.bmask[b] >> d) & 1ull) {
            const double* Sd = E.S + 6 * d;
            double wx[3];
            cross3(Sd, E.xw + 3 * c, wx);
            val = Sd[3 + r] + wx[r];
        }
        E.J[idx] = R(val);
    }
    T.sync();
}

// K^T = J M^-1 (k x n; FP64 solves, stored in working precision),
// G = J M^-1 J^T accumulated in FP64 (kept as Gd; the sweeps round it to
// working precision as they read it), g = J v_f (+ phi/dt on normal rows in gap mode 1), and the
// inverses of the 3x3 diagonal blocks of G for the local solves.
template <class R>
DSIM_HD void delassus(const Team& T, Env<R>& E, const Params& P) {
    const int n = E.nv, k = E.k;
    double* Kd = E.scr;  // k x n in FP64: J M^-1
    for (int idx = T.tid; idx < k * n; idx += T.nt) {
        const int r = idx / n, i = idx - r * n;
        const R* Jr = E.J + r * n;
        double s = 0;
        for (int l = 0; l < n; ++l) s += double(Jr[l]) * E.Mi[l * n + i];
        Kd[idx] = s;
    }
    T.sync();
    // (the FP64 step layout keeps K^T in the product's own storage)
    if (static_cast<void*>(E.KT) != static_cast<void*>(Kd))
        for (int idx = T.tid; idx < k * n; idx += T.nt) E.KT[idx] = R(Kd[idx]);
    for (int idx = T.tid; idx < k * k; idx += T.nt) {
        const int a = idx / k, c = idx - a * k;
        if (c > a) continue;
        double s = 0;
        const double* x = Kd + a * n;
        const R* y = E.J + c * n;
        for (int i = 0; i < n; ++i) s += x[i] * double(y[i]);
        E.Gd[a * k + c] = s;
        E.Gd[c * k + a] = s;
    }
    for (int r = T.tid; r < k; r += T.nt) {
        double s = 0;
        const R* x = E.J + r * n;
        for (int i = 0; i < n; ++i) s += double(x[i]) * E.vf[i];
        if (P.gap_mode == 1 && (r % 3) == 2) {
            // Baumgarte form (Appendix D): phi/dt - kp [phi/dt]_- - kd (J v)_N
            const double z = (E.xw[r] + E.org[2]) / P.dt;
            double jv = 0;
            for (int i = 0; i < n; ++i) jv += double(x[i]) * E.v[i];
            s += z - P.kp * (z < 0 ? z : 0.0) - P.kd * jv;
        }
        E.gd[r] = s;
        E.g[r] = R(s);
    }
    T.sync();
    for (int c = T.tid; c < E.nc; c += T.nt) {
        // pseudo-inverse of the contact's 3x3 block (symmetric positive
        // semidefinite) by Jacobi rotations in FP64; eigenvalues below a
        // relative threshold count as zero.  A contact point that cannot move
        // in some direction has a singular block, and the Gauss-Seidel
        // sticking impulse is then the minimum-norm one: an inverse of the
        // rounded block would turn rounding noise along that direction into
        // an unbounded impulse.
        double a[9], V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                a[3 * i + j] = 0.5 * (E.Gd[(3 * c + i) * k + 3 * c + j] + E.Gd[(3 * c + j) * k + 3 * c + i]);
        for (int sweep = 0; sweep < 8; ++sweep) {
            const double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
            const double dia = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
            if (!(off > 1e-32 * dia)) break;
            for (int pq = 0; pq < 3; ++pq) {
                const int pp = pq == 2 ? 1 : 0, qq = pq == 0 ? 1 : 2;
                const double apq = a[3 * pp + qq];
                if (apq == 0.0) continue;
                // rotation annihilating a_pq (symmetric Schur decomposition)
                const double th = (a[3 * qq + qq] - a[3 * pp + pp]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < 3; ++r) {  // a <- a G (columns p, q)
                    const double x = a[3 * r + pp], y = a[3 * r + qq];
                    a[3 * r + pp] = cs * x - sn * y;
                    a[3 * r + qq] = sn * x + cs * y;
                }
                for (int r = 0; r < 3; ++r) {  // a <- G^T a (rows p, q)
                    const double x = a[3 * pp + r], y = a[3 * qq + r];
                    a[3 * pp + r] = cs * x - sn * y;
                    a[3 * qq + r] = sn * x + cs * y;
                }
                for (int r = 0; r < 3; ++r) {  // V <- V G
                    const double x = V[3 * r + pp], y = V[3 * r + qq];
                    V[3 * r + pp] = cs * x - sn * y;
                    V[3 * r + qq] = sn * x + cs * y;
                }
            }
        }
        const double lmax = fmax(a[0], fmax(a[4], a[8]));
        const double cut = lmax * (sizeof(R) == 4 ? 1e-6 : 1e-12);
        double wi[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int e = 0; e < 3; ++e) {
            const double l = a[4 * e];
            if (!(l > cut)) continue;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) wi[3 * i + j] += V[3 * i + e] * V[3 * j + e] / l;
        }
        R* Wi = E.Winv + 9 * c;
        for (int i = 0; i < 9; ++i) Wi[i] = R(wi[i]);
    }
    T.sync();
}

}  // namespace dsim
