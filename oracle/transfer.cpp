/*
 * Covariant polarized transfer along a stored geodesic.
 * Test infrastructure only (CPU oracle).
 *
 * Sec. 2.1: after the geodesic is saved, the covariant fully polarized
 * transfer equations are integrated along it toward the observer; the
 * polarization is carried as a complex coherency matrix in the coordinate
 * frame, and plasma and coefficients are evaluated at every step.  Readings
 * (the scheme itself is in a paper not reproduced here):
 *  - N^{mu nu} is a Hermitian complex 4x4 matrix, zero at the far end;
 *  - Strang splitting: at each stored point n (from the far end to the
 *    camera) a radiative update over w_n = (D_n + D_{n+1})/2, where D_n is
 *    |dlam| of the step that reached point n (D_0 = D_{end+1} = 0); between
 *    points, parallel transport dN/dlam = -(A N + N A^T), A^mu_b =
 *    Gamma^mu_{ab} K^a, by Heun's method over D_n;
 *  - radiative update: project N on the fluid tetrad legs e1, e2
 *    (I = N11 + N22, Q = N11 - N22, U = 2 Re N12, V = -2 Im N12), apply the
 *    exact constant-coefficient solution of dS/dlam = J - K S over w_n,
 *    rebuild N from S on the same legs; where every coefficient is zero (no
 *    plasma) the update is the identity on S and N is left as it is (the
 *    rebuild would only drop components along K, which no later projection
 *    sees);
 *  - fluid tetrad: e0 = u, e3 = unit vector along K + (K.u) u (equal to
 *    (K + (K.u) u)/(-K.u) for null K), e2 along the part of b
 *    orthogonal to u and e3 (fallback d_theta, then d_r), e1 completing a
 *    right-handed tetrad (det[e0, e1, e2, e3] > 0 in Kerr-Schild components);
 *  - invariant coefficients: J = (L/nu_obs) j/nu^2, A = (L/nu_obs) nu alpha,
 *    R = (L/nu_obs) nu rho, nu = nu_obs (-K.u), L = G M/c^2;
 *  - camera output: N projected on the pixel's screen legs, times nu_obs^3.
 */
#include <cmath>
#include <limits>
#include <cstring>
#include "oracle_internal.h"

namespace orc {

/* ---- constant-coefficient update ---- */

/* Propagation matrix rows (A_I, A_Q, A_U, A_V), (A_Q, A_I, R_V, -R_U),
 * (A_U, -R_V, A_I, R_Q), (A_V, R_U, -R_Q, A_I), U terms zero.  The update
 * S(w) = e^{-K w} S + (int_0^w e^{-K s} ds) J is read off the exponential of
 * the augmented 5x5 matrix [[-K w, J w], [0, 0]] (Van Loan 1978). */
void mueller_step(const double coef[8], const double S_in[4], double w, double S_out[4]) {
    double JI = coef[0], JQ = coef[1], JV = coef[2];
    double AI = coef[3], AQ = coef[4], AV = coef[5];
    double RQ = coef[6], RV = coef[7];
    double AU = 0.0, RU = 0.0, JU = 0.0;
    double K[4][4] = {{AI, AQ, AU, AV}, {AQ, AI, RV, -RU}, {AU, -RV, AI, RQ}, {AV, RU, -RQ, AI}};
    double J[4] = {JI, JQ, JU, JV};
    double M[25], E[25];
    std::memset(M, 0, sizeof(M));
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) M[i * 5 + j] = -K[i][j] * w;
        M[i * 5 + 4] = J[i] * w;
    }
    expm(5, M, E);
    for (int i = 0; i < 4; ++i) {
        double s = E[i * 5 + 4];
        for (int j = 0; j < 4; ++j) s += E[i * 5 + j] * S_in[j];
        S_out[i] = s;
    }
}

/* ---- tetrads ---- */

static double det4(const double M[4][4]) {
    double A[4][4];
    std::memcpy(A, M, sizeof(A));
    double det = 1.0;
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int i = col + 1; i < 4; ++i)
            if (std::fabs(A[i][col]) > std::fabs(A[piv][col])) piv = i;
        if (A[piv][col] == 0.0) return 0.0;
        if (piv != col) {
            for (int j = 0; j < 4; ++j) std::swap(A[piv][j], A[col][j]);
            det = -det;
        }
        det *= A[col][col];
        for (int i = col + 1; i < 4; ++i) {
            double f = A[i][col] / A[col][col];
            for (int j = col; j < 4; ++j) A[i][j] -= f * A[col][j];
        }
    }
    return det;
}

/* v orthogonalised against e0 (timelike, e0.e0 = -1) and the spatial legs listed. */
static void project_out(const Mat4 g, double v[4], const double e0[4], const double* legs[],
                        int nlegs) {
    double p0 = dot(g, v, e0);
    for (int mu = 0; mu < 4; ++mu) v[mu] += p0 * e0[mu];
    for (int l = 0; l < nlegs; ++l) {
        double pl = dot(g, v, legs[l]);
        for (int mu = 0; mu < 4; ++mu) v[mu] -= pl * legs[l][mu];
    }
}

struct FluidFrame {
    double e0[4], e1[4], e2[4], e3[4];
};

static void fluid_frame(const Mat4 g, const double u[4], const double K[4], const double b[4],
                        FluidFrame* F) {
    /* e3: unit spatial direction of K in the fluid frame.  For an exactly null
     * K this is (K + (K.u) u)/(-K.u); normalising explicitly keeps the tetrad
     * orthonormal when the stored K carries the integrator's null drift. */
    double Ku = dot(g, K, u);
    double v3[4];
    for (int mu = 0; mu < 4; ++mu) v3[mu] = K[mu] + Ku * u[mu];
    double n3 = std::sqrt(dot(g, v3, v3));
    for (int mu = 0; mu < 4; ++mu) {
        F->e0[mu] = u[mu];
        F->e3[mu] = v3[mu] / n3;
    }
    const double* l3[1] = {F->e3};
    /* e2: along the field's part transverse to u and e3 */
    double bb = dot(g, b, b);
    double bn = (bb > 0.0) ? std::sqrt(bb) : 0.0;
    double v[4];
    for (int mu = 0; mu < 4; ++mu) v[mu] = b[mu];
    project_out(g, v, F->e0, l3, 1);
    double vv = dot(g, v, v);
    double vn = (vv > 0.0) ? std::sqrt(vv) : 0.0;
    if (!(bn > 0.0) || !(vn >= 1e-10 * bn)) {
        /* fallback: d_theta, then d_r */
        double cand[2][4] = {{0.0, 0.0, 1.0, 0.0}, {0.0, 1.0, 0.0, 0.0}};
        for (int c = 0; c < 2; ++c) {
            double cn = std::sqrt(dot(g, cand[c], cand[c]));
            for (int mu = 0; mu < 4; ++mu) v[mu] = cand[c][mu];
            project_out(g, v, F->e0, l3, 1);
            vv = dot(g, v, v);
            vn = (vv > 0.0) ? std::sqrt(vv) : 0.0;
            if (vn >= 1e-10 * cn) break;
        }
    }
    for (int mu = 0; mu < 4; ++mu) F->e2[mu] = v[mu] / vn;
    /* e1: the coordinate direction with the largest part outside span(e0, e2, e3) */
    const double* l23[2] = {F->e2, F->e3};
    double best[4] = {0, 0, 0, 0}, bestn = -1.0;
    for (int k = 0; k < 4; ++k) {
        double c[4] = {0, 0, 0, 0};
        c[k] = 1.0;
        project_out(g, c, F->e0, l23, 2);
        double cc = dot(g, c, c);
        double cn = (cc > 0.0) ? std::sqrt(cc) : 0.0;
        /* compare the residual relative to the size of the coordinate vector */
        double ref[4] = {0, 0, 0, 0};
        ref[k] = 1.0;
        double rr = std::fabs(dot(g, ref, ref));
        double rel = (rr > 0.0) ? cn / std::sqrt(rr) : 0.0;
        if (rel > bestn) {
            bestn = rel;
            for (int mu = 0; mu < 4; ++mu) best[mu] = c[mu] / cn;
        }
    }
    for (int mu = 0; mu < 4; ++mu) F->e1[mu] = best[mu];
    double D[4][4];
    for (int mu = 0; mu < 4; ++mu) {
        D[0][mu] = F->e0[mu];
        D[1][mu] = F->e1[mu];
        D[2][mu] = F->e2[mu];
        D[3][mu] = F->e3[mu];
    }
    if (det4(D) < 0.0)
        for (int mu = 0; mu < 4; ++mu) F->e1[mu] = -F->e1[mu];
}

/* ---- coherency matrix <-> Stokes on two legs ---- */

static void project(const Mat4 g, const CMat4 N, const double e1[4], const double e2[4],
                    double S[4]) {
    double l1[4], l2[4];
    lower(g, e1, l1);
    lower(g, e2, l2);
    cplx n11 = 0.0, n22 = 0.0, n12 = 0.0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
            n11 += l1[mu] * l1[nu] * N[mu][nu];
            n22 += l2[mu] * l2[nu] * N[mu][nu];
            n12 += l1[mu] * l2[nu] * N[mu][nu];
        }
    S[0] = (n11 + n22).real();
    S[1] = (n11 - n22).real();
    S[2] = 2.0 * n12.real();
    S[3] = -2.0 * n12.imag();
}

static void rebuild(CMat4 N, const double S[4], const double e1[4], const double e2[4]) {
    cplx n11 = 0.5 * (S[0] + S[1]);
    cplx n22 = 0.5 * (S[0] - S[1]);
    cplx n12 = cplx(0.5 * S[2], -0.5 * S[3]);
    cplx n21 = std::conj(n12);
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            N[mu][nu] = n11 * e1[mu] * e1[nu] + n22 * e2[mu] * e2[nu] + n12 * e1[mu] * e2[nu] +
                        n21 * e2[mu] * e1[nu];
}

/* ---- parallel transport ---- */

static void connection_along(double a, double m, const double* pt, double A[4][4]) {
    double G[4][4][4];
    christoffel(a, m, pt[0], pt[1], G);
    const double* K = pt + 3;
    for (int mu = 0; mu < 4; ++mu)
        for (int be = 0; be < 4; ++be) {
            double s = 0.0;
            for (int al = 0; al < 4; ++al) s += G[mu][al][be] * K[al];
            A[mu][be] = s;
        }
}

/* F(A, N) = -(A N + N A^T) */
static void transport_rhs(const double A[4][4], const CMat4 N, CMat4 F) {
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
            cplx s = 0.0;
            for (int be = 0; be < 4; ++be) s += A[mu][be] * N[be][nu] + N[mu][be] * A[nu][be];
            F[mu][nu] = -s;
        }
}

static void heun(const double An[4][4], const double Anm1[4][4], double D, CMat4 N) {
    CMat4 F1, Ns, F2;
    transport_rhs(An, N, F1);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Ns[i][j] = N[i][j] + D * F1[i][j];
    transport_rhs(Anm1, Ns, F2);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) N[i][j] += 0.5 * D * (F1[i][j] + F2[i][j]);
}

/* ---- one radiative update at a stored point ---- */

static void radiative_update(const or_camera* cam, double L_cm, const or_model* model,
                             const or_snapshot* snap, const double* pt, double w, CMat4 N) {
    double a = cam->a, m = (double)cam->mass_factor;
    double r = pt[0], th = pt[1], ph = pt[2];
    const double* K = pt + 3;
    Mat4 g;
    metric(a, m, r, th, g);
    Plasma p;
    const int pk = plasma(model, snap, a, m, r, th, ph, L_cm, &p);
    if (pk == 2) {
        /* non-finite snapshot data at an emitting point: the ray's Stokes
         * vector becomes non-finite, and the pixel is written as zeros with
         * status NONFINITE */
        N[0][0] = cplx(std::numeric_limits<double>::quiet_NaN(), 0.0);
        return;
    }
    if (!pk) return;  /* no valid fluid frame */

    double Ku = dot(g, K, p.u);
    double nu = cam->freq_hz * (-Ku);
    double coef[8];
    if (model->kind == OR_MODEL_SLAB_FIXED) {
        bool inside = r < model->slab_radius;
        for (int k = 0; k < 8; ++k) coef[k] = inside ? model->slab_coef[k] : 0.0;
    } else {
        double bb = dot(g, p.b, p.b);
        double bn = (bb > 0.0) ? std::sqrt(bb) : 0.0;
        double cth = (bn > 0.0) ? dot(g, K, p.b) / (bn * (-Ku)) : 0.0;
        double c[8];
        if (model->electrons == 1)
            kappa_coefficients(OR_DIST_KAPPA, model->kappa, p.ne, p.thetae, p.B, nu, cth, c);
        else
            thermal_coefficients(p.ne, p.thetae, p.B, nu, cth, c);
        double fac = L_cm / cam->freq_hz;
        for (int k = 0; k < 3; ++k) coef[k] = fac * c[k] / (nu * nu);
        for (int k = 3; k < 8; ++k) coef[k] = fac * nu * c[k];
        if (model->kind == OR_MODEL_SLAB_PLASMA && r < model->slab_radius)
            for (int k = 0; k < 3; ++k) coef[k] += model->slab_jextra[k];
    }
    /* No emission, absorption or rotation (e.g. no plasma): the update is the
     * identity on the Stokes vector, and projecting N on the fluid legs and
     * rebuilding it would only drop its components along K, which no later
     * projection sees; the point leaves N as it is. */
    bool zero = true;
    for (int k = 0; k < 8; ++k) zero = zero && coef[k] == 0.0;
    if (zero && !model->update_empty) return;
    FluidFrame F;
    fluid_frame(g, p.u, K, p.b, &F);
    double S[4], S2[4];
    project(g, N, F.e1, F.e2, S);
    mueller_step(coef, S, w, S2);
    rebuild(N, S2, F.e1, F.e2);
}

int transfer(const or_camera* cam, const or_units* units, const or_model* model,
             const or_snapshot* snap, const double ex[4], const double ey[4],
             const double* path, int32_t n_end, double S_out[4]) {
    double a = cam->a, m = (double)cam->mass_factor;
    double L_cm = G_NEWTON * units->M_bh_g / (C_LIGHT * C_LIGHT);
    CMat4 N;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) N[i][j] = 0.0;
    double An[4][4], Anm1[4][4];
    for (int32_t n = n_end; n >= 0; --n) {
        const double* pt = path + 8 * (size_t)n;
        double Dn = std::fabs(pt[7]);
        double Dn1 = (n < n_end) ? std::fabs(path[8 * (size_t)(n + 1) + 7]) : 0.0;
        if (n == 0) Dn = 0.0;
        double w = 0.5 * (Dn + Dn1);
        radiative_update(cam, L_cm, model, snap, pt, w, N);
        if (n > 0) {
            connection_along(a, m, pt, An);
            connection_along(a, m, path + 8 * (size_t)(n - 1), Anm1);
            heun(An, Anm1, Dn, N);
        }
    }
    Mat4 g;
    metric(a, m, cam->r_cam, cam->incl_deg * PI / 180.0, g);
    double S[4];
    project(g, N, ex, ey, S);
    double nu3 = cam->freq_hz * cam->freq_hz * cam->freq_hz;
    for (int k = 0; k < 4; ++k) S_out[k] = S[k] * nu3;
    return 0;
}

}  // namespace orc

extern "C" {

void or_mueller_step(const double coef[8], const double S_in[4], double w, double S_out[4]) {
    orc::mueller_step(coef, S_in, w, S_out);
}

int or_transfer_path(const or_camera* cam, const or_units* units, const or_model* model,
                     const or_snapshot* snap, double alpha, double beta, const double* path,
                     int32_t n_end, double S_out[4]) {
    if (orc::validate_camera(cam) != 0 || orc::validate_model(model, snap, cam) != 0) return -1;
    if (!units || !(units->M_bh_g > 0.0) || !(units->dist_cm > 0.0) || n_end < 0) return -1;
    orc::CameraFrame cf;
    orc::camera_frame(cam, &cf);
    double ex[4], ey[4];
    orc::screen_legs(cam, cf, alpha, beta, ex, ey);
    return orc::transfer(cam, units, model, snap, ex, ey, path, n_end, S_out);
}

}
