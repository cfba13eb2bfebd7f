/*
 * Oracle: discrete operators.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 *  - K-hat x by CSR (Remark: K = D^-1 K-hat).
 *  - GL_i(psi) = (K psi)_i - psi_i (1 - |psi_i|^2)      (discrete GL equations)
 *  - (J(psi) phi)_i = (K phi)_i + (2|psi_i|^2 - 1) phi_i + psi_i^2 conj(phi_i)
 *                                                      (discrete Jacobian)
 *  - <u, v>_R = Re sum_i |V_i| conj(u_i) v_i           (discrete inner products)
 *  - F(psi) = sum_edges alpha |psi_j - U_jk psi_k|^2
 *             + sum_i |V_i| (-|psi_i|^2 + |psi_i|^4 / 2) (discrete energy)
 *  - H = K-hat + 2 D |psi|^2, the matrix of the preconditioner operator
 *    P = K + 2|psi|^2 scaled by D (Sec. 4.1).
 */
#include "oracle.h"

void orc_khat_apply(const orc_mesh *m, const cplx *x, cplx *y)
{
    for (int64_t i = 0; i < m->n; ++i) {
        cplx s = 0;
        for (int64_t p = m->rp[i]; p < m->rp[i + 1]; ++p) s += m->kv[p] * x[m->ci[p]];
        y[i] = s;
    }
}

void orc_gl(const orc_mesh *m, const cplx *psi, cplx *out)
{
    orc_khat_apply(m, psi, out);
    for (int64_t i = 0; i < m->n; ++i) {
        double a2 = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
        out[i] = out[i] / m->vol[i] - psi[i] * (1.0 - a2);
    }
}

void orc_jac(const orc_mesh *m, const cplx *psi, const cplx *phi, cplx *out)
{
    orc_khat_apply(m, phi, out);
    for (int64_t i = 0; i < m->n; ++i) {
        double a2 = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
        out[i] = out[i] / m->vol[i] + (2.0 * a2 - 1.0) * phi[i] + psi[i] * psi[i] * conj(phi[i]);
    }
}

double orc_inner(const orc_mesh *m, const cplx *u, const cplx *v)
{
    double s = 0.0;
    for (int64_t i = 0; i < m->n; ++i) s += m->vol[i] * creal(conj(u[i]) * v[i]);
    return s;
}

double orc_energy(const orc_mesh *m, const cplx *psi)
{
    double f1 = 0.0, f2 = 0.0;
    for (int64_t q = 0; q < m->ne; ++q) {
        cplx d = psi[m->ej[q]] - m->U[q] * psi[m->ek[q]];
        f1 += m->alpha[q] * (creal(d) * creal(d) + cimag(d) * cimag(d));
    }
    for (int64_t i = 0; i < m->n; ++i) {
        double a2 = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
        f2 += m->vol[i] * (-a2 + 0.5 * a2 * a2);
    }
    return f1 + f2;
}

void orc_hmat_values(const orc_mesh *m, const cplx *psi, cplx *hv)
{
    for (int64_t i = 0; i < m->n; ++i)
        for (int64_t p = m->rp[i]; p < m->rp[i + 1]; ++p) {
            hv[p] = m->kv[p];
            if (m->ci[p] == i) {
                double a2 = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
                hv[p] += 2.0 * m->vol[i] * a2;
            }
        }
}
