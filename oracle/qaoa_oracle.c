/*
 * qaoa_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, single-threaded FP64 reference for the exact QAOA-for-QUBO
 * statevector computation of the paper ("A Distributed Quantum Approximate
 * Optimization Algorithm Simulator for Engineering Design Optimization").
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant with the HIP
 * library; every routine is written from the paper's definitions:
 *
 *   canonical form          Sec. "QUBO Formulation", eq. (3)-(6)
 *   cost Hamiltonian        Sec. "Mapping QUBO to Quantum Cost Hamiltonian", eq. (8)
 *   cost unitary            eq. (10)      U_C(gamma) = exp(-i gamma H_C)
 *   QAOA state              eq. (11)      U_M(b_p)U_C(g_p)...U_M(b_1)U_C(g_1)|+>^n
 *   mixer                   eq. (12)-(13) U_M(beta) = exp(-i beta sum_i X_i)
 *   expectation / objective eq. (15), (17)
 *
 * Conventions (the paper's decoding section): variable z_i (i = 1..n) is
 * qubit i-1, i.e. bit (i-1) of the basis index.  States are arrays of 2^n
 * complex doubles stored as interleaved (re, im) pairs.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no -ffast-math, no OpenMP).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* eq. (4)-(5): l_i = f_i + H_ii ;  b_ij = H_ij + H_ji for i < j.
 * H is n x n row-major; f may be NULL (treated as zero).  b is written as a
 * full n x n row-major matrix of which only the strict upper triangle is set
 * (the rest is zero). */
void orc_canonicalise(int n, const double *H, const double *f, double *ell, double *b)
{
    for (int i = 0; i < n; ++i) {
        ell[i] = (f ? f[i] : 0.0) + H[(size_t)i * n + i];
        for (int j = 0; j < n; ++j) b[(size_t)i * n + j] = 0.0;
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            b[(size_t)i * n + j] = H[(size_t)i * n + j] + H[(size_t)j * n + i];
}

/* eq. (6) for integer coefficients: C(z) = c0 + sum_i l_i z_i + sum_{i<j} b_ij z_i z_j,
 * exactly, in 64-bit integers.  b is n x n row-major (strict upper triangle used). */
void orc_cost_diag_int(int n, const int64_t *ell, const int64_t *b, int64_t c0, int64_t *diag)
{
    const uint64_t dim = (uint64_t)1 << n;
    for (uint64_t z = 0; z < dim; ++z) {
        int64_t acc = c0;
        for (int i = 0; i < n; ++i)
            if ((z >> i) & 1u) acc += ell[i];
        for (int i = 0; i < n; ++i) {
            if (!((z >> i) & 1u)) continue;
            for (int j = i + 1; j < n; ++j)
                if ((z >> j) & 1u) acc += b[(size_t)i * n + j];
        }
        diag[z] = acc;
    }
}

/* eq. (6) for real coefficients, in FP64, summed in the canonical order:
 * start from c0, add l_i for ascending i, then b_ij row by row (i ascending,
 * then j ascending), skipping terms whose bits are zero. */
void orc_cost_diag_real(int n, const double *ell, const double *b, double c0, double *diag)
{
    const uint64_t dim = (uint64_t)1 << n;
    for (uint64_t z = 0; z < dim; ++z) {
        double acc = c0;
        for (int i = 0; i < n; ++i)
            if ((z >> i) & 1u) acc += ell[i];
        for (int i = 0; i < n; ++i) {
            if (!((z >> i) & 1u)) continue;
            for (int j = i + 1; j < n; ++j)
                if ((z >> j) & 1u) acc += b[(size_t)i * n + j];
        }
        diag[z] = acc;
    }
}

/* |+>^n : every amplitude 2^(-n/2)  (eq. (11), initial state). */
static void plus_state(int n, cplx *psi)
{
    const uint64_t dim = (uint64_t)1 << n;
    const double a = 1.0 / sqrt((double)dim);
    for (uint64_t z = 0; z < dim; ++z) psi[z] = a;
}

/* psi(z) *= exp(-i * sign * gamma * C(z))   (eq. (10); sign = -1 gives the inverse).
 * theta = gamma * C(z) is one FP64 product; cos/sin are libm on the unreduced angle. */
void orc_apply_phase(int n, const double *diag, double gamma, int sign, double *psi_ri)
{
    cplx *psi = (cplx *)psi_ri;
    const uint64_t dim = (uint64_t)1 << n;
    for (uint64_t z = 0; z < dim; ++z) {
        const double theta = gamma * diag[z];
        const cplx u = cos(theta) - I * (sign * sin(theta));
        psi[z] = psi[z] * u;
    }
}

/* U_M(beta) = exp(-i beta sum_q X_q) = prod_q RX_q(2 beta)  (eq. (12)-(13)).
 * On each qubit q, the pair (a, b) = (psi(z), psi(z + 2^q)) with bit q of z
 * clear becomes (cos(beta) a - i sin(beta) b, -i sin(beta) a + cos(beta) b).
 * sign = -1 applies the inverse RX(-2 beta). */
void orc_apply_mixer(int n, double beta, int sign, double *psi_ri)
{
    cplx *psi = (cplx *)psi_ri;
    const uint64_t dim = (uint64_t)1 << n;
    const double c = cos(beta), s = sign * sin(beta);
    for (int q = 0; q < n; ++q) {
        const uint64_t m = (uint64_t)1 << q;
        for (uint64_t z = 0; z < dim; ++z) {
            if (z & m) continue;
            const cplx a = psi[z], bb = psi[z | m];
            psi[z] = c * a - I * s * bb;
            psi[z | m] = -I * s * a + c * bb;
        }
    }
}

/* eq. (11): |gamma, beta> for x = [gamma_1, beta_1, ..., gamma_p, beta_p]. */
void orc_qaoa_state(int n, const double *diag, int p, const double *x, double *psi_ri)
{
    plus_state(n, (cplx *)psi_ri);
    for (int k = 0; k < p; ++k) {
        orc_apply_phase(n, diag, x[2 * k], +1, psi_ri);
        orc_apply_mixer(n, x[2 * k + 1], +1, psi_ri);
    }
}

/* Partitioned variant: the cost unitary of every layer is applied as a
 * sequence of diagonal factors exp(-i gamma C_d), d = 0..ndiag-1, where the
 * C_d are the per-QPU local parts followed by the cross-QPU part (eq. (16)).
 * diags holds ndiag consecutive arrays of 2^n entries. */
void orc_qaoa_state_multi(int n, int ndiag, const double *diags, int p, const double *x, double *psi_ri)
{
    const uint64_t dim = (uint64_t)1 << n;
    plus_state(n, (cplx *)psi_ri);
    for (int k = 0; k < p; ++k) {
        for (int d = 0; d < ndiag; ++d)
            orc_apply_phase(n, diags + (size_t)d * dim, x[2 * k], +1, psi_ri);
        orc_apply_mixer(n, x[2 * k + 1], +1, psi_ri);
    }
}

/* eq. (15)/(17): <psi|H_C|psi> = sum_z |psi(z)|^2 C(z), accumulated in z order. */
double orc_expectation(int n, const double *diag, const double *psi_ri)
{
    const cplx *psi = (const cplx *)psi_ri;
    const uint64_t dim = (uint64_t)1 << n;
    double e = 0.0;
    for (uint64_t z = 0; z < dim; ++z) {
        const double pz = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
        e += pz * diag[z];
    }
    return e;
}

/* Sum over q of <lam| X_q |psi>. */
static cplx sum_x_expect(int n, const cplx *lam, const cplx *psi)
{
    const uint64_t dim = (uint64_t)1 << n;
    cplx acc = 0.0;
    for (int q = 0; q < n; ++q) {
        const uint64_t m = (uint64_t)1 << q;
        for (uint64_t z = 0; z < dim; ++z) acc += conj(lam[z]) * psi[z ^ m];
    }
    return acc;
}

/* Exact gradient of E(x) = <x|H_C|x> by the adjoint method.
 *
 * With psi the final state and lam = H_C psi, sweep the layers backwards.
 * The derivative of U_M(beta) is -i H_M U_M(beta) and that of U_C(gamma) is
 * -i H_C U_C(gamma), so
 *     dE/dbeta_k  = 2 Im <lam_k | H_M | psi_k>   (both taken after mixer k),
 *     dE/dgamma_k = 2 Im <lam'_k| H_C | psi'_k>  (both taken after phase k),
 * and moving from one point to the previous one applies the inverse layer
 * factor to both vectors.  Output is interleaved like x.  Returns E. */
double orc_adjoint_gradient(int n, const double *diag, int p, const double *x, double *grad)
{
    const uint64_t dim = (uint64_t)1 << n;
    cplx *psi = (cplx *)malloc(sizeof(cplx) * dim);
    cplx *lam = (cplx *)malloc(sizeof(cplx) * dim);
    orc_qaoa_state(n, diag, p, x, (double *)psi);
    const double e = orc_expectation(n, diag, (const double *)psi);
    for (uint64_t z = 0; z < dim; ++z) lam[z] = diag[z] * psi[z];
    for (int k = p - 1; k >= 0; --k) {
        grad[2 * k + 1] = 2.0 * cimag(sum_x_expect(n, lam, psi));
        orc_apply_mixer(n, x[2 * k + 1], -1, (double *)psi);
        orc_apply_mixer(n, x[2 * k + 1], -1, (double *)lam);
        cplx acc = 0.0;
        for (uint64_t z = 0; z < dim; ++z) acc += conj(lam[z]) * diag[z] * psi[z];
        grad[2 * k] = 2.0 * cimag(acc);
        if (k > 0) {
            orc_apply_phase(n, diag, x[2 * k], -1, (double *)psi);
            orc_apply_phase(n, diag, x[2 * k], -1, (double *)lam);
        }
    }
    free(psi);
    free(lam);
    return e;
}
