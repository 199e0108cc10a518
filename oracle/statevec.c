/*
 * oracle/statevec.c -- plain, slow FP64 reference for the VQE hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code with the GPU
 * library: gates are applied as explicit 2^k x 2^k matrices by the textbook
 * gather / multiply / scatter loop, the energy is evaluated term by term,
 * and gradients come from parameter-shift rules or from a plain adjoint
 * sweep.
 *
 * What it follows (arXiv 2601.09951):
 *   - Eq. (2), Section 3.1: E(theta) = <psi(theta)|H|psi(theta)>.
 *   - Eq. (4), Section 3.3: |psi(theta)> = U(theta)|HF>, a product of
 *     parameterised unitaries applied to a 2^N-amplitude state.
 *   - Eq. (5), Section 3.3: the double excitation, read as the qubit Givens
 *     rotation between |0011> and |1100> (the printed exponent is not
 *     anti-Hermitian, so the rotation form is the reading taken).
 *   - Algorithm 1, Section 4.2: per bond length, theta <- 0, then a fixed
 *     number of (energy, gradient, optimiser step) iterations, then the
 *     energy at the final parameters.
 *   - Section 3.4: Adam with learning rate 0.01 (Kingma-Ba form, epsilon
 *     outside the square root, as in Optax which the paper switches to in
 *     Section 4.4.1).
 *   - Section 4.3: the parameter-shift gradient (two evaluations per
 *     parameter for generators with eigenvalues +-1; four for the
 *     excitation gates whose generators have eigenvalues {-1, 0, 1}).
 *
 * Conventions: wire w is bit (n-1-w) of the amplitude index.  Pauli strings
 * are (xmask, zmask) over amplitude-index bits, with
 *     P |b> = i^{popcount(x & z)} (-1)^{popcount(z & b)} |b xor x>.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* gate kinds (this file's own numbering) */
enum {
    ORC_RX = 0, ORC_RY = 1, ORC_RZ = 2, ORC_H = 3, ORC_X = 4,
    ORC_CNOT = 5, ORC_CZ = 6, ORC_SINGLE_EXC = 7, ORC_DOUBLE_EXC = 8
};

static int g_threads = 1;

void orc_set_threads(int t) { g_threads = t < 1 ? 1 : t; }
int orc_get_threads(void) { return g_threads; }

static int arity(int kind) {
    switch (kind) {
    case ORC_RX: case ORC_RY: case ORC_RZ: case ORC_H: case ORC_X: return 1;
    case ORC_CNOT: case ORC_CZ: case ORC_SINGLE_EXC: return 2;
    case ORC_DOUBLE_EXC: return 4;
    default: return -1;
    }
}

int orc_is_parametric(int kind) {
    return kind == ORC_RX || kind == ORC_RY || kind == ORC_RZ ||
           kind == ORC_SINGLE_EXC || kind == ORC_DOUBLE_EXC;
}

/* ------------------------------------------------------------------------
 * Gate matrices, in the local basis |w0 w1 ... w_{k-1}> where w0 (the first
 * listed wire) is the most significant local bit.  c = cos(a/2), s = sin(a/2).
 * ---------------------------------------------------------------------- */
static int gate_matrix(int kind, double a, cplx *M)
{
    const double c = cos(0.5 * a), s = sin(0.5 * a);
    int k = arity(kind);
    if (k < 0) return -1;
    int d = 1 << k;
    for (int i = 0; i < d * d; ++i) M[i] = 0;
#define E(r, col) M[(r) * d + (col)]
    switch (kind) {
    case ORC_RX: /* exp(-i a X / 2) */
        E(0, 0) = c; E(0, 1) = -I * s; E(1, 0) = -I * s; E(1, 1) = c; break;
    case ORC_RY: /* exp(-i a Y / 2) */
        E(0, 0) = c; E(0, 1) = -s; E(1, 0) = s; E(1, 1) = c; break;
    case ORC_RZ: /* exp(-i a Z / 2) */
        E(0, 0) = cexp(-0.5 * I * a); E(1, 1) = cexp(0.5 * I * a); break;
    case ORC_H:
        E(0, 0) = M_SQRT1_2; E(0, 1) = M_SQRT1_2; E(1, 0) = M_SQRT1_2; E(1, 1) = -M_SQRT1_2; break;
    case ORC_X:
        E(0, 1) = 1; E(1, 0) = 1; break;
    case ORC_CNOT: /* control = first wire, target = second */
        E(0, 0) = 1; E(1, 1) = 1; E(2, 3) = 1; E(3, 2) = 1; break;
    case ORC_CZ:
        E(0, 0) = 1; E(1, 1) = 1; E(2, 2) = 1; E(3, 3) = -1; break;
    case ORC_SINGLE_EXC: /* |01> -> c|01> + s|10>,  |10> -> c|10> - s|01> */
        E(0, 0) = 1; E(3, 3) = 1;
        E(1, 1) = c; E(1, 2) = -s; E(2, 1) = s; E(2, 2) = c; break;
    case ORC_DOUBLE_EXC: /* |0011> -> c|0011> + s|1100>, |1100> -> c|1100> - s|0011> */
        for (int i = 0; i < 16; ++i) E(i, i) = 1;
        E(3, 3) = c; E(3, 12) = -s; E(12, 3) = s; E(12, 12) = c; break;
    }
#undef E
    return k;
}

/* Generator G of a parametric gate, U(a) = exp(-i a G / 2). */
static int generator_matrix(int kind, cplx *M)
{
    int k = arity(kind);
    if (k < 0 || !orc_is_parametric(kind)) return -1;
    int d = 1 << k;
    for (int i = 0; i < d * d; ++i) M[i] = 0;
#define E(r, col) M[(r) * d + (col)]
    switch (kind) {
    case ORC_RX: E(0, 1) = 1; E(1, 0) = 1; break;           /* X */
    case ORC_RY: E(0, 1) = -I; E(1, 0) = I; break;          /* Y */
    case ORC_RZ: E(0, 0) = 1; E(1, 1) = -1; break;          /* Z */
    case ORC_SINGLE_EXC: E(1, 2) = -I; E(2, 1) = I; break;  /* (Y(x)X - X(x)Y)/2 */
    case ORC_DOUBLE_EXC: E(3, 12) = -I; E(12, 3) = I; break;
    }
#undef E
    return k;
}

/* Apply a k-qubit matrix to wires[0..k-1]: for every index whose target
 * bits are all clear, gather the 2^k amplitudes, multiply, scatter. */
static void apply_matrix(int n, cplx *psi, int k, const int *wires, const cplx *M)
{
    const uint64_t dim = 1ull << n;
    const int d = 1 << k;
    uint64_t tmask = 0;
    int pos[4];
    for (int j = 0; j < k; ++j) {
        pos[j] = n - 1 - wires[j];
        tmask |= 1ull << pos[j];
    }
    int64_t base;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1 && n >= 12)
    for (base = 0; base < (int64_t)dim; ++base) {
        if ((uint64_t)base & tmask) continue;
        uint64_t idx[16];
        cplx in[16];
        for (int a = 0; a < d; ++a) {
            uint64_t i = (uint64_t)base;
            for (int j = 0; j < k; ++j)
                if ((a >> (k - 1 - j)) & 1) i |= 1ull << pos[j];
            idx[a] = i;
            in[a] = psi[i];
        }
        for (int a = 0; a < d; ++a) {
            cplx acc = 0;
            for (int b = 0; b < d; ++b) acc += M[a * d + b] * in[b];
            psi[idx[a]] = acc;
        }
    }
}

static void dagger(int k, const cplx *M, cplx *Md)
{
    int d = 1 << k;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) Md[c * d + r] = conj(M[r * d + c]);
}

static int check_wires(int n, int kind, const int *wires)
{
    int k = arity(kind);
    if (k < 0) return -1;
    for (int j = 0; j < k; ++j) {
        if (wires[j] < 0 || wires[j] >= n) return -1;
        for (int i = 0; i < j; ++i)
            if (wires[i] == wires[j]) return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
void orc_prepare(int n, uint64_t ref, cplx *psi)
{
    uint64_t dim = 1ull << n;
    for (uint64_t i = 0; i < dim; ++i) psi[i] = 0;
    psi[ref] = 1;
}

int orc_apply_gate(int n, cplx *psi, int kind, const int *wires, double angle, int adjoint)
{
    cplx M[256], Md[256];
    if (check_wires(n, kind, wires)) return -1;
    int k = gate_matrix(kind, angle, M);
    if (adjoint) {
        dagger(k, M, Md);
        apply_matrix(n, psi, k, wires, Md);
    } else {
        apply_matrix(n, psi, k, wires, M);
    }
    return 0;
}

int orc_apply_generator(int n, cplx *psi, int kind, const int *wires)
{
    cplx G[256];
    if (check_wires(n, kind, wires)) return -1;
    int k = generator_matrix(kind, G);
    if (k < 0) return -1;
    apply_matrix(n, psi, k, wires, G);
    return 0;
}

static double gate_angle(int g, const int *pidx, const double *fixed, const double *theta)
{
    return pidx[g] >= 0 ? theta[pidx[g]] : fixed[g];
}

/* U(theta) |psi>: gates in list order.  wires is [n_gates][4]. */
int orc_apply_circuit(int n, cplx *psi, int n_gates, const int *kind, const int *wires,
                      const int *pidx, const double *fixed, const double *theta)
{
    for (int g = 0; g < n_gates; ++g) {
        int rc = orc_apply_gate(n, psi, kind[g], wires + 4 * g,
                                gate_angle(g, pidx, fixed, theta), 0);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Neumaier-compensated summation (Neumaier 1974), used so that the oracle's
 * own rounding error stays far below the parity tolerances.
 * ---------------------------------------------------------------------- */
typedef struct { double s, c; } nsum;

static inline void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

static inline cplx ipow(int e)
{
    switch (e & 3) { case 0: return 1; case 1: return I; case 2: return -1; default: return -I; }
}

/* <psi|P|psi> for one Pauli string, summed over every basis index. */
void orc_expect_pauli(int n, const cplx *psi, uint64_t x, uint64_t z, double *re, double *im)
{
    const uint64_t dim = 1ull << n;
    const cplx phase = ipow(__builtin_popcountll(x & z));
    int T = g_threads > 1 && n >= 12 ? g_threads : 1;
    nsum pr[256], pi[256];
    if (T > 256) T = 256;
    for (int t = 0; t < T; ++t) { pr[t].s = pr[t].c = pi[t].s = pi[t].c = 0; }
#pragma omp parallel num_threads(T) if (T > 1)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint64_t lo = dim * (uint64_t)t / (uint64_t)T, hi = dim * (uint64_t)(t + 1) / (uint64_t)T;
        for (uint64_t b = lo; b < hi; ++b) {
            double sgn = (__builtin_popcountll(z & b) & 1) ? -1.0 : 1.0;
            cplx v = conj(psi[b ^ x]) * phase * sgn * psi[b];
            nadd(&pr[t], creal(v));
            nadd(&pi[t], cimag(v));
        }
    }
    nsum R = {0, 0}, Im = {0, 0};
    for (int t = 0; t < T; ++t) {
        nadd(&R, pr[t].s); nadd(&R, pr[t].c);
        nadd(&Im, pi[t].s); nadd(&Im, pi[t].c);
    }
    *re = nval(&R);
    *im = nval(&Im);
}

/* E = sum_t c_t <psi|P_t|psi>, term by term, ungrouped. */
void orc_expect(int n, const cplx *psi, int64_t T, const uint64_t *x, const uint64_t *z,
                const double *coeff, double *re, double *im)
{
    nsum R = {0, 0}, Im = {0, 0};
    for (int64_t t = 0; t < T; ++t) {
        double r, i;
        orc_expect_pauli(n, psi, x[t], z[t], &r, &i);
        nadd(&R, coeff[t] * r);
        nadd(&Im, coeff[t] * i);
    }
    *re = nval(&R);
    *im = nval(&Im);
}

/* out = H psi, one term at a time: (P psi)[b xor x] += phase (-1)^{z.b} psi[b]. */
void orc_apply_hamiltonian(int n, const cplx *psi, int64_t T, const uint64_t *x,
                           const uint64_t *z, const double *coeff, cplx *out)
{
    const uint64_t dim = 1ull << n;
    for (uint64_t b = 0; b < dim; ++b) out[b] = 0;
    for (int64_t t = 0; t < T; ++t) {
        const cplx ph = coeff[t] * ipow(__builtin_popcountll(x[t] & z[t]));
        int64_t b;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1 && n >= 12)
        for (b = 0; b < (int64_t)dim; ++b) {
            double sgn = (__builtin_popcountll(z[t] & (uint64_t)b) & 1) ? -1.0 : 1.0;
            out[(uint64_t)b ^ x[t]] += ph * sgn * psi[b];
        }
    }
}

/* ------------------------------------------------------------------------
 * Energy and gradients for one parameter vector.
 * ---------------------------------------------------------------------- */
typedef struct {
    int n, n_gates, n_params;
    const int *kind, *wires, *pidx;
    const double *fixed;
    uint64_t ref;
    int64_t T;
    const uint64_t *x, *z;
    const double *coeff;
} problem;

static double energy_at(const problem *P, const double *theta, cplx *work, double *im_out)
{
    double re, im;
    orc_prepare(P->n, P->ref, work);
    orc_apply_circuit(P->n, work, P->n_gates, P->kind, P->wires, P->pidx, P->fixed, theta);
    orc_expect(P->n, work, P->T, P->x, P->z, P->coeff, &re, &im);
    if (im_out) *im_out = im;
    return re;
}

/* energy with the angle of gate g replaced by (angle_g + shift) */
static double energy_gate_shift(const problem *P, const double *theta, int g, double shift, cplx *work)
{
    double re, im;
    orc_prepare(P->n, P->ref, work);
    for (int h = 0; h < P->n_gates; ++h) {
        double a = gate_angle(h, P->pidx, P->fixed, theta);
        if (h == g) a += shift;
        orc_apply_gate(P->n, work, P->kind[h], P->wires + 4 * h, a, 0);
    }
    orc_expect(P->n, work, P->T, P->x, P->z, P->coeff, &re, &im);
    return re;
}

/* Parameter-shift gradient, gate by gate (the chain rule sums shared
 * parameters).  Generators with eigenvalues +-1 (RX, RY, RZ): the two-term
 * rule [E(a + pi/2) - E(a - pi/2)] / 2.  Excitation gates (eigenvalues
 * -1, 0, 1, so frequencies 1/2 and 1 in E(a)): the four-term rule
 *   d+ [E(a + pi/2) - E(a - pi/2)] - d- [E(a + 3pi/2) - E(a - 3pi/2)],
 * d+- = (sqrt2 +- 1) / (4 sqrt2), obtained by fitting
 * a0 + a1 cos(a/2) + b1 sin(a/2) + a2 cos a + b2 sin a. */
static void grad_param_shift(const problem *P, const double *theta, double *grad, cplx *work)
{
    const double dp = (M_SQRT2 + 1.0) / (4.0 * M_SQRT2), dm = (M_SQRT2 - 1.0) / (4.0 * M_SQRT2);
    for (int p = 0; p < P->n_params; ++p) grad[p] = 0;
    for (int g = 0; g < P->n_gates; ++g) {
        int p = P->pidx[g];
        if (p < 0) continue;
        double gg;
        if (P->kind[g] == ORC_SINGLE_EXC || P->kind[g] == ORC_DOUBLE_EXC) {
            gg = dp * (energy_gate_shift(P, theta, g, M_PI_2, work) - energy_gate_shift(P, theta, g, -M_PI_2, work))
               - dm * (energy_gate_shift(P, theta, g, 1.5 * M_PI, work) - energy_gate_shift(P, theta, g, -1.5 * M_PI, work));
        } else {
            gg = 0.5 * (energy_gate_shift(P, theta, g, M_PI_2, work) - energy_gate_shift(P, theta, g, -M_PI_2, work));
        }
        grad[p] += gg;
    }
}

/* Plain adjoint sweep: with U_l = exp(-i a_l G_l / 2),
 *   dE/da_l = 2 Re <lam_l| (-i G_l / 2) |psi_l> = Im <lam_l|G_l|psi_l>,
 * psi_l the state after gate l and lam_l = U_{l+1}^dag ... U_L^dag H psi_L. */
static double grad_adjoint(const problem *P, const double *theta, double *grad,
                           cplx *psi, cplx *lam, cplx *mu)
{
    const uint64_t dim = 1ull << P->n;
    double re, im;
    for (int p = 0; p < P->n_params; ++p) grad[p] = 0;
    orc_prepare(P->n, P->ref, psi);
    orc_apply_circuit(P->n, psi, P->n_gates, P->kind, P->wires, P->pidx, P->fixed, theta);
    orc_apply_hamiltonian(P->n, psi, P->T, P->x, P->z, P->coeff, lam);
    orc_expect(P->n, psi, P->T, P->x, P->z, P->coeff, &re, &im);
    for (int g = P->n_gates - 1; g >= 0; --g) {
        const int *w = P->wires + 4 * g;
        double a = gate_angle(g, P->pidx, P->fixed, theta);
        if (P->pidx[g] >= 0) {
            memcpy(mu, psi, dim * sizeof(cplx));
            orc_apply_generator(P->n, mu, P->kind[g], w);
            nsum acc = {0, 0};
            for (uint64_t b = 0; b < dim; ++b) nadd(&acc, cimag(conj(lam[b]) * mu[b]));
            grad[P->pidx[g]] += nval(&acc);
        }
        orc_apply_gate(P->n, psi, P->kind[g], w, a, 1);
        orc_apply_gate(P->n, lam, P->kind[g], w, a, 1);
    }
    return re;
}

/* Public entry points.  method 0 = parameter shift, 1 = adjoint. */
int orc_energy(int n, int n_gates, const int *kind, const int *wires, const int *pidx,
               const double *fixed, int n_params, uint64_t ref, int64_t T, const uint64_t *x,
               const uint64_t *z, const double *coeff, const double *theta, double *energy,
               double *energy_im)
{
    problem P = {n, n_gates, n_params, kind, wires, pidx, fixed, ref, T, x, z, coeff};
    cplx *work = malloc(sizeof(cplx) << n);
    if (!work) return -2;
    *energy = energy_at(&P, theta, work, energy_im);
    free(work);
    return 0;
}

int orc_energy_grad(int n, int n_gates, const int *kind, const int *wires, const int *pidx,
                    const double *fixed, int n_params, uint64_t ref, int64_t T,
                    const uint64_t *x, const uint64_t *z, const double *coeff,
                    const double *theta, int method, double *energy, double *grad)
{
    problem P = {n, n_gates, n_params, kind, wires, pidx, fixed, ref, T, x, z, coeff};
    cplx *a = malloc(sizeof(cplx) << n), *b = NULL, *c = NULL;
    if (!a) return -2;
    if (method == 1) {
        b = malloc(sizeof(cplx) << n);
        c = malloc(sizeof(cplx) << n);
        if (!b || !c) { free(a); free(b); free(c); return -2; }
        *energy = grad_adjoint(&P, theta, grad, a, b, c);
    } else {
        *energy = energy_at(&P, theta, a, NULL);
        grad_param_shift(&P, theta, grad, a);
    }
    free(a); free(b); free(c);
    return 0;
}

/* One Adam step (Kingma & Ba, Algorithm 1; epsilon added to sqrt(v_hat)),
 * t = 1 on the first call. */
void orc_adam_step(int P, double *theta, double *m, double *v, const double *g, int t,
                   double lr, double b1, double b2, double eps)
{
    for (int p = 0; p < P; ++p) {
        m[p] = b1 * m[p] + (1.0 - b1) * g[p];
        v[p] = b2 * v[p] + (1.0 - b2) * g[p] * g[p];
        double mh = m[p] / (1.0 - pow(b1, t));
        double vh = v[p] / (1.0 - pow(b2, t));
        theta[p] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* The per-bond-length VQE loop of Algorithm 1: theta starts at theta0, then
 * `iters` rounds of (energy, gradient, optimiser step).  opt 0 = Adam
 * (lr, b1, b2, eps), opt 1 = plain gradient descent with step lr.  The
 * energy before every step goes to energies[0..iters-1], the energy at the
 * final parameters to energies[iters]; theta is updated in place. */
int orc_vqe_run(int n, int n_gates, const int *kind, const int *wires, const int *pidx,
                const double *fixed, int n_params, uint64_t ref, int64_t T, const uint64_t *x,
                const uint64_t *z, const double *coeff, double *theta, int iters, int opt,
                double lr, double b1, double b2, double eps, int grad_method, double *energies)
{
    problem P = {n, n_gates, n_params, kind, wires, pidx, fixed, ref, T, x, z, coeff};
    double *g = calloc((size_t)n_params, sizeof(double));
    double *m = calloc((size_t)n_params, sizeof(double));
    double *v = calloc((size_t)n_params, sizeof(double));
    cplx *a = malloc(sizeof(cplx) << n), *b = malloc(sizeof(cplx) << n), *c = malloc(sizeof(cplx) << n);
    if (!g || !m || !v || !a || !b || !c) {
        free(g); free(m); free(v); free(a); free(b); free(c);
        return -2;
    }
    for (int it = 0; it < iters; ++it) {
        if (grad_method == 1) {
            energies[it] = grad_adjoint(&P, theta, g, a, b, c);
        } else {
            energies[it] = energy_at(&P, theta, a, NULL);
            grad_param_shift(&P, theta, g, a);
        }
        if (opt == 0) {
            orc_adam_step(n_params, theta, m, v, g, it + 1, lr, b1, b2, eps);
        } else {
            for (int p = 0; p < n_params; ++p) theta[p] -= lr * g[p];
        }
    }
    energies[iters] = energy_at(&P, theta, a, NULL);
    free(g); free(m); free(v); free(a); free(b); free(c);
    return 0;
}
