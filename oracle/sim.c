/*
 * Oracle: plain complex128 gate application, written straight from the
 * definition of gate application in the paper's introduction (Eq. 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the GPU path.
 *
 * Conventions (the paper leaves them open; readings recorded in the design
 * notes):
 *   - qubit q is bit q of the amplitude index (stride 2^q), as in the paper's
 *     one-qubit kernel, which uses k = 1 << target;
 *   - inside the 2^k x 2^k gate matrix, targets[0] is the most significant
 *     bit of the row/column index (Eq. 1 lists tau_1 first);
 *   - the gate acts only where every control bit is 1.
 *
 * The computation is deliberately out-of-place (two buffers) and loops over
 * output amplitudes: for each output index i it rebuilds the sum of Eq. 1
 * over the 2^k values tau' of the target bits.  No grouping, no pairing, no
 * in-place update: those belong to the fast path this file checks.
 */
#include <complex.h>
#include <stdint.h>

typedef double _Complex cplx;

/* Eq. 1: psi'(sigma) = sum_{tau'} G(tau, tau') psi(sigma with targets := tau')
 * where tau is the value of the target bits of the output index. */
void oracle_apply_gate(int n, const cplx *in, cplx *out, const cplx *G,
                       const int *targets, int k, const int *controls, int c)
{
    const int64_t dim = (int64_t)1 << n;
    const int64_t gdim = (int64_t)1 << k;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        int active = 1;
        for (int j = 0; j < c; ++j)
            if (((i >> controls[j]) & 1) == 0) active = 0;
        if (!active) {
            out[i] = in[i];
            continue;
        }
        /* tau: the output's target bits, targets[0] as the most significant */
        int64_t tau = 0;
        for (int j = 0; j < k; ++j)
            tau |= ((i >> targets[j]) & 1) << (k - 1 - j);
        /* the output index with every target bit cleared */
        int64_t rest = i;
        for (int j = 0; j < k; ++j)
            rest &= ~((int64_t)1 << targets[j]);
        cplx acc = 0.0;
        for (int64_t tp = 0; tp < gdim; ++tp) {
            int64_t src = rest;
            for (int j = 0; j < k; ++j)
                src |= ((tp >> (k - 1 - j)) & 1) << targets[j];
            acc += G[tau * gdim + tp] * in[src];
        }
        out[i] = acc;
    }
}

/* Squared modulus of every amplitude, in double precision (the building block
 * of measurement probabilities; the sums over unmeasured bits are done by the
 * Python side with numpy's pairwise summation). */
void oracle_abs2(int n, const cplx *in, double *out)
{
    const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        double re = creal(in[i]), im = cimag(in[i]);
        out[i] = re * re + im * im;
    }
}

/* Fill with the computational basis state |x>. */
void oracle_basis_state(int n, cplx *out, int64_t x)
{
    const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) out[i] = (i == x) ? 1.0 : 0.0;
}

/* Number of OpenMP threads the gate loop will use (0 when built without
 * OpenMP), so the baseline timing can state its core count. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 0;
#endif
}
