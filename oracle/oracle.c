/*
 * Plain FP64 CPU oracle for sequences of Pauli rotations.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may call,
 * link or load this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code with the HIP path.
 *
 * What it computes (paper, "Software implementation" and Supplementary
 * Methods, "Pauli-string bit representation"):
 *   - A Pauli string P is a pair of masks (x, z): bit q of x is set when the
 *     letter on qubit q is X or Y, bit q of z when it is Y or Z.
 *   - On a basis state, P|i> = w(i) |i XOR x>, with w(i) a fourth root of
 *     unity: one factor i per Y letter (i^{popcount(x & z)}, taken mod 4)
 *     and one factor -1 per Y or Z letter acting on a 1 bit of the *source*
 *     index i ((-1)^{popcount(i & z)}).
 *   - A rotation is exp(i phi P) = cos(phi) I + i sin(phi) P.  It is applied
 *     in the paper's two steps: (i) form P psi (a permutation of the array
 *     with phases), (ii) take the linear combination cos(phi) psi +
 *     i sin(phi) (P psi).
 *
 * Step (i) is written in the scatter form: every source amplitude psi[i] is
 * sent to w[i ^ x] with its phase.  There is no pairing, blocking or fusion.
 * The overlap <psi0|psi> = sum_k conj(psi0[k]) psi[k] and the squared norm
 * use Neumaier-compensated FP64 summation in index order.
 *
 * State layout: 2^n complex doubles (C99 double _Complex, i.e. interleaved
 * real and imaginary parts), index k = amplitude of basis state |k>.
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

typedef double _Complex cplx;

static int popcount64(uint64_t v) {
    int c = 0;
    while (v) {
        v &= v - 1;
        c++;
    }
    return c;
}

/* i^m for m = 0, 1, 2, 3 */
static cplx ipow(int m) {
    switch (m & 3) {
    case 0: return 1.0;
    case 1: return I;
    case 2: return -1.0;
    default: return -I;
    }
}

/* w <- P psi in the scatter form.  w must not alias psi. */
void oracle_pauli_apply(int n, uint64_t x, uint64_t z, const cplx *psi, cplx *w) {
    const uint64_t N = (uint64_t)1 << n;
    const cplx yphase = ipow(popcount64(x & z));
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < (int64_t)N; s++) {
        uint64_t i = (uint64_t)s;
        double sign = (popcount64(i & z) & 1) ? -1.0 : 1.0;
        w[i ^ x] = yphase * sign * psi[i];
    }
}

/*
 * psi <- R_M ... R_2 R_1 psi with R_j = exp(i phi_j P_j), rotations taken in
 * the order given (entry 0 first).  work is caller scratch of 2^n entries.
 */
void oracle_apply(int n, size_t M, const uint64_t *x, const uint64_t *z,
                  const double *phi, cplx *psi, cplx *work) {
    const uint64_t N = (uint64_t)1 << n;
    for (size_t j = 0; j < M; j++) {
        memset(work, 0, sizeof(cplx) * N);
        oracle_pauli_apply(n, x[j], z[j], psi, work);
        const double c = cos(phi[j]);
        const cplx is = I * sin(phi[j]);
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < (int64_t)N; s++) {
            psi[s] = c * psi[s] + is * work[s];
        }
    }
}

/* Neumaier-compensated running sum of one real component. */
typedef struct {
    double sum, comp;
} neumaier;

static void neu_add(neumaier *a, double v) {
    double t = a->sum + v;
    if (fabs(a->sum) >= fabs(v))
        a->comp += (a->sum - t) + v;
    else
        a->comp += (v - t) + a->sum;
    a->sum = t;
}

/* out = <psi0|psi> = sum_k conj(psi0[k]) psi[k], summed in index order. */
void oracle_overlap(int n, const cplx *psi0, const cplx *psi, double out[2]) {
    const uint64_t N = (uint64_t)1 << n;
    neumaier re = {0.0, 0.0}, im = {0.0, 0.0};
    for (uint64_t k = 0; k < N; k++) {
        cplx p = conj(psi0[k]) * psi[k];
        neu_add(&re, creal(p));
        neu_add(&im, cimag(p));
    }
    out[0] = re.sum + re.comp;
    out[1] = im.sum + im.comp;
}

/* sum_k |psi[k]|^2, summed in index order. */
double oracle_norm2(int n, const cplx *psi) {
    const uint64_t N = (uint64_t)1 << n;
    neumaier a = {0.0, 0.0};
    for (uint64_t k = 0; k < N; k++) {
        neu_add(&a, creal(psi[k]) * creal(psi[k]));
        neu_add(&a, cimag(psi[k]) * cimag(psi[k]));
    }
    return a.sum + a.comp;
}

/* Number of threads the OpenMP loops use (1 when built without OpenMP). */
int oracle_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
