// Hamiltonians, product-formula schedules, error reporting.
//
// Schedules (Methods, "Hamiltonian simulation"; time sign e^{+itH}; entry 0
// of a rotation list acts first):
//   first-order Trotter (Eq. define-trotter), phi = (t/S) h;
//   second-order Trotter, per step forward at ((t/S) h) 0.5 then reversed;
//   qDRIFT, N draws with p_j = |h_j| / lambda at sgn(h_j) ((lambda t) / N);
//   partially randomised (Eq. hamil_split): the L_det largest-|h| terms as
//   second-order Trotter around r qDRIFT draws from the rest per step.
// Lexicographic ordering of deterministic terms (Methods, "Data analysis")
// is a stable sort by (x, z) as unsigned integers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"
#include "objects.h"

namespace prx {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

prx_status fail(prx_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

prx_status hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PRX_ERR_HIP;
}

// SplitMix64 (Steele, Lea and Flood, 2014): Weyl sequence with increment
// 0x9E3779B97F4A7C15 followed by the variant-13 finaliser.
struct SplitMix64 {
    uint64_t state;
    explicit SplitMix64(uint64_t seed) : state(seed) {}
    uint64_t next() {
        state += 0x9E3779B97F4A7C15ull;
        uint64_t v = state;
        v = (v ^ (v >> 30)) * 0xBF58476D1CE4E5B9ull;
        v = (v ^ (v >> 27)) * 0x94D049BB133111EBull;
        return v ^ (v >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

// Running sums of |h| (left to right); the sampler picks the first index
// whose running sum exceeds u * total.
struct Sampler {
    std::vector<double> prefix;
    explicit Sampler(const std::vector<double> &mags) {
        prefix.resize(mags.size());
        double s = 0.0;
        for (size_t i = 0; i < mags.size(); ++i) {
            s += mags[i];
            prefix[i] = s;
        }
    }
    double total() const { return prefix.empty() ? 0.0 : prefix.back(); }
    size_t draw(SplitMix64 &rng) const {
        const double target = rng.uniform() * total();
        auto it = std::upper_bound(prefix.begin(), prefix.end(), target);
        if (it == prefix.end()) --it;
        return (size_t)(it - prefix.begin());
    }
};

static inline double sgn(double h) { return h < 0 ? -1.0 : 1.0; }

static std::vector<size_t> suffix_sorted(const prx_ham &H, std::vector<size_t> idx) {
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
        if (H.x[a] != H.x[b]) return H.x[a] < H.x[b];
        return H.z[a] < H.z[b];
    });
    return idx;
}

static void push(prx_sched &s, uint64_t x, uint64_t z, double phi) {
    s.x.push_back(x);
    s.z.push_back(z);
    s.phi.push_back(phi);
}

}  // namespace prx

using namespace prx;

extern "C" {

const char *prx_last_error(void) { return g_last_error.c_str(); }
const char *prx_version(void) { return "prx 0.1 (gfx950)"; }

prx_status prx_ham_create(int n, size_t L, const uint64_t *x, const uint64_t *z,
                          const double *h, prx_ham **out) {
    if (!out || !x || !z || !h) return fail(PRX_ERR_INVALID, "null pointer");
    if (n < 1 || n > 63) return fail(PRX_ERR_INVALID, "n must be in [1, 63]");
    if (L == 0) return fail(PRX_ERR_INVALID, "L must be positive");
    const uint64_t lim = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    for (size_t l = 0; l < L; ++l) {
        if ((x[l] & ~lim) || (z[l] & ~lim))
            return fail(PRX_ERR_INVALID, "term " + std::to_string(l) + " acts beyond qubit n-1");
        if (!std::isfinite(h[l]))
            return fail(PRX_ERR_INVALID, "term " + std::to_string(l) + " has a non-finite h");
    }
    prx_ham *H = new (std::nothrow) prx_ham;
    if (!H) return fail(PRX_ERR_OOM, "out of host memory");
    try {
        H->n = n;
        H->x.assign(x, x + L);
        H->z.assign(z, z + L);
        H->h.assign(h, h + L);
    } catch (...) {
        delete H;
        return fail(PRX_ERR_OOM, "out of host memory");
    }
    *out = H;
    return PRX_OK;
}

void prx_ham_destroy(prx_ham *H) { delete H; }

prx_status prx_ham_lambda(const prx_ham *H, double *out) {
    if (!H || !out) return fail(PRX_ERR_INVALID, "null pointer");
    double s = 0.0;
    for (double v : H->h) s += std::fabs(v);
    *out = s;
    return PRX_OK;
}

prx_status prx_sched_from_rotations(int n, size_t M, const uint64_t *x, const uint64_t *z,
                                    const double *phi, prx_sched **out) {
    if (!out || (M && (!x || !z || !phi))) return fail(PRX_ERR_INVALID, "null pointer");
    if (n < 1 || n > 63) return fail(PRX_ERR_INVALID, "n must be in [1, 63]");
    const uint64_t lim = (1ull << n) - 1ull;
    for (size_t j = 0; j < M; ++j) {
        if ((x[j] & ~lim) || (z[j] & ~lim))
            return fail(PRX_ERR_INVALID, "rotation " + std::to_string(j) + " acts beyond qubit n-1");
        if (!std::isfinite(phi[j]))
            return fail(PRX_ERR_INVALID, "rotation " + std::to_string(j) + " has a non-finite angle");
    }
    prx_sched *s = new (std::nothrow) prx_sched;
    if (!s) return fail(PRX_ERR_OOM, "out of host memory");
    try {
        s->n = n;
        s->x.assign(x, x + M);
        s->z.assign(z, z + M);
        s->phi.assign(phi, phi + M);
    } catch (...) {
        delete s;
        return fail(PRX_ERR_OOM, "out of host memory");
    }
    *out = s;
    return PRX_OK;
}

prx_status prx_sched_trotter(const prx_ham *H, int order, double t, int steps,
                             prx_reorder reorder, prx_sched **out) {
    if (!H || !out) return fail(PRX_ERR_INVALID, "null pointer");
    if (order != 1 && order != 2) return fail(PRX_ERR_INVALID, "order must be 1 or 2");
    if (steps < 1) return fail(PRX_ERR_INVALID, "steps must be >= 1");
    if (!std::isfinite(t)) return fail(PRX_ERR_INVALID, "t must be finite");
    if (reorder < PRX_REORDER_NONE || reorder > PRX_REORDER_SUFFIX)
        return fail(PRX_ERR_INVALID, "bad reorder mode");
    std::vector<size_t> idx(H->h.size());
    std::iota(idx.begin(), idx.end(), 0);
    if (reorder == PRX_REORDER_SUFFIX) idx = suffix_sorted(*H, idx);
    prx_sched *s = new (std::nothrow) prx_sched;
    if (!s) return fail(PRX_ERR_OOM, "out of host memory");
    try {
        s->n = H->n;
        const double delta = t / steps;
        const size_t per = idx.size() * (size_t)order;
        s->x.reserve(per * steps);
        s->z.reserve(per * steps);
        s->phi.reserve(per * steps);
        for (int st = 0; st < steps; ++st) {
            if (order == 1) {
                for (size_t l : idx) push(*s, H->x[l], H->z[l], delta * H->h[l]);
            } else {
                for (size_t l : idx) push(*s, H->x[l], H->z[l], (delta * H->h[l]) * 0.5);
                for (auto it = idx.rbegin(); it != idx.rend(); ++it)
                    push(*s, H->x[*it], H->z[*it], (delta * H->h[*it]) * 0.5);
            }
        }
    } catch (...) {
        delete s;
        return fail(PRX_ERR_OOM, "out of host memory");
    }
    *out = s;
    return PRX_OK;
}

prx_status prx_sched_qdrift(const prx_ham *H, double t, size_t N, uint64_t seed,
                            prx_sched **out) {
    if (!H || !out) return fail(PRX_ERR_INVALID, "null pointer");
    if (N < 1) return fail(PRX_ERR_INVALID, "N must be >= 1");
    if (!std::isfinite(t)) return fail(PRX_ERR_INVALID, "t must be finite");
    std::vector<double> mags(H->h.size());
    for (size_t l = 0; l < mags.size(); ++l) mags[l] = std::fabs(H->h[l]);
    Sampler smp(mags);
    const double lam = smp.total();
    if (!(lam > 0.0)) return fail(PRX_ERR_INVALID, "lambda must be positive");
    prx_sched *s = new (std::nothrow) prx_sched;
    if (!s) return fail(PRX_ERR_OOM, "out of host memory");
    try {
        s->n = H->n;
        SplitMix64 rng(seed);
        const double ang = (lam * t) / (double)N;
        s->x.reserve(N);
        s->z.reserve(N);
        s->phi.reserve(N);
        for (size_t i = 0; i < N; ++i) {
            const size_t j = smp.draw(rng);
            push(*s, H->x[j], H->z[j], sgn(H->h[j]) * ang);
        }
    } catch (...) {
        delete s;
        return fail(PRX_ERR_OOM, "out of host memory");
    }
    *out = s;
    return PRX_OK;
}

prx_status prx_sched_partial(const prx_ham *H, size_t L_det, double t, int steps,
                             size_t r_per_step, uint64_t seed, prx_reorder reorder,
                             prx_sched **out) {
    if (!H || !out) return fail(PRX_ERR_INVALID, "null pointer");
    const size_t L = H->h.size();
    if (L_det > L) return fail(PRX_ERR_INVALID, "L_det exceeds the number of terms");
    if (steps < 1) return fail(PRX_ERR_INVALID, "steps must be >= 1");
    if (!std::isfinite(t)) return fail(PRX_ERR_INVALID, "t must be finite");
    if (L_det < L && r_per_step == 0)
        return fail(PRX_ERR_INVALID, "r_per_step must be >= 1 when the random part is non-empty");
    if (reorder < PRX_REORDER_NONE || reorder > PRX_REORDER_SUFFIX)
        return fail(PRX_ERR_INVALID, "bad reorder mode");
    // D: the L_det largest |h| (ties to the lower index), in original order.
    std::vector<size_t> rank(L);
    std::iota(rank.begin(), rank.end(), 0);
    std::stable_sort(rank.begin(), rank.end(), [&](size_t a, size_t b) {
        return std::fabs(H->h[a]) > std::fabs(H->h[b]);
    });
    std::vector<char> inD(L, 0);
    for (size_t i = 0; i < L_det; ++i) inD[rank[i]] = 1;
    std::vector<size_t> D, R;
    for (size_t l = 0; l < L; ++l) (inD[l] ? D : R).push_back(l);
    if (reorder == PRX_REORDER_SUFFIX) D = suffix_sorted(*H, D);
    std::vector<double> magsR(R.size());
    for (size_t i = 0; i < R.size(); ++i) magsR[i] = std::fabs(H->h[R[i]]);
    Sampler smp(magsR);
    const double lamR = smp.total();
    if (!R.empty() && !(lamR > 0.0))
        return fail(PRX_ERR_INVALID, "random part has zero weight");
    prx_sched *s = new (std::nothrow) prx_sched;
    if (!s) return fail(PRX_ERR_OOM, "out of host memory");
    try {
        s->n = H->n;
        SplitMix64 rng(seed);
        const double delta = t / steps;
        const double ang = R.empty() ? 0.0 : (lamR * delta) / (double)r_per_step;
        for (int st = 0; st < steps; ++st) {
            for (size_t l : D) push(*s, H->x[l], H->z[l], (delta * H->h[l]) * 0.5);
            if (!R.empty()) {
                for (size_t i = 0; i < r_per_step; ++i) {
                    const size_t j = R[smp.draw(rng)];
                    push(*s, H->x[j], H->z[j], sgn(H->h[j]) * ang);
                }
            }
            for (auto it = D.rbegin(); it != D.rend(); ++it)
                push(*s, H->x[*it], H->z[*it], (delta * H->h[*it]) * 0.5);
        }
    } catch (...) {
        delete s;
        return fail(PRX_ERR_OOM, "out of host memory");
    }
    *out = s;
    return PRX_OK;
}

prx_status prx_sched_view(const prx_sched *s, int *n, size_t *M, const uint64_t **x,
                          const uint64_t **z, const double **phi) {
    if (!s) return fail(PRX_ERR_INVALID, "null schedule");
    if (n) *n = s->n;
    if (M) *M = s->x.size();
    if (x) *x = s->x.data();
    if (z) *z = s->z.data();
    if (phi) *phi = s->phi.data();
    return PRX_OK;
}

void prx_sched_destroy(prx_sched *s) { delete s; }

}  // extern "C"
