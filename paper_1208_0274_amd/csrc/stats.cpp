// Threshold H from an E-value (Section 7: H = ceil((ln(K m n) - ln E) / lambda)).
//
// lambda and K are the Karlin-Altschul statistics of ungapped local alignment
// scores (Karlin and Altschul, PNAS 87, 1990), computed from the scoring scheme
// and the residue background:
//   lambda: the positive root of  sum_{a,b} p_a p_b exp(lambda s(a,b)) = 1;
//   H:      the relative entropy  lambda sum p_a p_b s(a,b) exp(lambda s(a,b));
//   K:      lambda d exp(-2 sigma) / (H (1 - exp(-lambda d))), with d the span
//           (gcd) of the scores and
//           sigma = sum_{k>=1} (1/k) (E[exp(lambda S_k); S_k < 0] + P(S_k >= 0)),
//           S_k the sum of k independent pair scores.
// They need a negative expected score and some positive score.  For gapped
// scoring they are the ungapped values: gapped alignments score higher by
// chance, so the H they give is a lower threshold than gapped statistics
// would (more hits reported, none missed).
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <vector>

#include "alae_internal.h"

using namespace alae;

extern "C" {

alae_status alae_karlin_altschul(const alae_scoring *scoring, alae_alphabet alphabet, const double *background,
                                 alae_karlin *out) {
    if (!scoring || !out) {
        set_error("alae_karlin_altschul: null argument");
        return ALAE_E_ARG;
    }
    const int sigma = alphabet_sigma(alphabet);
    if (!sigma) {
        set_error("alae_karlin_altschul: unknown alphabet %d", (int)alphabet);
        return ALAE_E_ARG;
    }
    if (scoring->use_matrix && !scoring->matrix) {
        set_error("alae_karlin_altschul: use_matrix set but matrix is NULL");
        return ALAE_E_ARG;
    }
    std::vector<double> p(sigma, 1.0 / sigma);
    if (background) {
        double sum = 0.0;
        for (int a = 0; a < sigma; ++a) {
            if (!(background[a] >= 0.0)) {
                set_error("alae_karlin_altschul: negative background frequency");
                return ALAE_E_ARG;
            }
            sum += background[a];
        }
        if (!(sum > 0.0)) {
            set_error("alae_karlin_altschul: background frequencies sum to zero");
            return ALAE_E_ARG;
        }
        for (int a = 0; a < sigma; ++a) p[a] = background[a] / sum;
    }
    // distribution of one pair's score
    std::map<int, double> dist;
    for (int a = 0; a < sigma; ++a)
        for (int b = 0; b < sigma; ++b) {
            const int s = scoring->use_matrix ? (int)scoring->matrix[a * sigma + b] : (a == b ? scoring->sa : scoring->sb);
            const double w = p[a] * p[b];
            if (w > 0.0) dist[s] += w;
        }
    double mean = 0.0;
    int d = 0;
    for (const auto &kv : dist) {
        mean += kv.first * kv.second;
        d = std::gcd(d, std::abs(kv.first));
    }
    if (!(mean < 0.0) || dist.rbegin()->first <= 0 || d == 0) {
        set_error("alae_karlin_altschul: the expected pair score must be negative and some score positive");
        return ALAE_E_SCORING;
    }
    auto f = [&](double l) {
        double v = -1.0;
        for (const auto &kv : dist) v += kv.second * std::exp(l * kv.first);
        return v;
    };
    // f(0) = 0, f decreases first (negative mean) and grows without bound: bracket the root
    double lo = 1e-12, hi = 1.0;
    while (f(hi) <= 0.0) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        (f(mid) > 0.0 ? hi : lo) = mid;
    }
    const double lambda = 0.5 * (lo + hi);
    double H = 0.0;
    for (const auto &kv : dist) H += kv.second * kv.first * std::exp(lambda * kv.first);
    H *= lambda;
    // sigma by the distribution of S_k, until the terms fall below 1e-14
    std::map<long, double> cur{{0, 1.0}};
    double sig = 0.0;
    for (int k = 1; k <= 100000; ++k) {
        std::map<long, double> nxt;
        for (const auto &v : cur)
            for (const auto &s : dist) nxt[v.first + s.first] += v.second * s.second;
        cur.clear();
        double term = 0.0;
        for (const auto &v : nxt) {
            if (v.second < 1e-300) continue;
            cur.insert(v);
            term += v.first < 0 ? v.second * std::exp(lambda * v.first) : v.second;
        }
        sig += term / k;
        if (term / k < 1e-14 && k > 8) break;
    }
    const double K = lambda * d * std::exp(-2.0 * sig) / (H * (1.0 - std::exp(-lambda * d)));
    memset(out, 0, sizeof(*out));
    out->lambda = lambda;
    out->K = K;
    out->H = H;
    return ALAE_OK;
}

alae_status alae_evalue_threshold(const alae_karlin *stats, uint64_t m, uint64_t n, double evalue, int32_t *H) {
    if (!stats || !H || m == 0 || n == 0 || !(evalue > 0.0) || !(stats->lambda > 0.0) || !(stats->K > 0.0)) {
        set_error("alae_evalue_threshold: null argument, empty sizes, E <= 0 or statistics not positive");
        return ALAE_E_ARG;
    }
    const double h = (std::log(stats->K * (double)m * (double)n) - std::log(evalue)) / stats->lambda;
    const double c = std::ceil(h);
    *H = c < 1.0 ? 1 : (int32_t)c;  // the zero floor needs H >= 1
    return ALAE_OK;
}

}  // extern "C"
