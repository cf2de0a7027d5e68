// Chunk rules of the loop-scheduling techniques whose chunk depends on the
// requesting worker (the "more complex" techniques the paper leaves to
// future work, Section 6), shared by the spin kernel's claim code and the
// host functions of the C ABI.
//
//   WF  (weighted factoring, Hummel, Schmidt, Uma and Wein 1996): factoring's
//       batches of P requests; a request of a worker of relative speed w
//       (the weights sum to P) in batch b gets ceil(w c_b), c_b being FAC2's
//       chunk of batch b (ceil(R_b / (x P)) along FAC2's own schedule).
//   AWF (adaptive weighted factoring, Banicescu, Velusamy and Devaprasad
//       2003, adapting after every chunk as in Carino and Banicescu 2008):
//       WF with weights from measured rates, w_i = P r_i / sum_j r_j, where
//       r_i = (sum_k k n_ik) / (sum_k k t_ik) over worker i's completed chunks
//       k = 1, 2, ... (iterations per unit time, later chunks weighing more).
//   AF  (adaptive factoring, Banicescu and Liu 2000): a request of worker i
//       with R iterations left gets
//           K_i = (D + 2 T R - sqrt(D^2 + 4 D T R)) / (2 mu_i),
//       D = sum_j sigma_j^2 / mu_j, T = 1 / sum_j (1 / mu_j), from the mean and
//       standard deviation of each worker's iteration times.
// The sums over workers run over those with a measurement, scaled by P over
// their number; a worker without one has weight 1 (AWF) or gets FAC2's
// first-batch chunk (AF).  Every chunk is at least min_chunk and at most R.
#pragma once

#include <math.h>
#include <stdint.h>

namespace si {

__host__ __device__ inline int64_t clamp_chunk(double k, int64_t remaining, int64_t min_chunk) {
    if (!(k >= 0.0)) k = 0.0;  // NaN or negative: the smallest chunk
    if (k > 4.0e18) k = 4.0e18;
    int64_t c = (int64_t)ceil(k);
    if (c < min_chunk) c = min_chunk;
    if (c < 1) c = 1;
    return c < remaining ? c : remaining;
}

// WF / AWF: a request of weight w in a batch whose FAC2 chunk is `base`.
__host__ __device__ inline int64_t wf_chunk(double w, int64_t base, int64_t remaining,
                                            int64_t min_chunk) {
    return clamp_chunk(w * (double)base, remaining, min_chunk);
}

// AWF: the weight of a worker of rate `rate` when the n_meas measured
// workers' rates sum to rate_sum (P workers in all).
__host__ __device__ inline double awf_weight(double rate, double rate_sum, int n_meas, int P) {
    if (!(rate > 0.0) || !(rate_sum > 0.0) || n_meas <= 0) return 1.0;
    return (double)P * rate / (rate_sum * (double)P / (double)n_meas);
}

// AF: (D, T) from the sums over the n_meas measured workers of
// sigma^2 / mu and 1 / mu, scaled to P workers.
__host__ __device__ inline void af_terms(double var_over_mu_sum, double inv_mu_sum, int n_meas,
                                         int P, double* D, double* T) {
    const double scale = (double)P / (double)n_meas;
    *D = var_over_mu_sum * scale;
    *T = 1.0 / (inv_mu_sum * scale);
}

__host__ __device__ inline int64_t af_chunk(double D, double T, int64_t remaining, double mu,
                                            int64_t min_chunk) {
    const double R = (double)remaining;
    const double k = (D + 2.0 * T * R - sqrt(D * D + 4.0 * D * T * R)) / (2.0 * mu);
    return clamp_chunk(k, remaining, min_chunk);
}

}  // namespace si
