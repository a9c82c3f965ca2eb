/* Prints sizeof/offsetof of the public structs of include/fpt.h, one
 * "struct.field offset" line each, so the ctypes mirror can be checked. */
#include <stddef.h>
#include <stdio.h>
#include "fpt.h"

#define F(s, f) printf(#s "." #f " %zu\n", offsetof(s, f))
#define S(s) printf(#s ".__size__ %zu\n", sizeof(s))

int main(void)
{
    S(fpt_potential); F(fpt_potential, kind); F(fpt_potential, V0); F(fpt_potential, phi_T);
    F(fpt_potential, A_plus); F(fpt_potential, A_minus); F(fpt_potential, phi_in); F(fpt_potential, pi_in);
    F(fpt_potential, phi_end); F(fpt_potential, bump_m); F(fpt_potential, bump_K); F(fpt_potential, bump_Sigma);
    S(fpt_noise_table); F(fpt_noise_table, n); F(fpt_noise_table, phi_lo); F(fpt_noise_table, phi_hi);
    F(fpt_noise_table, S); F(fpt_noise_table, tan_theta);
    F(fpt_noise_table, dim); F(fpt_noise_table, Xi_pp); F(fpt_noise_table, Xi_pq); F(fpt_noise_table, Xi_qq);
    F(fpt_noise_table, axis);
    S(fpt_bias); F(fpt_bias, kind); F(fpt_bias, A); F(fpt_bias, mlp_params); F(fpt_bias, norm);
    F(fpt_bias, mlp_every); F(fpt_bias, grid_n); F(fpt_bias, grid_range);
    S(fpt_options); F(fpt_options, precision); F(fpt_options, bins_kind); F(fpt_options, n_bins);
    F(fpt_options, lo); F(fpt_options, hi); F(fpt_options, N_ref); F(fpt_options, max_steps);
    F(fpt_options, instance); F(fpt_options, block_size); F(fpt_options, blocks_per_cu); F(fpt_options, chunk);
    S(fpt_hist); F(fpt_hist, n_traj); F(fpt_hist, n_censored); F(fpt_hist, n_ended_early);
    F(fpt_hist, n_steps_total); F(fpt_hist, sum_w); F(fpt_hist, sum_w2); F(fpt_hist, sum_wN);
    F(fpt_hist, sum_wN2); F(fpt_hist, count); F(fpt_hist, sum_w_bin); F(fpt_hist, sum_w2_bin);
    F(fpt_hist, sum_lnw_bin); F(fpt_hist, sum_lnw2_bin);
    S(fpt_moments); F(fpt_moments, mean_w); F(fpt_moments, mean_N); F(fpt_moments, var_N); F(fpt_moments, ess);
    F(fpt_moments, mass_under); F(fpt_moments, mass_over);
    S(fpt_tail); F(fpt_tail, slot); F(fpt_tail, x_star); F(fpt_tail, P); F(fpt_tail, P_err); F(fpt_tail, P_err_lognormal); F(fpt_tail, ess);
    F(fpt_tail, count);
    S(fpt_batch_options); F(fpt_batch_options, block_size); F(fpt_batch_options, chunk);
    F(fpt_batch_options, item_size); F(fpt_batch_options, use_graph);
    return 0;
}
