/* Prints sizeof / offsetof of the C ABI structs of include/mgp.h, so the
 * test-suite can check the Python binding's ctypes mirrors against them. */
#include <stddef.h>
#include <stdio.h>

#include "mgp.h"

#define F(T, m) printf("\"%s.%s\": %zu,\n", #T, #m, offsetof(T, m))
#define S(T) printf("\"%s\": %zu,\n", #T, sizeof(T))

int main(void)
{
    printf("{\n");
    S(mgp_params); F(mgp_params, variant); F(mgp_params, B); F(mgp_params, epsilon); F(mgp_params, seed);
    F(mgp_params, stream_id); F(mgp_params, partition_bytes); F(mgp_params, b_max); F(mgp_params, segment);
    S(mgp_stats); F(mgp_stats, w_sum); F(mgp_stats, ratio); F(mgp_stats, b_raw); F(mgp_stats, w_max); F(mgp_stats, B);
    F(mgp_stats, clamped); F(mgp_stats, status); F(mgp_stats, n); F(mgp_stats, tag);
    S(mgp_filter_desc); F(mgp_filter_desc, w_dev); F(mgp_filter_desc, n); F(mgp_filter_desc, B);
    F(mgp_filter_desc, epsilon); F(mgp_filter_desc, seed); F(mgp_filter_desc, stream_id); F(mgp_filter_desc, reserved);
    F(mgp_filter_desc, ancestors_dev); F(mgp_filter_desc, states_dev); F(mgp_filter_desc, out_states_dev);
    F(mgp_filter_desc, stats_dev);
    S(mgp_batch_config); F(mgp_batch_config, variant); F(mgp_batch_config, d); F(mgp_batch_config, partition_bytes);
    F(mgp_batch_config, b_max); F(mgp_batch_config, block_threads); F(mgp_batch_config, particles_per_thread);
    F(mgp_batch_config, schedule); F(mgp_batch_config, use_graph); F(mgp_batch_config, tune_cache);
    S(mgp_batch_info); F(mgp_batch_info, filters); F(mgp_batch_info, block_threads);
    F(mgp_batch_info, particles_per_thread); F(mgp_batch_info, schedule); F(mgp_batch_info, from_cache);
    F(mgp_batch_info, xcds); F(mgp_batch_info, particles); F(mgp_batch_info, tiles); F(mgp_batch_info, device_bytes);
    F(mgp_batch_info, est_particle_steps); F(mgp_batch_info, grid);
    S(mgp_server_config); F(mgp_server_config, variant); F(mgp_server_config, d);
    F(mgp_server_config, partition_bytes); F(mgp_server_config, b_max); F(mgp_server_config, hbm_budget);
    F(mgp_server_config, streams); F(mgp_server_config, max_batch); F(mgp_server_config, max_batch_particles);
    F(mgp_server_config, max_n); F(mgp_server_config, simulate); F(mgp_server_config, sim_us_fixed);
    F(mgp_server_config, sim_ns_per_particle); F(mgp_server_config, sim_fail_every); F(mgp_server_config, reserved);
    S(mgp_request); F(mgp_request, w_dev); F(mgp_request, n); F(mgp_request, B); F(mgp_request, epsilon);
    F(mgp_request, seed); F(mgp_request, stream_id); F(mgp_request, reserved); F(mgp_request, states_dev);
    S(mgp_request_result); F(mgp_request_result, state); F(mgp_request_result, status); F(mgp_request_result, B);
    F(mgp_request_result, n); F(mgp_request_result, ancestors_dev); F(mgp_request_result, out_states_dev);
    F(mgp_request_result, t_submit); F(mgp_request_result, t_admit); F(mgp_request_result, t_dispatch);
    F(mgp_request_result, t_done);
    S(mgp_server_stats); F(mgp_server_stats, submitted); F(mgp_server_stats, admitted);
    F(mgp_server_stats, completed); F(mgp_server_stats, failed); F(mgp_server_stats, cancelled);
    F(mgp_server_stats, released); F(mgp_server_stats, micro_batches); F(mgp_server_stats, queued);
    F(mgp_server_stats, in_flight); F(mgp_server_stats, pool_bytes); F(mgp_server_stats, pool_in_use);
    F(mgp_server_stats, pool_peak); F(mgp_server_stats, max_concurrent_batches);
    S(mgp_sir_config); F(mgp_sir_config, variant); F(mgp_sir_config, runs); F(mgp_sir_config, n);
    F(mgp_sir_config, steps); F(mgp_sir_config, B); F(mgp_sir_config, partition_bytes); F(mgp_sir_config, epsilon);
    F(mgp_sir_config, seed); F(mgp_sir_config, b_max); F(mgp_sir_config, use_graph);
    F(mgp_sir_config, block_threads); F(mgp_sir_config, particles_per_thread); F(mgp_sir_config, reserved);
    F(mgp_sir_config, reserved2);
    S(mgp_sir_buffers); F(mgp_sir_buffers, x_dev); F(mgp_sir_buffers, w_dev); F(mgp_sir_buffers, xbar_dev);
    F(mgp_sir_buffers, ancestors_dev); F(mgp_sir_buffers, ld); F(mgp_sir_buffers, device_bytes);
    F(mgp_sir_buffers, accept_grid); F(mgp_sir_buffers, block_threads); F(mgp_sir_buffers, particles_per_thread);
    printf("\"end\": 0\n}\n");
    return 0;
}
