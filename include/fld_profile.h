/*
 * fld_profile.h -- per-kernel timing hook of the FLD library.
 *
 * For measuring one kernel's average launch duration inside a running
 * workload: while a kernel id is selected, every launch of that kernel is
 * bracketed by two hipEvents recorded on the stream it is launched on, and
 * the library accumulates the elapsed times.  Other kernels are untouched.
 * Host-side state is process-global and not thread-safe: select, run, read
 * from one thread.
 */
#ifndef FLD_PROFILE_H_
#define FLD_PROFILE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of kernel ids; names via fld_profile_kernel_name. */
int32_t fld_profile_num_kernels(void);

/* Stable name of kernel id k (NULL if out of range). */
const char *fld_profile_kernel_name(int32_t k);

/* Select kernel id k for timing (-1: none; -2: every kernel, for a survey
 * run) and clear the accumulators.  Returns 0, or -1 for a bad id. */
int32_t fld_profile_select(int32_t k);

/* Synchronise the recorded events and report, for kernel id k, the summed
 * duration in milliseconds and the number of timed launches.  Returns 0, or
 * -1 for a bad id / HIP error. */
int32_t fld_profile_read(int32_t k, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* FLD_PROFILE_H_ */
