// Vector-ALU issue-rate probe (libpa_probe.so), a measuring instrument for
// the roofline of the Metropolis pass; not part of the population-annealing
// library.
#pragma once
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Runs `blocks` workgroups of 256 lanes, each lane `iters` rounds of one
   instruction kind (0 three-input xor, 1 32x32->64 multiply-add, 2
   two-input xor, 3 Philox4x32-10 blocks), twice on `stream` (NULL: the null
   stream); *ms receives the event-timed duration of the second run.
   Returns 0, or a negative code on a bad argument (-1), a failed
   allocation (-2) or a failed HIP call (-4). */
int pa_probe_valu(int32_t kind, int32_t blocks, int32_t iters, void* stream,
                  double* ms);

#ifdef __cplusplus
}
#endif
