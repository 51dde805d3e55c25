/*
 * mpdd_testing.h -- test hooks of libmpdd's request server (mpdd.h).
 *
 * For tests of the server's scheduling and failure paths that must run
 * without a GPU or must force a failure from the host.  Not part of the
 * product interface: production callers pass flags = 0 to
 * mpdd_server_create and leave mpdd_request.inject at 0.  The hooks live in
 * the same library (one build), and are declared here so that mpdd.h shows
 * only the product calls.
 */
#ifndef MPDD_TESTING_H
#define MPDD_TESTING_H

#include "mpdd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* mpdd_server_create flag: no GPU is used; each group completes after a
 * simulated time (set by mpdd_server_set_fake_rate); h may be NULL. */
#define MPDD_SERVER_FAKE_DEVICE 1

/* mpdd_request.inject values: a forced failure of that request only. */
#define MPDD_INJECT_NONE 0
#define MPDD_INJECT_DEVICE_ERROR 1     /* its launch reports a device error (MPDD_ERR_HIP) */
#define MPDD_INJECT_ALLOC_FAILURE 2    /* it fails admission as if out of memory */

/* Fake-device servers only: simulated throughput (dd-flops per second) and
 * per-group latency (seconds).  Returns 0 or MPDD_ERR_ARG. */
int mpdd_server_set_fake_rate(mpdd_server s, double dd_flops_per_s, double group_latency_s);

#ifdef __cplusplus
}
#endif

#endif /* MPDD_TESTING_H */
