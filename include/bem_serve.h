/*
 * bem_serve.h -- continuous-batching request server over the solve path of
 * bem.h: many independent scattering problems (each a bem_desc with its own
 * geometry, size and wavenumbers, and its own incident angles) arrive over
 * time and are solved concurrently on one GPU.
 *
 * Each request runs the whole path of bem.h (geometry tables, assembly of the
 * Calderon-ordered Burton-Miller matrix, plane-wave right-hand sides of
 * Sec. 7, restarted GMRES, far field) in the precision the server was created
 * with (bem_prec): BEM_F64; BEM_F32 (FP32 matrix and products inside FP64
 * residual refinement); BEM_MIXED (FP32 products, refinement residuals with
 * the FP64 matrix).
 *
 * Scheduling:
 *   - the server owns `slots` worker threads, each with its own non-blocking
 *     HIP stream at the default priority; a request runs entirely on one
 *     slot's stream, so the device work of up to `slots` requests overlaps
 *     (up to slots * fuse with fused batches, bem_server_opts.fuse);
 *   - every request's device buffers (geometry tables, matrix, solver
 *     workspace, right-hand sides, solution, far field) are one contiguous
 *     block of the caller-owned arena; the block is the request's footprint
 *     (bem_server_footprint), held from admission to completion;
 *   - admission: as soon as a slot is free, the oldest waiting request whose
 *     footprint fits a free range of the arena is admitted; a request that
 *     has been passed over 2 * slots times by younger ones admits no younger
 *     one before itself (no starvation);
 *   - results do not depend on what else runs: every reduction inside the
 *     path has a fixed order, and every request's products use the launch
 *     shapes of a copy of the tuned-shape table (and of the BEM_MV_CFG
 *     overrides) taken by bem_server_create, so a request gives bit-identical
 *     output alone or in the mix, whatever bem_tune / bem_tune_import calls
 *     the process makes meanwhile.
 *
 * The server allocates no device memory.  Host memory: request copies and
 * one pinned flag buffer per slot (fuse parts of it with fused batches).
 */
#ifndef BEM_SERVE_H
#define BEM_SERVE_H

#include "bem.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bem_server bem_server;

typedef struct {
    int slots;              /* requests in flight at once, 1..16                        */
    int device;             /* HIP device of the arena                                 */
    void *arena_dev;        /* caller-owned device memory, 256-byte aligned             */
    size_t arena_bytes;     /* its size; kept until bem_server_destroy returns         */
    int prec;               /* bem_prec of every request                               */
    bem_solve_opts solve;   /* GMRES options of every request (bem_solve)              */
    int ndir;               /* far-field directions reported per right-hand side, >= 1 */
    const double *dirs;     /* [ndir] direction angles (host; copied at create)        */
    int fuse;               /* 0 or 1: a slot runs one request at a time; 2..8: a slot
                               that admits a request also admits up to fuse - 1 more
                               waiting ones that fit and solves them together
                               (bem_solve_batch: restart cycles in step, one fused set
                               of orthogonalisation launches per Krylov step for all
                               of them); their results are posted when the batch ends */
} bem_server_opts;

/* Outcome of one request. */
typedef struct {
    long long id;           /* the id bem_server_submit returned                        */
    int status;             /* bem_status of the request (BEM_E_NOCONV: far field of the last iterate) */
    int n;                  /* system order                                            */
    int nrhs;               /* right-hand sides (incident angles)                      */
    int iters_max;          /* largest GMRES iteration count over the right-hand sides */
    int refine_max;         /* largest restart / refinement count                      */
    double rel_residual_max;/* largest final relative residual                        */
    size_t footprint;       /* arena bytes the request held                           */
    double t_submit;        /* seconds since bem_server_create: submission,            */
    double t_admit;         /*   admission to a slot,                                  */
    double t_done;          /*   far field copied to the caller's host buffer          */
    char message[160];      /* bem_last_error text when status != BEM_OK               */
} bem_server_result;

/* Validate the options, copy the directions, create the slot streams and
 * threads.  BEM_E_ARG: slots outside 1..16, a null or unaligned arena, ndir < 1,
 * prec not a bem_prec, restart < 1, fuse outside 0..8.  BEM_E_DEVICE: stream
 * or thread set-up failed.                                                   */
bem_status bem_server_create(const bem_server_opts *opts, bem_server **out);

/* Arena bytes a request would hold (plus bem_create's validation errors). */
bem_status bem_server_footprint(const bem_server *s, const bem_desc *desc, int nrhs, size_t *bytes);

/* Queue one request: desc and angles[nrhs] are copied (host pointers, read
 * during the call); the far field, nrhs x ndir complex128 with the directions
 * fastest (F[r * ndir + d]), is written to farfield_host, a caller-owned host
 * buffer that must stay valid until the request's result has been returned by
 * bem_server_poll.  Errors of the description (bem_create) are returned here
 * and queue nothing; BEM_E_NOMEM: the footprint exceeds the whole arena;
 * BEM_E_ARG: nrhs outside 1..256 or null pointers; BEM_E_STATE: the server is
 * shutting down.                                                             */
bem_status bem_server_submit(bem_server *s, const bem_desc *desc, int nrhs, const double *angles,
                             bem_z *farfield_host, long long *id);

/* Move up to max finished results to out[0..*count) in completion order,
 * waiting up to wait_ms milliseconds (0: do not wait, < 0: until at least one
 * is available or nothing is pending).                                       */
bem_status bem_server_poll(bem_server *s, bem_server_result *out, int max, int *count, int wait_ms);

/* Counters: requests submitted, waiting, running, finished-but-unpolled;
 * arena bytes in use now and the largest in use at any time.               */
typedef struct {
    long long submitted, waiting, running, unpolled;
    size_t arena_in_use, arena_high_water;
} bem_server_stats;
bem_status bem_server_stat(bem_server *s, bem_server_stats *out);

/* Finish every queued and running request, then stop and join the threads,
 * destroy the streams and free the server's host memory.  Results not polled
 * are dropped.                                                               */
bem_status bem_server_destroy(bem_server *s);

#ifdef __cplusplus
}
#endif
#endif /* BEM_SERVE_H */
