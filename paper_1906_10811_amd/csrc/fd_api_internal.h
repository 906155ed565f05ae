// fd_api_internal.h -- helpers shared by the host-side translation units of
// libfd (error state, descriptor validation, layout).  Not part of the ABI.
#pragma once

#include "../../include/fd.h"
#include "fd_internal.h"

// Record a thread-local error message and return `code`.
int fdi_fail(int code, const char *fmt, ...);
// Validate a grid description (sets the error message on failure).
bool fdi_check_desc(const fd_grid_desc *d);
// Device layout of one field of a grid.
fd::Layout fdi_layout(const fd_grid_desc *d);
// Maximal-order central second-derivative weights c_0..c_r of radius r.
void fdi_second_derivative_weights(int r, double *c);

// Chunked forward modelling, used by fd_forward, fd_gradient and the server.
int fdi_forward_prepare(fd_grid *g, const fd_shot *sh, int nt, double dt, hipStream_t s);
int fdi_forward_zero_state(fd_grid *g, hipStream_t s);
int fdi_forward_steps(fd_grid *g, const fd_shot *sh, int nt, int n0, int n1, float *rec_out,
                      void **ckpt, int K, hipStream_t s);
int fdi_grid_device(const fd_grid *g);

#include <vector>
// Binomial checkpoint schedule (fd_checkpoint.cpp).
int fdi_checkpoint_plan(int nt, int slots, std::vector<fd_ckpt_action> *actions, long long *fwd);
