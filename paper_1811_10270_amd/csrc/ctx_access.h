// Internal accessors of the library context for the solvers built on the
// evaluation entry points (same library, separate translation unit).
#ifndef EHD_CTX_ACCESS_H
#define EHD_CTX_ACCESS_H

#include <hip/hip_runtime.h>

#include "ehdbim.h"

hipStream_t ehd_ctx_stream(const ehd_ctx* ctx);
int ehd_ctx_device(const ehd_ctx* ctx);
int ehd_ctx_ndrops(const ehd_ctx* ctx);
int ehd_ctx_drop_p(const ehd_ctx* ctx, int d);
int ehd_ctx_graph_on(const ehd_ctx* ctx);
// Record `msg` as the context's last error and return `code`.
int ehd_ctx_fail(ehd_ctx* ctx, int code, const char* msg);

#endif
