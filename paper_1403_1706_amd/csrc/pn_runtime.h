// Internal interface between the C ABI's mapping path (pn_api.hip) and the
// serving loop (pn_serve.hip).
#pragma once

#include "../../include/peanut.h"
#include "pn_internal.h"

namespace pnrt {

int ctx_device(const pn_ctx *c);
int ref_device(const pn_ref *r);

// Filtration, validation and canonicalisation of a built index with
// per-read k on the device (d_k, one byte per read).  The sorted hits stay
// in workspace buffers of the context, valid until its next mapping call:
// all hits (if want_all) and the best stratum (if want_best).
int map_to_workspace(pn_ctx *c, const pn_ref *ref, const pn_index *x, const uint8_t *d_k,
                     bool want_all, bool want_best, const pn_hit **d_all, uint64_t *n_all,
                     const pn_hit **d_best, uint64_t *n_best, hipStream_t st);

}  // namespace pnrt
