/*
 * oem_debug.h - test hooks of liboem.  Host functions that expose the
 * index arithmetic of the kernels so that it can be checked on a machine
 * without a GPU.  Not part of the method's interface (include/oem.h).
 */
#ifndef OEM_DEBUG_H
#define OEM_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The four column indices that a Gram-pass loader thread reads from one row
 * of p elements for its group of columns col .. col + 3 (col a multiple of 4,
 * any value up to the padded panel width).  vec_ok: whether 16-byte loads
 * are allowed (X suitably aligned).  cols: host array of 4.  Returns 1 when
 * the group is read with one 16-byte load, 0 when column by column,
 * OEM_E_INVAL on bad arguments.  Every index written is in [0, p). */
int oem_debug_gram_load_columns(int32_t p, int32_t col, int32_t vec_ok, int32_t *cols);

/* Measurement hook: the Lanczos step counts of the handle's derived
 * problems (q = 0 full data, q = 1 + k training rows of fold k) from the
 * last oem_fit_path / oem_cv, copied into steps (host, at most nq entries;
 * negative: the Gershgorin fallback was used).  Returns the number of
 * problems, or OEM_E_STATE when nothing has been derived yet. */
int oem_debug_lanczos_steps(void *handle, int32_t *steps, int32_t nq);

#ifdef __cplusplus
}
#endif
#endif
