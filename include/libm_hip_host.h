/* libm_hip_host: the host (CPU) build of libm_hip's evaluators in their
 * bit-consistent form.
 *
 * The paper's library offers functions whose results are bit-wise the same
 * on every platform (Section 3.3).  libm_hip_host_eval computes, on the host,
 * exactly the bits that libm_hip_consistent_eval (libm_hip.h) computes on the
 * GPU: both are the same evaluator source with every primitive an IEEE
 * operation (correctly rounded division and square root instead of the
 * hardware estimates, a seed for x^(-1/3) from fused multiply-adds only).
 * The accuracy bounds are those of the default entry points (1.0 ULP for
 * u10, 3.5 ULP for u35, exact for fmod/remainder), and so are the special
 * values.
 *
 * Arguments: fn, v as for libm_hip_eval; t is LIBM_HIP_F64 or LIBM_HIP_F32;
 * a, b (NULL for unary functions), out are HOST arrays of n elements of that
 * type, owned by the caller; out may equal a or b.  The call is synchronous
 * and single-threaded (element by element) and keeps no state.
 * Returns LIBM_HIP_OK; LIBM_HIP_ERR_INVALID for a NULL array with n > 0;
 * LIBM_HIP_ERR_UNSUPPORTED for another dtype or a (fn, v) the library does
 * not serve.  Requires round-to-nearest-even (the default mode).
 */
#ifndef LIBM_HIP_HOST_H
#define LIBM_HIP_HOST_H

#include "libm_hip.h"

#ifdef __cplusplus
extern "C" {
#endif

libm_hip_status libm_hip_host_eval(libm_hip_fn fn, libm_hip_variant v, libm_hip_dtype t,
                                   const void* a, const void* b, void* out, size_t n);

/* Instrumented exact remainder (Section 5, "FP Remainder", Algorithm 1):
 * out[i] = fmod(x[i], y[i]) exactly as libm_hip_host_eval computes it, and
 * steps[i] = the number of long-division digit steps the element took (0
 * when |x| < |y| or for the special cases).  The paper's worked example
 * (1e40 mod 0.75) takes 3 steps; in general about ceil(log2(|x/y|) / 52)
 * (binary32: / 23), plus at most one more for the exponent-scaled digits of
 * quotients beyond the format's range.  t is LIBM_HIP_F64 or LIBM_HIP_F32;
 * x, y, out are host arrays of that type, steps an int32 array, all of n
 * elements and caller-owned.  Returns LIBM_HIP_OK, LIBM_HIP_ERR_INVALID for
 * a NULL array with n > 0, LIBM_HIP_ERR_UNSUPPORTED for another dtype. */
libm_hip_status libm_hip_host_fmod_steps(libm_hip_dtype t, const void* x, const void* y,
                                         void* out, int32_t* steps, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* LIBM_HIP_HOST_H */
