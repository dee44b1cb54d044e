// F32 instantiation of the element operator (see ax_impl.h).
#include "ax_impl.h"

namespace semx {
template int launch_ax<float>(const Level &, const float *, const float *, const float *, const float *,
                            float *, double, double, const float *, double *, int64_t *, hipStream_t,
                            const int *);
template int launch_ax_multi<float>(const Level &, const float *, const float *, const float *, const float *,
                                 int64_t, float *, int64_t, const VSet &, double, double, const float *,
                                 double *, int64_t, int64_t *, hipStream_t, const int *, int);
}  // namespace semx
