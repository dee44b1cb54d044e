// F64 instantiation of the element operator (see ax_impl.h).
#include "ax_impl.h"

namespace semx {
template int launch_ax<double>(const Level &, const double *, const double *, const double *, const double *,
                            double *, double, double, const double *, double *, int64_t *, hipStream_t,
                            const int *);
}  // namespace semx
