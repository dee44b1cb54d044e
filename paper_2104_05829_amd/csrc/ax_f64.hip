// F64 instantiation of the element operator (see ax_impl.h).
#include "ax_impl.h"

namespace semx {
template int launch_ax<double>(const Level &, const double *, const double *, const double *, const double *,
                            double *, double, double, const double *, double *, int64_t *, hipStream_t,
                            const int *);
template int launch_ax_multi<double>(const Level &, const double *, const double *, const double *, const double *,
                                 int64_t, double *, int64_t, const VSet &, double, double, const double *,
                                 double *, int64_t, int64_t *, hipStream_t, const int *, int);
}  // namespace semx
