// backward.hip -- placeholder launcher (adjoint kernel not built yet).
#include "vd_internal.h"
void vd_launch_backward(const vd_cells_s *, const GridView &, const double *, const double *, const double *,
                        double *, double *, hipStream_t) {}
