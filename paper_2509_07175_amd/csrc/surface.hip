// surface.hip -- placeholder launcher (restricted VD kernel not built yet).
#include "vd_internal.h"
void vd_launch_surface(const GridView &, const DomainView &, const CellsDev &, hipStream_t) {}
