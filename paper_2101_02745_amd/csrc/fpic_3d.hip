// 3D periodic boxes.
#include "fpic_3d.h"
#include "fpic_internal.h"

namespace fpic3d {

struct Ctx3D {
    int unused;
};

static int no3d() { return fpic::fail(FPIC_EUNSUPPORTED, "3D boxes are not implemented yet"); }

int workspace_bytes(const fpic_config &, const fpic_tuning *, size_t *) { return no3d(); }
int create(const fpic_config &, const fpic_tuning *, void *, size_t, fpic_stream, Ctx3D **) { return no3d(); }
int set_state(Ctx3D *, const double *, int64_t) { return no3d(); }
int get_state(Ctx3D *, double *) { return no3d(); }
int step(Ctx3D *, int64_t) { return no3d(); }
int moments(Ctx3D *, double *) { return no3d(); }
int flavor_totals(Ctx3D *, double *) { return no3d(); }
int check(Ctx3D *, double *) { return no3d(); }
int get_step(Ctx3D *, int64_t *) { return no3d(); }
int sync(Ctx3D *) { return no3d(); }
int profile(Ctx3D *, int, double *) { return no3d(); }
void destroy(Ctx3D *c) { delete c; }
int autotune(const fpic_config &, void *, size_t, fpic_stream, fpic_tuning *, double *) { return no3d(); }

}  // namespace fpic3d
