// 3D periodic boxes (fpic_3d.hip): same C ABI as the 1D path.
#pragma once

#include <cstdint>

#include "fpic.h"

namespace fpic3d {

struct Ctx3D;

int workspace_bytes(const fpic_config &cfg, const fpic_tuning *tune, size_t *bytes);
int create(const fpic_config &cfg, const fpic_tuning *tune, void *ws, size_t bytes,
           fpic_stream stream, Ctx3D **out);
int set_state(Ctx3D *c, const double *state, int64_t step0);
int get_state(Ctx3D *c, double *state);
int step(Ctx3D *c, int64_t nsteps);
int moments(Ctx3D *c, double *out);
int flavor_totals(Ctx3D *c, double *out);
int check(Ctx3D *c, double r[3]);
int get_step(Ctx3D *c, int64_t *step);
int sync(Ctx3D *c);
int profile(Ctx3D *c, int nsteps, double *ms);
void destroy(Ctx3D *c);
int autotune(const fpic_config &cfg, void *ws, size_t bytes, fpic_stream stream,
             fpic_tuning *best, double *ms_per_step);
// the context's stream, device scratch (>= 4000 doubles), pinned host
// staging (>= 64 doubles) and cell count, for diagnostics
void diag_buffers(Ctx3D *c, void **stream, double **scratch, double **hbuf, int64_t *ncell);

}  // namespace fpic3d
