#include "ridc2d.h"
#include "ridc_internal.h"

namespace ridc {

struct Plan2D {
  int dummy;
};

int plan2d_validate(const ridc_problem*) { return fail(RIDC_E_UNSUPPORTED, "2D not built yet"); }
size_t plan2d_workspace_bytes(const ridc_problem*) { return 0; }
int plan2d_create(const ridc_problem*, double, double* const*, const int*, const double*,
                  const int64_t*, char*, size_t, hipStream_t, Plan2D**) {
  return fail(RIDC_E_UNSUPPORTED, "2D not built yet");
}
void plan2d_destroy(Plan2D*) {}
int plan2d_arm(Plan2D*, int64_t, hipStream_t) { return RIDC_E_UNSUPPORTED; }
int plan2d_step(Plan2D* const*, int, const int64_t*, hipStream_t) { return RIDC_E_UNSUPPORTED; }
void plan2d_cost(const Plan2D*, double*, double*) {}

}  // namespace ridc
