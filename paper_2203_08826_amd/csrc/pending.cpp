// Entry points declared in qsv.h whose kernels are not in this build yet:
// each returns QSV_ERR_UNSUPPORTED with a message.
#include "qsv_internal.h"
using namespace qsv;
extern "C" {
static int nyi(const char *f) { return fail(QSV_ERR_UNSUPPORTED, std::string(f) + ": not in this build"); }
int qsv_plan_create(int, int, const qsv_gate *, int, const qsv_plan_options *, qsv_plan **) { return nyi("qsv_plan_create"); }
int qsv_plan_stats_get(const qsv_plan *, qsv_plan_stats *) { return nyi("qsv_plan_stats_get"); }
int qsv_plan_blocks(const qsv_plan *, int *, int) { return nyi("qsv_plan_blocks"); }
int qsv_plan_execute(const qsv_plan *, void *, void *) { return nyi("qsv_plan_execute"); }
void qsv_plan_destroy(qsv_plan *) {}
int qsv_apply_block(void *, int, int, const void *, const int *, int, void *) { return nyi("qsv_apply_block"); }
int qsv_run_pass(void *, int, int, const qsv_gate *, int, const int *, int, void *) { return nyi("qsv_run_pass"); }
int qsv_adjoint_grad(void *, void *, int, int, const qsv_gate *, int, double *, void *) { return nyi("qsv_adjoint_grad"); }
int qsv_mlp_forward(const float *, const int *, int, const float *, int, float *, float *, void *) { return nyi("qsv_mlp_forward"); }
int qsv_mlp_backward(const float *, const int *, int, const float *, int, const float *, const float *, const float *, float *, float *, void *) { return nyi("qsv_mlp_backward"); }
int qsv_mlp_adam(float *, const float *, float *, float *, int, int, float, float, float, float, void *) { return nyi("qsv_mlp_adam"); }
int qsv_mlp_param_count(const int *, int) { return nyi("qsv_mlp_param_count"); }
int qsv_cost_model_set(const float *, const int *, int, const float *, const float *) { return nyi("qsv_cost_model_set"); }
int qsv_cost_features(int, int, int, const int *, int, int, int, int, float *) { return nyi("qsv_cost_features"); }
}
