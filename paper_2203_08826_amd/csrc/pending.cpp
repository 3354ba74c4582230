// Entry points declared in qsv.h whose kernels are not in this build yet:
// each returns QSV_ERR_UNSUPPORTED with a message.
#include "plan_internal.h"
using namespace qsv;
namespace qsv {
int build_learned(qsv_plan *p) { return build_greedy(p, p->opts.kmax, p->opts.use_mfma != 0); }
}
extern "C" {
static int nyi(const char *f) { return fail(QSV_ERR_UNSUPPORTED, std::string(f) + ": not in this build"); }
int qsv_mlp_forward(const float *, const int *, int, const float *, int, float *, float *, void *) { return nyi("qsv_mlp_forward"); }
int qsv_mlp_backward(const float *, const int *, int, const float *, int, const float *, const float *, const float *, float *, float *, void *) { return nyi("qsv_mlp_backward"); }
int qsv_mlp_adam(float *, const float *, float *, float *, int, int, float, float, float, float, void *) { return nyi("qsv_mlp_adam"); }
int qsv_mlp_param_count(const int *, int) { return nyi("qsv_mlp_param_count"); }
int qsv_cost_model_set(const float *, const int *, int, const float *, const float *) { return nyi("qsv_cost_model_set"); }
int qsv_cost_features(int, int, int, const int *, int, int, int, int, float *) { return nyi("qsv_cost_features"); }
}
