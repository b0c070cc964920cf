#include "feint.h"
extern "C" {
feint_status feint_mixed_plan_create(int64_t, feint_form, feint_mixed_plan **) { return FEINT_ERR_UNSUPPORTED_FORM; }
feint_status feint_mixed_bucket(feint_mixed_plan *, const int8_t *, int64_t, int64_t *, int64_t *, uint32_t *, void *) { return FEINT_ERR_UNSUPPORTED_FORM; }
feint_status feint_integrate_mixed(feint_mixed_plan *, const feint_elements *, void *, void *, const int64_t *, const int64_t *, uint32_t *, void *) { return FEINT_ERR_UNSUPPORTED_FORM; }
feint_status feint_mixed_graph_capture(feint_mixed_plan *, const feint_elements *, const int8_t *, void *, void *, int64_t *, int64_t *, uint32_t *, void *) { return FEINT_ERR_UNSUPPORTED_FORM; }
feint_status feint_mixed_graph_launch(feint_mixed_plan *, void *) { return FEINT_ERR_UNSUPPORTED_FORM; }
void feint_mixed_plan_destroy(feint_mixed_plan *) {}
}
