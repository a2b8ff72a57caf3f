// placeholder replaced by the rank-predictor implementation
#include "hmat_internal.h"
using namespace hm;
extern "C" {
void hmat_train_opts_default(hmat_train_opts* o) { if (o) *o = hmat_train_opts{}; }
#define NOTYET { set_last_error("rank model not built yet"); return HMAT_ERR_INTERNAL; }
hmat_status hmat_rank_model_create(uint64_t, hmat_rank_model*) NOTYET
hmat_status hmat_rank_model_destroy(hmat_rank_model) NOTYET
hmat_status hmat_rank_model_train(hmat_rank_model, const float*, const float*, int64_t, const hmat_train_opts*) NOTYET
hmat_status hmat_rank_model_predict(hmat_rank_model, const float*, int64_t, float*, void*) NOTYET
hmat_status hmat_rank_model_get(hmat_rank_model, float*, int64_t*) NOTYET
hmat_status hmat_rank_model_set(hmat_rank_model, const float*, int64_t) NOTYET
hmat_status hmat_rank_model_grad(hmat_rank_model, const float*, const float*, int64_t, float*, float*) NOTYET
hmat_status hmat_product_features(hmat, float*, float*, int64_t*) NOTYET
}
