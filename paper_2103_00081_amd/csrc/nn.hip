// Learned preconditioner entry points (network kernels land in this file).
#include "internal.h"

using namespace hts;

namespace hts {
hts_status guard_call(const std::function<void()> &f);
}

extern "C" {

hts_status hts_nn_create(const hts_nn_desc *, hts_nn **out)
{
    if (out) *out = nullptr;
    return guard_call([&] { throw Error(HTS_ERR_UNSUPPORTED, "learned preconditioner not built yet"); });
}
void hts_nn_destroy(hts_nn *) {}
hts_status hts_nn_harvest(hts_nn *, hts_mesh *const *, int32_t, int32_t, double, int32_t)
{
    return guard_call([&] { throw Error(HTS_ERR_UNSUPPORTED, "learned preconditioner not built yet"); });
}
hts_status hts_nn_train(hts_nn *, int32_t, double, int32_t, hts_train_stats *)
{
    return guard_call([&] { throw Error(HTS_ERR_UNSUPPORTED, "learned preconditioner not built yet"); });
}
hts_status hts_nn_save(const hts_nn *, const char *)
{
    return guard_call([&] { throw Error(HTS_ERR_UNSUPPORTED, "learned preconditioner not built yet"); });
}
hts_status hts_nn_load(hts_nn *, const char *)
{
    return guard_call([&] { throw Error(HTS_ERR_UNSUPPORTED, "learned preconditioner not built yet"); });
}

}  // extern "C"
