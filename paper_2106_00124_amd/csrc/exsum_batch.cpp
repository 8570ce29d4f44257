// exsum_batch.cpp -- batched form (placeholder until the batched executor lands).
#include "exsum_internal.hpp"
using namespace exs;
extern "C" {
exs_status exs_batch_create(const exs_job*, int32_t, const char*, exs_batch**) {
    return set_error(EXS_EUNSUPPORTED, "batched form not built yet");
}
exs_status exs_batch_workspace_size(const exs_batch*, size_t*) {
    return set_error(EXS_EUNSUPPORTED, "batched form not built yet");
}
exs_status exs_batch_launch(exs_batch*, void*, size_t, void*) {
    return set_error(EXS_EUNSUPPORTED, "batched form not built yet");
}
exs_status exs_batch_launch_eager(exs_batch*, void*, size_t, void*) {
    return set_error(EXS_EUNSUPPORTED, "batched form not built yet");
}
exs_status exs_batch_info(const exs_batch*, int32_t*, int64_t*) {
    return set_error(EXS_EUNSUPPORTED, "batched form not built yet");
}
void exs_batch_destroy(exs_batch*) {}
exs_status exs_server_create(size_t, int32_t, exs_server**) {
    return set_error(EXS_EUNSUPPORTED, "serving form not built yet");
}
exs_status exs_server_submit(exs_server*, const exs_job*, uint64_t*) {
    return set_error(EXS_EUNSUPPORTED, "serving form not built yet");
}
exs_status exs_server_poll(exs_server*, uint64_t, const void**, const void**, double*) {
    return set_error(EXS_EUNSUPPORTED, "serving form not built yet");
}
exs_status exs_server_drain(exs_server*) {
    return set_error(EXS_EUNSUPPORTED, "serving form not built yet");
}
exs_status exs_server_release(exs_server*, uint64_t) {
    return set_error(EXS_EUNSUPPORTED, "serving form not built yet");
}
exs_status exs_server_stats(exs_server*, double*, double*, double*, double*, int64_t*, int64_t*,
                            int64_t*) {
    return set_error(EXS_EUNSUPPORTED, "serving form not built yet");
}
void exs_server_destroy(exs_server*) {}
}
