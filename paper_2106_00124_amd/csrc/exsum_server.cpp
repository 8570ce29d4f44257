// exsum_server.cpp -- serving form (placeholder until the serving runtime lands).
#include "exsum_internal.hpp"
using namespace exs;
extern "C" {
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
