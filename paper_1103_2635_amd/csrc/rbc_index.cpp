// rbc_index.cpp -- Random Ball Cover build and search (Sec. 4 and Sec. 5).
#include <hip/hip_runtime.h>

#include "../../include/rbc.h"
#include "rbc_host.h"

using namespace rbc;

extern "C" {

int rbc_build(const float*, int64_t, int64_t, int32_t, const rbc_build_params*, void*,
              rbc_index** out) {
    if (out) *out = nullptr;
    return set_err(RBC_EUNSUPPORTED, "rbc_build is not implemented yet");
}
int rbc_search_workspace_size(const rbc_index*, int64_t, int32_t, const rbc_search_opts*,
                              size_t*) {
    return set_err(RBC_EUNSUPPORTED, "rbc_search is not implemented yet");
}
int rbc_search(const rbc_index*, const float*, int64_t, int64_t, int32_t, const rbc_search_opts*,
               int64_t*, float*, void*, size_t, void*) {
    return set_err(RBC_EUNSUPPORTED, "rbc_search is not implemented yet");
}
int rbc_index_info(const rbc_index*, int64_t*, int32_t*, int64_t*, int32_t*, int32_t*, size_t*) {
    return set_err(RBC_EUNSUPPORTED, "not implemented yet");
}
int rbc_index_export(const rbc_index*, int64_t*, double*, int64_t*, int64_t*) {
    return set_err(RBC_EUNSUPPORTED, "not implemented yet");
}
void rbc_free(rbc_index*) {}

}  // extern "C"
