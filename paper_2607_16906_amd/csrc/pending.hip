// Entry points whose kernels live in later translation units of the build.
#include "common.h"

using namespace hz;

extern "C" size_t fgmres_batched_workspace_size(int, const hz_problem* const*, const no_net*, const hz_opts*) {
    return 0;
}
extern "C" int fgmres_solve_batched(int, const hz_problem* const*, const no_net*, const hz_opts*,
                                    const void* const*, void* const*, void*, size_t, hz_info*, void*) {
    set_error("fgmres_solve_batched: not built");
    return HZ_ERR_ARG;
}
