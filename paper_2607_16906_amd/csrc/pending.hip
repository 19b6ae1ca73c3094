// Entry points whose kernels live in later translation units of the build.
#include "common.h"

using namespace hz;

extern "C" size_t no_train_workspace_size(const no_net*, const hz_problem*, int, no_prec) { return 0; }
extern "C" int no_loss_backward(const no_net*, int, const hz_problem* const*, const void*, int, no_prec, float*,
                                float*, float*, void*, size_t, void*) {
    set_error("no_loss_backward: not built");
    return HZ_ERR_ARG;
}
extern "C" size_t no_adam_workspace_size(const no_net*) { return 0; }
extern "C" int no_adam_step(no_net*, float*, float*, float*, const float*, int, float, float, float, float, float,
                            void*, size_t, void*) {
    set_error("no_adam_step: not built");
    return HZ_ERR_ARG;
}
extern "C" size_t fgmres_batched_workspace_size(int, const hz_problem* const*, const no_net*, const hz_opts*) {
    return 0;
}
extern "C" int fgmres_solve_batched(int, const hz_problem* const*, const no_net*, const hz_opts*,
                                    const void* const*, void* const*, void*, size_t, hz_info*, void*) {
    set_error("fgmres_solve_batched: not built");
    return HZ_ERR_ARG;
}
