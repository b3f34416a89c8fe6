// Instantiations of the per-stage task kernel: float32 accumulation,
// dtype masks 16 ... 31 (one translation unit each, so they compile in parallel).
#include "hm_stream.h"

namespace hm {
namespace dev {

extern const TaskKernel kTasks32hi[16];
const TaskKernel kTasks32hi[16] = {
    &k_owner_tasks<false, 16>,
    &k_owner_tasks<false, 17>,
    &k_owner_tasks<false, 18>,
    &k_owner_tasks<false, 19>,
    &k_owner_tasks<false, 20>,
    &k_owner_tasks<false, 21>,
    &k_owner_tasks<false, 22>,
    &k_owner_tasks<false, 23>,
    &k_owner_tasks<false, 24>,
    &k_owner_tasks<false, 25>,
    &k_owner_tasks<false, 26>,
    &k_owner_tasks<false, 27>,
    &k_owner_tasks<false, 28>,
    &k_owner_tasks<false, 29>,
    &k_owner_tasks<false, 30>,
    &k_owner_tasks<false, 31>,
};

}  // namespace dev
}  // namespace hm
