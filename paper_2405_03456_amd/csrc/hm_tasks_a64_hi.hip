// Instantiations of the per-stage task kernel: float64 accumulation,
// dtype masks 16 ... 31 (one translation unit each, so they compile in parallel).
#include "hm_stream.h"

namespace hm {
namespace dev {

extern const TaskKernel kTasks64hi[16];
const TaskKernel kTasks64hi[16] = {
    &k_owner_tasks<true, 16>,
    &k_owner_tasks<true, 17>,
    &k_owner_tasks<true, 18>,
    &k_owner_tasks<true, 19>,
    &k_owner_tasks<true, 20>,
    &k_owner_tasks<true, 21>,
    &k_owner_tasks<true, 22>,
    &k_owner_tasks<true, 23>,
    &k_owner_tasks<true, 24>,
    &k_owner_tasks<true, 25>,
    &k_owner_tasks<true, 26>,
    &k_owner_tasks<true, 27>,
    &k_owner_tasks<true, 28>,
    &k_owner_tasks<true, 29>,
    &k_owner_tasks<true, 30>,
    &k_owner_tasks<true, 31>,
};

}  // namespace dev
}  // namespace hm
