// Instantiations of the per-stage task kernel: float32 accumulation,
// dtype masks 0 ... 15 (one translation unit each, so they compile in parallel).
#include "hm_stream.h"

namespace hm {
namespace dev {

extern const TaskKernel kTasks32lo[16];
const TaskKernel kTasks32lo[16] = {
    &k_owner_tasks<false, 0>,
    &k_owner_tasks<false, 1>,
    &k_owner_tasks<false, 2>,
    &k_owner_tasks<false, 3>,
    &k_owner_tasks<false, 4>,
    &k_owner_tasks<false, 5>,
    &k_owner_tasks<false, 6>,
    &k_owner_tasks<false, 7>,
    &k_owner_tasks<false, 8>,
    &k_owner_tasks<false, 9>,
    &k_owner_tasks<false, 10>,
    &k_owner_tasks<false, 11>,
    &k_owner_tasks<false, 12>,
    &k_owner_tasks<false, 13>,
    &k_owner_tasks<false, 14>,
    &k_owner_tasks<false, 15>,
};

}  // namespace dev
}  // namespace hm
