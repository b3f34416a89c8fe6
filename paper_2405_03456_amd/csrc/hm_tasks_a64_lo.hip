// Instantiations of the per-stage task kernel: float64 accumulation,
// dtype masks 0 ... 15 (one translation unit each, so they compile in parallel).
#include "hm_stream.h"

namespace hm {
namespace dev {

extern const TaskKernel kTasks64lo[16];
const TaskKernel kTasks64lo[16] = {
    &k_owner_tasks<true, 0>,
    &k_owner_tasks<true, 1>,
    &k_owner_tasks<true, 2>,
    &k_owner_tasks<true, 3>,
    &k_owner_tasks<true, 4>,
    &k_owner_tasks<true, 5>,
    &k_owner_tasks<true, 6>,
    &k_owner_tasks<true, 7>,
    &k_owner_tasks<true, 8>,
    &k_owner_tasks<true, 9>,
    &k_owner_tasks<true, 10>,
    &k_owner_tasks<true, 11>,
    &k_owner_tasks<true, 12>,
    &k_owner_tasks<true, 13>,
    &k_owner_tasks<true, 14>,
    &k_owner_tasks<true, 15>,
};

}  // namespace dev
}  // namespace hm
