// Instantiations of the per-stage task kernel for stages holding the byte-
// aligned codecs of Sec. 4.1: float32 accumulation, one codec with FP64
// (kCodecMasks; one translation unit per group, so they compile in parallel).
#include "hm_stream.h"

namespace hm {
namespace dev {

extern const TaskKernel kTasksCodec32Single[11];
const TaskKernel kTasksCodec32Single[11] = {
    &k_owner_tasks<false, kCodecMasks[0]>,
    &k_owner_tasks<false, kCodecMasks[1]>,
    &k_owner_tasks<false, kCodecMasks[2]>,
    &k_owner_tasks<false, kCodecMasks[3]>,
    &k_owner_tasks<false, kCodecMasks[4]>,
    &k_owner_tasks<false, kCodecMasks[5]>,
    &k_owner_tasks<false, kCodecMasks[6]>,
    &k_owner_tasks<false, kCodecMasks[7]>,
    &k_owner_tasks<false, kCodecMasks[8]>,
    &k_owner_tasks<false, kCodecMasks[9]>,
    &k_owner_tasks<false, kCodecMasks[10]>,
};

}  // namespace dev
}  // namespace hm
