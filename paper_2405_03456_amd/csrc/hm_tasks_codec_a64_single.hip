// Instantiations of the per-stage task kernel for stages holding the byte-
// aligned codecs of Sec. 4.1: float64 accumulation, one codec with FP64
// (kCodecMasks; one translation unit per group, so they compile in parallel).
#include "hm_stream.h"

namespace hm {
namespace dev {

extern const TaskKernel kTasksCodec64Single[11];
const TaskKernel kTasksCodec64Single[11] = {
    &k_owner_tasks<true, kCodecMasks[0]>,
    &k_owner_tasks<true, kCodecMasks[1]>,
    &k_owner_tasks<true, kCodecMasks[2]>,
    &k_owner_tasks<true, kCodecMasks[3]>,
    &k_owner_tasks<true, kCodecMasks[4]>,
    &k_owner_tasks<true, kCodecMasks[5]>,
    &k_owner_tasks<true, kCodecMasks[6]>,
    &k_owner_tasks<true, kCodecMasks[7]>,
    &k_owner_tasks<true, kCodecMasks[8]>,
    &k_owner_tasks<true, kCodecMasks[9]>,
    &k_owner_tasks<true, kCodecMasks[10]>,
};

}  // namespace dev
}  // namespace hm
