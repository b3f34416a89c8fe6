// Instantiations of the per-stage task kernel for stages holding the byte-
// aligned codecs of Sec. 4.1: float64 accumulation, whole codec families
// (kCodecMasks; one translation unit per group, so they compile in parallel).
#include "hm_stream.h"

namespace hm {
namespace dev {

extern const TaskKernel kTasksCodec64Family[3];
const TaskKernel kTasksCodec64Family[3] = {
    &k_owner_tasks<true, kCodecMasks[11]>,
    &k_owner_tasks<true, kCodecMasks[12]>,
    &k_owner_tasks<true, kCodecMasks[13]>,
};

}  // namespace dev
}  // namespace hm
