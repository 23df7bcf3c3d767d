// Reduced-precision Gram of a once-rounded Z (placeholder until the MFMA
// bf16/f32 kernels land).
#include "pc_internal.h"

namespace pc {

hipError_t launch_gram_lowprec(const Inst&, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace pc
