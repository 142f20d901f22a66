// Mixed-precision (MFMA) beamformer -- placeholder until the MFMA path lands.
#include "dev_common.h"
#include "kernels.h"

namespace fftbf {

bool mix_supported(int, int, int) { return false; }
size_t mix_table_bytes(int, int) { return 0; }
hipError_t launch_mix_tables(void*, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_mix(const MixArgs&, int, int, int64_t, hipStream_t) { return hipErrorNotSupported; }

}  // namespace fftbf
