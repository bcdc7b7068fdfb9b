// 3D kernels (forward and adjoint): not compiled in this build yet.
#include "fd_kernels.h"

namespace fdw {

bool have_fwd3d(int, int, int) { return false; }
bool launch_fwd3d(const StepArgs&, int, int, int, hipStream_t) { return false; }
bool launch_adj3d(const AdjArgs&, int, int, int, hipStream_t) { return false; }

}  // namespace fdw
