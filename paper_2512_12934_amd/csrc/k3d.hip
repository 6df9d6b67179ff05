// k3d.hip -- D3Q19 instantiation of the step kernels and their launchers.
#include "launch_impl.h"

template struct lbm::Launcher<3>;
