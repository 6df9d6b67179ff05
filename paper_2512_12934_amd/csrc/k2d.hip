// k2d.hip -- D2Q9 instantiation of the step kernels and their launchers.
#include "launch_impl.h"

template struct lbm::Launcher<2>;
