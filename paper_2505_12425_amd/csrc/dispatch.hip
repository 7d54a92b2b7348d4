// dispatch.hip -- chooses the kernel for one image.
#include "kr_device.h"

namespace kr {

hipError_t launch_resize(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    return launch_generic(OP_RESIZE, c, st, dt, j, e, s);
}

hipError_t launch_warp(int c, kr_dtype st, kr_dtype dt, const ImageJob &j, const Epilogue &e, hipStream_t s)
{
    return launch_generic(OP_WARP, c, st, dt, j, e, s);
}

}  // namespace kr
