"""MI355X (gfx950) brute-force charge-transport Monte Carlo with carrier
repulsion (Xie et al., arXiv:2506.09712, Sec. 2.1 and Algorithm 1), and the
simplified spherical model of Sec. 2.2 (Eq. 7), and the parameterised event
generation of Sec. 3 and Sec. 4.2.

The simulation runs in the HIP kernels of libct.so behind the C ABI of
include/ct.h; this package holds the kernels' sources (csrc/), the in-tree
build (build.py) and the ctypes binding (binding.py).
"""
from .binding import (  # noqa: F401
    CT_DIFFUSION, CT_DRIFT, CT_ELECTRONS, CT_FP32, CT_FP64, CT_OPT_AUTOTUNE, CT_OPT_ONE_SIDED,
    CT_OPT_TIMING,
    CT_REPULSION, CT_SPHERICAL, CtError, EXPORTS, ct_generate, generate, make_gen_params,
    Simulator, ct_bind_workspace, ct_collect, ct_destroy, ct_event_carriers, ct_field,
    ct_init_sensor, ct_philox, ct_seed_events, ct_seed_events_noalloc, ct_set_launch, ct_step,
    ct_workspace_bytes, load,
    make_params, EventDescs, run,
)
