"""Low-scaling GW hot path (arXiv:2104.09857) on MI355X: HIP kernels behind a
C ABI (include/gw.h, libgw.so) and this thin Python binding.

    from paper_2104_09857_amd import gw
    gw.build_gt / gw.contract_chi / gw.screen_w / gw.contract_sigma / gw.continue_qp
"""
