"""MI355X-native rank-one lamination of incremental damage potentials.

The compute path lives in the HIP library ``libr1.so`` (C-ABI declared in
``include/r1.h``); ``paper_2211_14318_amd.r1`` is its thin Python binding.
``paper_2211_14318_amd.workloads`` draws the seeded synthetic inputs.
"""
