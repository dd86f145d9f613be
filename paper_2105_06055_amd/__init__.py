"""MI355X-native fast convolution-based peridynamics (FCBM-EC).

The compute path lives in the HIP library ``libpdfcbm.so`` (C ABI declared in
``include/pd_fcbm.h``); ``paper_2105_06055_amd.binding`` marshals arguments to it.
Submodules are imported lazily so that ``workloads`` can be used without the
HIP library.
"""
