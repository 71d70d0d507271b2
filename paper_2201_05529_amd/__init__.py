"""MI355X-native PT-TEBD hot path (arXiv 2201.05529).

The compute path is the HIP library ``libpt_tebd.so`` (C ABI declared in
``include/pt_tebd.h``); ``paper_2201_05529_amd.binding`` marshals arguments
to it.  Importing the package does not load the library; the binding does,
and it raises if the library is missing.
"""
