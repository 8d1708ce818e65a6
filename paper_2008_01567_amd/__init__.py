"""MI355X-native forward-model proximal map of multi-slice fusion (4D cone-beam CT).

The compute path is the HIP library ``libmsf.so`` built from ``csrc/``; the
Python binding in ``paper_2008_01567_amd.msf`` only marshals arguments.
``paper_2008_01567_amd.synth`` generates seeded synthetic inputs.
"""
