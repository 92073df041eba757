"""MI355X-native Vlasov translation with a coalesced ghost domain.

The compute path lives in the HIP library ``libvlasov.so`` (C ABI declared in
``include/vlasov.h``); ``binding`` wraps it with ctypes and ``workloads``
generates seeded synthetic plasma states.  Importing the package loads
nothing; ``binding`` loads the library on first use and fails loudly if it
is missing.
"""
