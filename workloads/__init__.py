"""Seeded synthetic input generators shared by the tests, the benchmark and the
smoke check.

This package holds none of the method's arithmetic: it only draws inputs
(slot layouts, memcpy request lists, channel message plans, network
initialisations, request arrival times) and the byte content of memory
pools.  Both the CPU oracle and the GPU library consume what it produces;
neither is imported here.
"""
