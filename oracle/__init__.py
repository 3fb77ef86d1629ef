"""CPU oracle of the HEVI step (test infrastructure only).

Imported by the test-suite, the smoke check and the CPU baseline leg of the
benchmark; never by the product path.
"""
