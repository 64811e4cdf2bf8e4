"""CPU oracle for suffix-array read matching -- test infrastructure only.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the product library.
"""
