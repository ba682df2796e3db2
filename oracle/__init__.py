"""FP64 CPU oracle of the monodomain explicit step -- test infrastructure only.

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
package; the GPU library never does.
"""
