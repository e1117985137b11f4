"""CPU oracle (test infrastructure only; never imported by the product path)."""
from .fdmt_oracle import (Tables, build_tables, channel_edges, merge_coefficient,
                          initialize, iterate, fdmt, fdmt_batch, fdmt_adjoint, path,
                          brute_point, brute_row, brute_ideal, round_half_up, boxcar, boxcar_candidates, boxcar_search,
                          fdmt_fft, fft_length, shift_vector)
