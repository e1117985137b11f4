#!/bin/bash
# Re-tunes the schedules of the benchmark workloads on the current GPU and
# writes them to the cache file given as $1 (default: this directory's
# <arch>.json). Each workload takes one to a few minutes (15 timed calls per
# candidate: the adjoint work-order candidates differ by about 1%).
set -e
cd "$(dirname "$0")/../.."
export FDMT_TUNE_CACHE=${1:-}
T="python -u -m paper_1411_5373_amd.autotune --write --reps 15"
# Nf=4096, Nt=65536, Nd=2048, 1.2-1.6 GHz: the step's forms
$T --nf 4096 --nt 65536 --nd 2048 --band 1.2 1.6 --in-dtype u8 --acc-dtype f32
$T --nf 4096 --nt 65536 --nd 2048 --band 1.2 1.6 --in-dtype f16 --acc-dtype f32
$T --nf 4096 --nt 65536 --nd 2048 --band 1.2 1.6 --in-dtype f32 --acc-dtype f32
$T --nf 4096 --nt 65536 --nd 2048 --band 1.2 1.6 --in-dtype u8 --acc-dtype i32
$T --nf 4096 --nt 65536 --nd 2048 --band 1.2 1.6 --in-dtype i32 --acc-dtype i32
# ragged beams: 256 beams, Nt log-uniform in [2048, 32768] (the benchmark's
# draw), Nf=1024, Nd=512, timed as one ragged batch; stored under Nt = 32511
$T --nf 1024 --nd 512 --band 1.2 1.6 --in-dtype f32 --acc-dtype f32 --ragged 256 2048 32768 14115376
# Nf=1024, Nt=8192, Nd=1024 and the 0.4-0.8 GHz batch-16 form
$T --nf 1024 --nt 8192 --nd 1024 --band 1.2 1.6 --in-dtype f32 --acc-dtype f32
$T --nf 1024 --nt 16384 --nd 1024 --band 0.4 0.8 --in-dtype f32 --acc-dtype f32
